/*
 * CPU FP64 oracle for two-player zero-sum sequence-form CFR.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The GPU product
 * path never calls it, shares no code with it, and must not fall back to it.
 *
 * What it computes, written out plainly in IEEE double, with every sum taken
 * in ascending index order and compiled without floating-point contraction:
 *
 *  - NextStrategy of sequence-form CFR (Algorithm 1): regret matching at
 *    every decision point (Section 2.1: L1-normalised positive regrets; a
 *    decision point whose positive regrets sum to zero plays uniformly,
 *    which is the "arbitrary strategy" the paper allows), then the top-down
 *    conversion x[(j,a)] = x[p_j] * b_j[a] with x[empty] = 1.
 *  - The payoff step of Section 2.1 (the "extra step" done as a sparse
 *    matrix-vector product): player 1 observes u1 = A y and player 2
 *    observes u2 = -A^T x, A being player 1's sequence-form payoff matrix
 *    with chance folded in.  A^T x is formed by scattering over the rows of
 *    A, so every column is summed in ascending row order.
 *  - ObserveUtility (Algorithm 1): bottom-up counterfactual values
 *    v[j] = sum_a b_j[a] * (u[(j,a)] + v[rho(j,a)]), where the value of an
 *    observation point is the sum of its children, then the regret update
 *    r_j += u_j - <b_j, u_j>.
 *  - Variants applied after ObserveUtility: CFR+ floors regrets at zero
 *    (Algorithm 3); DCFR multiplies positive regrets by t^a/(t^a+1) and
 *    negative ones by t^b/(t^b+1) (Algorithm 4); PCFR+ (Algorithm 5, with
 *    the prediction m^t = u^{t-1} of Section 3.5) plays regret matching on
 *    the floored regrets plus the instantaneous regret the prediction
 *    induces.  The PCFR+ prediction is kept as that instantaneous regret;
 *    a second, literal mode runs Algorithm 5's back-up / observe /
 *    next-strategy / restore sequence instead.
 *  - Alternating updates (Section 3.5): the two players' NextStrategy and
 *    ObserveUtility calls are not interleaved: player 1 observes A y^t and
 *    moves to x^{t+1}, then player 2 observes -A^T x^{t+1}.
 *  - Weighted average strategies in sequence form (Section 3.5 names
 *    quadratic weighting for DCFR) and, for evaluation, best responses by a
 *    bottom-up max-sweep (the paper names best response and exploitability
 *    as its metric and as future work for parallelisation; the max-sweep is
 *    the textbook dynamic program), NashConv = BR1 + BR2 and
 *    exploitability = NashConv / 2.
 *
 * Readings where the paper is silent (listed in the design notes): regrets
 * start at zero and t starts at 1; averaging weights are 1 (vanilla), t
 * (CFR+), t^gamma (DCFR) and t^2 (PCFR+) unless overridden; the DCFR factor
 * uses the sign of the regret after this iteration's update, with factor 1
 * at exactly zero; "current strategy" after T iterations is the strategy
 * regret matching gives from the regrets after iteration T.
 *
 * All-core build.  Compiled with -fopenmp, the same arithmetic runs on every
 * host core: each row of A y and each column of A^T x (the oracle then
 * keeps its own transpose of A, built by a counting sort over the rows in
 * ascending order, so every column is still summed in ascending row order
 * from 0.0), the per-decision-point and per-sequence loops, and the sweeps
 * one treeplex level at a time (deepest level first bottom-up, shallowest
 * first top-down; the decision points of one level depend only on deeper or
 * shallower levels).  Every stored value is computed by the same sequence of
 * floating-point operations as in the plain build, so the two builds give
 * bit-identical results (tested).  Without -fopenmp those blocks are not
 * compiled and the plain loops below are the whole oracle.
 *
 * Inputs are borrowed, not copied: the caller keeps the arrays alive for the
 * life of the solver.  Sequence 0 is the empty sequence.  Decision point j
 * owns sequences [first[j], first[j+1]); parent[j] < first[j].
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_VANILLA = 0, ORC_PLUS = 1, ORC_DCFR = 2, ORC_PCFR_PLUS = 3, ORC_PCFR = 4 };
enum { ORC_SIMULTANEOUS = 0, ORC_ALTERNATING = 1 };
enum { ORC_CURRENT = 0, ORC_AVERAGE = 1 };
enum { ORC_AVG_DEFAULT = 0, ORC_AVG_UNIFORM = 1, ORC_AVG_LINEAR = 2,
       ORC_AVG_QUADRATIC = 3, ORC_AVG_POW_GAMMA = 4 };

typedef struct {
    int64_t n_seq, n_inf;
    const int32_t *parent;  /* [n_inf]   parent sequence of decision point j */
    const int32_t *first;   /* [n_inf+1] first sequence of decision point j  */
    int64_t *child_ptr;     /* [n_seq+1] decision points below each sequence */
    int32_t *child;         /* [n_inf]   ascending within each sequence      */
    double *r;      /* cumulative regret, per sequence (entry 0 unused)   */
    double *m;      /* PCFR prediction as instantaneous regret            */
    double *b;      /* behavioural strategy of the current iterate        */
    double *x;      /* sequence-form strategy of the current iterate      */
    double *s;      /* weighted sum of played sequence-form strategies    */
    double *q;      /* last counterfactual utility per sequence           */
    double *v;      /* last value per decision point                      */
    double *vmax;   /* best-response value per decision point             */
    double *u_last; /* last observed utility (literal Algorithm 5 mode)   */
#ifdef _OPENMP
    int64_t n_levels;    /* decision levels (number of own earlier decisions) */
    int64_t *lvl_ptr;    /* [n_levels+1] decision points of level l:          */
    int32_t *lvl_inf;    /*   lvl_inf[lvl_ptr[l] .. lvl_ptr[l+1]), ascending  */
#endif
} orc_tfsdp;

typedef struct {
    orc_tfsdp pl[2];
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
    double *g1;     /* A y       (length n_seq of player 1) */
    double *g2;     /* A^T x     (length n_seq of player 2) */
    double *xb1, *xb2;
#ifdef _OPENMP
    int64_t *col_ptr;  /* [n_seq2+1] transpose of A: column k's nonzeros   */
    int32_t *row_idx;  /* [nnz]      in ascending row order                */
    double *val_t;     /* [nnz]                                            */
#endif
    double alpha, beta, gamma;
    int avg_kind, variant, mode, literal_pcfr, started;
    int64_t t;
    double W;
} orc_solver;

static int tfsdp_init(orc_tfsdp *p, int64_t n_seq, int64_t n_inf,
                      const int32_t *parent, const int32_t *first)
{
    memset(p, 0, sizeof(*p));
    p->n_seq = n_seq;
    p->n_inf = n_inf;
    p->parent = parent;
    p->first = first;
    p->child_ptr = (int64_t *)calloc((size_t)n_seq + 1, sizeof(int64_t));
    p->child = (int32_t *)calloc((size_t)(n_inf > 0 ? n_inf : 1), sizeof(int32_t));
    double **bufs[] = {&p->r, &p->m, &p->b, &p->x, &p->s, &p->q, &p->u_last};
    for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); ++i) {
        *bufs[i] = (double *)calloc((size_t)n_seq, sizeof(double));
        if (!*bufs[i]) return -1;
    }
    p->v = (double *)calloc((size_t)(n_inf > 0 ? n_inf : 1), sizeof(double));
    p->vmax = (double *)calloc((size_t)(n_inf > 0 ? n_inf : 1), sizeof(double));
    if (!p->child_ptr || !p->child || !p->v || !p->vmax) return -1;
    /* child lists: decision points grouped by parent sequence, ascending j */
    for (int64_t j = 0; j < n_inf; ++j) p->child_ptr[parent[j] + 1] += 1;
    for (int64_t s = 0; s < n_seq; ++s) p->child_ptr[s + 1] += p->child_ptr[s];
    int64_t *fill = (int64_t *)malloc(((size_t)n_seq + 1) * sizeof(int64_t));
    if (!fill) return -1;
    memcpy(fill, p->child_ptr, ((size_t)n_seq + 1) * sizeof(int64_t));
    for (int64_t j = 0; j < n_inf; ++j) p->child[fill[parent[j]]++] = (int32_t)j;
    free(fill);
#ifdef _OPENMP
    /* level of each decision point: 0 under the empty sequence, else one
     * more than the level of the decision point owning its parent sequence
     * (which comes earlier, since parent[j] < first[j]) */
    int32_t *lvl = (int32_t *)calloc((size_t)(n_inf > 0 ? n_inf : 1), sizeof(int32_t));
    int32_t *owner = (int32_t *)calloc((size_t)n_seq, sizeof(int32_t));
    if (!lvl || !owner) return -1;
    p->n_levels = 0;
    for (int64_t j = 0; j < n_inf; ++j) {
        for (int64_t a = first[j]; a < first[j + 1]; ++a) owner[a] = (int32_t)j;
        lvl[j] = parent[j] == 0 ? 0 : lvl[owner[parent[j]]] + 1;
        if (lvl[j] + 1 > p->n_levels) p->n_levels = lvl[j] + 1;
    }
    p->lvl_ptr = (int64_t *)calloc((size_t)p->n_levels + 1, sizeof(int64_t));
    p->lvl_inf = (int32_t *)calloc((size_t)(n_inf > 0 ? n_inf : 1), sizeof(int32_t));
    if (!p->lvl_ptr || !p->lvl_inf) return -1;
    for (int64_t j = 0; j < n_inf; ++j) p->lvl_ptr[lvl[j] + 1] += 1;
    for (int64_t l = 0; l < p->n_levels; ++l) p->lvl_ptr[l + 1] += p->lvl_ptr[l];
    int64_t *at = (int64_t *)malloc(((size_t)p->n_levels + 1) * sizeof(int64_t));
    if (!at) return -1;
    memcpy(at, p->lvl_ptr, ((size_t)p->n_levels + 1) * sizeof(int64_t));
    for (int64_t j = 0; j < n_inf; ++j) p->lvl_inf[at[lvl[j]]++] = (int32_t)j;
    free(at);
    free(lvl);
    free(owner);
#endif
    return 0;
}

static void tfsdp_free(orc_tfsdp *p)
{
    free(p->child_ptr); free(p->child); free(p->r); free(p->m); free(p->b);
    free(p->x); free(p->s); free(p->q); free(p->v); free(p->vmax); free(p->u_last);
#ifdef _OPENMP
    free(p->lvl_ptr); free(p->lvl_inf);
#endif
}

/* Regret matching at every decision point (Algorithm 1, behavioural step):
 * b_j = (r_j + m_j)^+ / ||(r_j + m_j)^+||_1, uniform when the norm is 0.  */
static void regret_matching(orc_tfsdp *p)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p->n_inf; ++j) {
        int64_t a0 = p->first[j], a1 = p->first[j + 1];
        double Z = 0.0;
        for (int64_t a = a0; a < a1; ++a) {
            double z = p->r[a] + p->m[a];
            Z = Z + (z > 0.0 ? z : 0.0);
        }
        for (int64_t a = a0; a < a1; ++a) {
            if (Z > 0.0) {
                double z = p->r[a] + p->m[a];
                p->b[a] = (z > 0.0 ? z : 0.0) / Z;
            } else {
                p->b[a] = 1.0 / (double)(a1 - a0);
            }
        }
    }
}

/* Top-down conversion to sequence form (Algorithm 1): decision points in
 * ascending index order are a top-down order because parent[j] < first[j]. */
static void sequence_form(orc_tfsdp *p)
{
    p->x[0] = 1.0;
#ifdef _OPENMP
    for (int64_t l = 0; l < p->n_levels; ++l) {
#pragma omp parallel for schedule(static)
        for (int64_t i = p->lvl_ptr[l]; i < p->lvl_ptr[l + 1]; ++i) {
            int64_t j = p->lvl_inf[i];
            double xp = p->x[p->parent[j]];
            for (int64_t a = p->first[j]; a < p->first[j + 1]; ++a) p->x[a] = xp * p->b[a];
        }
    }
#else
    for (int64_t j = 0; j < p->n_inf; ++j) {
        double xp = p->x[p->parent[j]];
        for (int64_t a = p->first[j]; a < p->first[j + 1]; ++a) p->x[a] = xp * p->b[a];
    }
#endif
}

/* g1 = A y, each row summed left to right. */
static void payoff_rows(const orc_solver *o, const double *y, double *g1)
{
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < o->pl[0].n_seq; ++i) {
        double acc = 0.0;
        for (int64_t e = o->row_ptr[i]; e < o->row_ptr[i + 1]; ++e)
            acc = acc + o->val[e] * y[o->col[e]];
        g1[i] = acc;
    }
}

/* g2 = A^T x, scattered over rows in ascending order. */
static void payoff_cols(const orc_solver *o, const double *x, double *g2)
{
#ifdef _OPENMP
    /* the same additions per column, from the transpose */
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t k = 0; k < o->pl[1].n_seq; ++k) {
        double acc = 0.0;
        for (int64_t e = o->col_ptr[k]; e < o->col_ptr[k + 1]; ++e)
            acc = acc + o->val_t[e] * x[o->row_idx[e]];
        g2[k] = acc;
    }
    return;
#endif
    for (int64_t k = 0; k < o->pl[1].n_seq; ++k) g2[k] = 0.0;
    for (int64_t i = 0; i < o->pl[0].n_seq; ++i) {
        double xi = x[i];
        for (int64_t e = o->row_ptr[i]; e < o->row_ptr[i + 1]; ++e)
            g2[o->col[e]] = g2[o->col[e]] + o->val[e] * xi;
    }
}

/* Counterfactual utility of sequence a: its own utility plus the values of
 * the decision points directly below it (an observation point's value is
 * the sum over its children; an end contributes nothing). */
static double cf_utility(const orc_tfsdp *p, const double *u, double sign,
                         int64_t a, const double *vals)
{
    double acc = sign * u[a];
    for (int64_t c = p->child_ptr[a]; c < p->child_ptr[a + 1]; ++c)
        acc = acc + vals[p->child[c]];
    return acc;
}

/* ObserveUtility (Algorithm 1) plus the variant's post-step.  With
 * keep_prediction the predictive variants store the instantaneous regret as
 * the next prediction; the literal Algorithm 5 mode re-derives it instead. */
static void observe_one(orc_tfsdp *p, int64_t j, const double *u, double sign, int variant,
                        double dpos, double dneg, int keep_prediction)
{
    int64_t a0 = p->first[j], a1 = p->first[j + 1];
    for (int64_t a = a0; a < a1; ++a) p->q[a] = cf_utility(p, u, sign, a, p->v);
    double V = 0.0;
    for (int64_t a = a0; a < a1; ++a) V = V + p->b[a] * p->q[a];
    p->v[j] = V;
    for (int64_t a = a0; a < a1; ++a) {
        double inst = p->q[a] - V;
        double r = p->r[a] + inst;
        switch (variant) {
        case ORC_PLUS:
            r = r > 0.0 ? r : 0.0;
            break;
        case ORC_DCFR:
            if (r > 0.0) r = r * dpos;
            else if (r < 0.0) r = r * dneg;
            break;
        case ORC_PCFR_PLUS:
            r = r > 0.0 ? r : 0.0;
            if (keep_prediction) p->m[a] = inst;
            break;
        case ORC_PCFR:
            if (keep_prediction) p->m[a] = inst;
            break;
        default:
            break;
        }
        p->r[a] = r;
    }
}

static void observe(orc_tfsdp *p, const double *u, double sign, int variant,
                    double dpos, double dneg, int keep_prediction)
{
#ifdef _OPENMP
    for (int64_t l = p->n_levels - 1; l >= 0; --l) {
#pragma omp parallel for schedule(static)
        for (int64_t i = p->lvl_ptr[l]; i < p->lvl_ptr[l + 1]; ++i)
            observe_one(p, p->lvl_inf[i], u, sign, variant, dpos, dneg, keep_prediction);
    }
#else
    for (int64_t j = p->n_inf - 1; j >= 0; --j)
        observe_one(p, j, u, sign, variant, dpos, dneg, keep_prediction);
#endif
}

static void accumulate_average(orc_tfsdp *p, double w)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < p->n_seq; ++s) p->s[s] = p->s[s] + w * p->x[s];
}

/* Algorithm 5 taken literally: back up r, keep b^{t-1}, observe the
 * prediction (the last utility) with plain ObserveUtility, run
 * NextStrategy, restore r. */
static void next_strategy_literal_predictive(orc_tfsdp *p, double sign)
{
    double *backup = (double *)malloc((size_t)p->n_seq * sizeof(double));
    memcpy(backup, p->r, (size_t)p->n_seq * sizeof(double));
    observe(p, p->u_last, sign, ORC_VANILLA, 1.0, 1.0, 0);
    regret_matching(p);
    sequence_form(p);
    memcpy(p->r, backup, (size_t)p->n_seq * sizeof(double));
    free(backup);
}

static void next_strategy(orc_solver *o, int player, double sign)
{
    orc_tfsdp *p = &o->pl[player];
    int predictive = o->variant == ORC_PCFR_PLUS || o->variant == ORC_PCFR;
    if (predictive && o->literal_pcfr) {
        next_strategy_literal_predictive(p, sign);
    } else {
        regret_matching(p);
        sequence_form(p);
    }
}

static double avg_weight(const orc_solver *o, double t)
{
    int kind = o->avg_kind;
    if (kind == ORC_AVG_DEFAULT) {
        switch (o->variant) {
        case ORC_PLUS: kind = ORC_AVG_LINEAR; break;
        case ORC_DCFR: kind = ORC_AVG_POW_GAMMA; break;
        case ORC_PCFR_PLUS: kind = ORC_AVG_QUADRATIC; break;
        default: kind = ORC_AVG_UNIFORM; break;
        }
    }
    switch (kind) {
    case ORC_AVG_LINEAR: return t;
    case ORC_AVG_QUADRATIC: return t * t;
    case ORC_AVG_POW_GAMMA: return pow(t, o->gamma);
    default: return 1.0;
    }
}

void orc_destroy(void *h);

/* Threads the loops above run on (1 in the plain build). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void *orc_create(int64_t n_seq1, int64_t n_inf1, const int32_t *par1, const int32_t *first1,
                 int64_t n_seq2, int64_t n_inf2, const int32_t *par2, const int32_t *first2,
                 int64_t nnz, const int64_t *row_ptr, const int32_t *col, const double *val,
                 double alpha, double beta, double gamma, int avg_kind, int literal_pcfr)
{
    orc_solver *o = (orc_solver *)calloc(1, sizeof(orc_solver));
    if (!o) return NULL;
    if (tfsdp_init(&o->pl[0], n_seq1, n_inf1, par1, first1) ||
        tfsdp_init(&o->pl[1], n_seq2, n_inf2, par2, first2)) {
        free(o);
        return NULL;
    }
    o->nnz = nnz;
    o->row_ptr = row_ptr;
    o->col = col;
    o->val = val;
    o->g1 = (double *)calloc((size_t)n_seq1, sizeof(double));
    o->g2 = (double *)calloc((size_t)n_seq2, sizeof(double));
    o->xb1 = (double *)calloc((size_t)n_seq1, sizeof(double));
    o->xb2 = (double *)calloc((size_t)n_seq2, sizeof(double));
#ifdef _OPENMP
    o->col_ptr = (int64_t *)calloc((size_t)n_seq2 + 1, sizeof(int64_t));
    o->row_idx = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    o->val_t = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    int64_t *at = (int64_t *)malloc(((size_t)n_seq2 + 1) * sizeof(int64_t));
    if (!o->col_ptr || !o->row_idx || !o->val_t || !at) {
        free(at);
        orc_destroy(o);
        return NULL;
    }
    for (int64_t e = 0; e < nnz; ++e) o->col_ptr[col[e] + 1] += 1;
    for (int64_t k = 0; k < n_seq2; ++k) o->col_ptr[k + 1] += o->col_ptr[k];
    memcpy(at, o->col_ptr, ((size_t)n_seq2 + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n_seq1; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t d = at[col[e]]++;
            o->row_idx[d] = (int32_t)i;
            o->val_t[d] = val[e];
        }
    free(at);
#endif
    o->alpha = alpha;
    o->beta = beta;
    o->gamma = gamma;
    o->avg_kind = avg_kind;
    o->literal_pcfr = literal_pcfr;
    /* t = 0: zero regrets, zero prediction -> uniform first strategies */
    for (int p = 0; p < 2; ++p) {
        regret_matching(&o->pl[p]);
        sequence_form(&o->pl[p]);
    }
    return o;
}

void orc_destroy(void *h)
{
    orc_solver *o = (orc_solver *)h;
    if (!o) return;
    tfsdp_free(&o->pl[0]);
    tfsdp_free(&o->pl[1]);
    free(o->g1); free(o->g2); free(o->xb1); free(o->xb2);
#ifdef _OPENMP
    free(o->col_ptr); free(o->row_idx); free(o->val_t);
#endif
    free(o);
}

int orc_step(void *h, int64_t n, int variant, int mode)
{
    orc_solver *o = (orc_solver *)h;
    if (!o || n < 0 || variant < 0 || variant > 4 || mode < 0 || mode > 1) return -1;
    if (o->started && (variant != o->variant || mode != o->mode)) return -2;
    o->variant = variant;
    o->mode = mode;
    o->started = 1;
    orc_tfsdp *P1 = &o->pl[0], *P2 = &o->pl[1];
    for (int64_t it = 0; it < n; ++it) {
        o->t += 1;
        double t = (double)o->t;
        double w = avg_weight(o, t);
        double ta = pow(t, o->alpha), tb = pow(t, o->beta);
        double dpos = ta / (ta + 1.0), dneg = tb / (tb + 1.0);
        if (mode == ORC_SIMULTANEOUS) {
            payoff_rows(o, P2->x, o->g1);
            payoff_cols(o, P1->x, o->g2);
            observe(P1, o->g1, 1.0, variant, dpos, dneg, !o->literal_pcfr);
            observe(P2, o->g2, -1.0, variant, dpos, dneg, !o->literal_pcfr);
            memcpy(P1->u_last, o->g1, (size_t)P1->n_seq * sizeof(double));
            memcpy(P2->u_last, o->g2, (size_t)P2->n_seq * sizeof(double));
            accumulate_average(P1, w);
            accumulate_average(P2, w);
            next_strategy(o, 0, 1.0);
            next_strategy(o, 1, -1.0);
        } else {
            payoff_rows(o, P2->x, o->g1);
            observe(P1, o->g1, 1.0, variant, dpos, dneg, !o->literal_pcfr);
            memcpy(P1->u_last, o->g1, (size_t)P1->n_seq * sizeof(double));
            accumulate_average(P1, w);
            next_strategy(o, 0, 1.0);
            payoff_cols(o, P1->x, o->g2);
            observe(P2, o->g2, -1.0, variant, dpos, dneg, !o->literal_pcfr);
            memcpy(P2->u_last, o->g2, (size_t)P2->n_seq * sizeof(double));
            accumulate_average(P2, w);
            next_strategy(o, 1, -1.0);
        }
        o->W = o->W + w;
    }
    return 0;
}

int64_t orc_iteration(void *h) { return ((orc_solver *)h)->t; }

double orc_total_weight(void *h) { return ((orc_solver *)h)->W; }

static void profile(orc_solver *o, int player, int kind, double *out)
{
    orc_tfsdp *p = &o->pl[player];
    if (kind == ORC_AVERAGE && o->W > 0.0) {
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < p->n_seq; ++s) out[s] = p->s[s] / o->W;
    } else {
        memcpy(out, p->x, (size_t)p->n_seq * sizeof(double));
    }
}

int orc_strategy(void *h, int player, int kind, double *out)
{
    orc_solver *o = (orc_solver *)h;
    if (!o || player < 0 || player > 1) return -1;
    profile(o, player, kind, out);
    return 0;
}

int orc_behavioral(void *h, int player, double *out)
{
    orc_solver *o = (orc_solver *)h;
    if (!o || player < 0 || player > 1) return -1;
    memcpy(out, o->pl[player].b, (size_t)o->pl[player].n_seq * sizeof(double));
    return 0;
}

int orc_regrets(void *h, int player, double *out)
{
    orc_solver *o = (orc_solver *)h;
    if (!o || player < 0 || player > 1) return -1;
    memcpy(out, o->pl[player].r, (size_t)o->pl[player].n_seq * sizeof(double));
    return 0;
}

int orc_prediction(void *h, int player, double *out)
{
    orc_solver *o = (orc_solver *)h;
    if (!o || player < 0 || player > 1) return -1;
    memcpy(out, o->pl[player].m, (size_t)o->pl[player].n_seq * sizeof(double));
    return 0;
}

/* Last counterfactual utilities q (per sequence) and decision-point values
 * v (per decision point) computed by ObserveUtility. */
int orc_last_observation(void *h, int player, double *q, double *v)
{
    orc_solver *o = (orc_solver *)h;
    if (!o || player < 0 || player > 1) return -1;
    orc_tfsdp *p = &o->pl[player];
    if (q) memcpy(q, p->q, (size_t)p->n_seq * sizeof(double));
    if (v) memcpy(v, p->v, (size_t)p->n_inf * sizeof(double));
    return 0;
}

/* Best-response value of a player facing the utility sign*u: bottom-up
 * max over actions of (own utility + values below), then the value at the
 * empty sequence. */
static void best_response_one(orc_tfsdp *p, int64_t j, const double *u, double sign)
{
    double best = 0.0;
    for (int64_t a = p->first[j]; a < p->first[j + 1]; ++a) {
        double val = cf_utility(p, u, sign, a, p->vmax);
        if (a == p->first[j] || val > best) best = val;
    }
    p->vmax[j] = best;
}

static double best_response(orc_tfsdp *p, const double *u, double sign)
{
#ifdef _OPENMP
    for (int64_t l = p->n_levels - 1; l >= 0; --l) {
#pragma omp parallel for schedule(static)
        for (int64_t i = p->lvl_ptr[l]; i < p->lvl_ptr[l + 1]; ++i)
            best_response_one(p, p->lvl_inf[i], u, sign);
    }
#else
    for (int64_t j = p->n_inf - 1; j >= 0; --j) best_response_one(p, j, u, sign);
#endif
    return cf_utility(p, u, sign, 0, p->vmax);
}

/* out[0] exploitability = NashConv/2, out[1] NashConv = BR1 + BR2,
 * out[2] BR1 = max_x x^T A ybar, out[3] BR2 = max_y -(xbar^T A y),
 * out[4] value xbar^T A ybar. */
int orc_exploitability(void *h, int kind, double *out)
{
    orc_solver *o = (orc_solver *)h;
    if (!o) return -1;
    profile(o, 0, kind, o->xb1);
    profile(o, 1, kind, o->xb2);
    payoff_rows(o, o->xb2, o->g1);
    payoff_cols(o, o->xb1, o->g2);
    double br1 = best_response(&o->pl[0], o->g1, 1.0);
    double br2 = best_response(&o->pl[1], o->g2, -1.0);
    double value = 0.0;
    for (int64_t s = 0; s < o->pl[0].n_seq; ++s) value = value + o->xb1[s] * o->g1[s];
    out[0] = (br1 + br2) / 2.0;
    out[1] = br1 + br2;
    out[2] = br1;
    out[3] = br2;
    out[4] = value;
    return 0;
}

/* Best-response value against an arbitrary opponent sequence-form strategy
 * (used by tests): player 0 maximises x^T A y_opp, player 1 maximises
 * -(x_opp^T A y). */
double orc_best_response_to(void *h, int player, const double *opp)
{
    orc_solver *o = (orc_solver *)h;
    if (player == 0) {
        payoff_rows(o, opp, o->g1);
        return best_response(&o->pl[0], o->g1, 1.0);
    }
    payoff_cols(o, opp, o->g2);
    return best_response(&o->pl[1], o->g2, -1.0);
}
