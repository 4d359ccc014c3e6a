// Host runtime and C ABI of libcfr (declared in include/cfr.h).
//
// cfr_create validates the game on the host, renumbers each treeplex into
// level order, lays out one device workspace, copies the game once and puts
// both players at the uniform strategy.  cfr_step then only enqueues
// kernels (or replays a captured graph of one iteration) on the caller's
// stream; the only host/device crossings are the copies in cfr_strategy,
// cfr_regrets and cfr_exploitability, which wait for the stream.
//
// Level order (internal numbering).  The level of a decision point is the
// number of its own earlier decisions: 0 under the empty sequence, else one
// more than the level of its parent sequence's decision point.  Decision
// points are numbered level by level, keeping the caller's order inside a
// level; each one's sequences follow consecutively.  The sequences of one
// level then form one contiguous range, so each level of a sweep is one
// launch over a range (Algorithm 2 applies one level graph per step).  The
// decision points below each sequence (the children of the observation
// point that follows it in Algorithm 1) are listed in child_ptr/child_idx,
// ascending.  When the caller's numbering is already level-major (the
// generator emits it), no permutation happens and the payoff arrays are
// used as given.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "cfr.h"
#include "cfr_internal.h"

using cfr::DevMatrix;
using cfr::DevPlayer;
using cfr::Scalars;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

std::string hip_msg(const char *what, hipError_t e)
{
    return std::string(what) + ": " + hipGetErrorString(e);
}

// ---------------------------------------------------------------------------
// Host validation
// ---------------------------------------------------------------------------

int validate_player(const cfr_player_desc &p, int who)
{
    char buf[256];
    const int64_t kMax = std::numeric_limits<int32_t>::max();
    if (p.n_seq < 1 || p.n_seq > kMax) {
        snprintf(buf, sizeof buf, "player %d: n_seq=%lld out of range [1, INT32_MAX]", who + 1,
                 (long long)p.n_seq);
        return fail(CFR_EINVAL, buf);
    }
    if (p.n_inf < 0 || p.n_inf > p.n_seq - 1) {
        snprintf(buf, sizeof buf, "player %d: n_inf=%lld out of range", who + 1, (long long)p.n_inf);
        return fail(CFR_EINVAL, buf);
    }
    if (p.n_inf == 0) {
        if (p.n_seq != 1)
            return fail(CFR_EINVAL, "player " + std::to_string(who + 1) +
                                        ": sequences without decision points");
        return CFR_OK;
    }
    if (!p.inf_parent || !p.inf_first_seq)
        return fail(CFR_EINVAL, "player " + std::to_string(who + 1) + ": null treeplex array");
    if (p.inf_first_seq[0] != 1 || p.inf_first_seq[p.n_inf] != p.n_seq)
        return fail(CFR_EINVAL, "player " + std::to_string(who + 1) +
                                    ": inf_first_seq must start at 1 and end at n_seq");
    for (int64_t j = 0; j < p.n_inf; ++j) {
        if (p.inf_first_seq[j + 1] <= p.inf_first_seq[j]) {
            snprintf(buf, sizeof buf, "player %d: decision point %lld has no action", who + 1,
                     (long long)j);
            return fail(CFR_EINVAL, buf);
        }
        int32_t par = p.inf_parent[j];
        if (par < 0 || par >= p.inf_first_seq[j]) {
            snprintf(buf, sizeof buf,
                     "player %d: decision point %lld has parent %d (must be in [0, %d))", who + 1,
                     (long long)j, par, p.inf_first_seq[j]);
            return fail(CFR_EINVAL, buf);
        }
    }
    return CFR_OK;
}

int validate_rows(const char *name, int64_t n_rows, int64_t n_cols, int64_t nnz,
                  const int64_t *ptr, const int32_t *idx, const double *val)
{
    char buf[256];
    if (!ptr || (nnz > 0 && (!idx || !val))) return fail(CFR_EINVAL, std::string(name) + ": null array");
    if (ptr[0] != 0 || ptr[n_rows] != nnz)
        return fail(CFR_EINVAL, std::string(name) + ": pointers must start at 0 and end at nnz");
    for (int64_t i = 0; i < n_rows; ++i) {
        if (ptr[i + 1] < ptr[i]) {
            snprintf(buf, sizeof buf, "%s: pointer of row %lld decreases", name, (long long)i);
            return fail(CFR_EINVAL, buf);
        }
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            if (idx[e] < 0 || idx[e] >= n_cols) {
                snprintf(buf, sizeof buf, "%s: index %d out of range in row %lld", name, idx[e],
                         (long long)i);
                return fail(CFR_EINVAL, buf);
            }
            if (e > ptr[i] && idx[e] <= idx[e - 1]) {
                snprintf(buf, sizeof buf, "%s: indices not strictly increasing in row %lld", name,
                         (long long)i);
                return fail(CFR_EINVAL, buf);
            }
            if (!std::isfinite(val[e])) {
                snprintf(buf, sizeof buf, "%s: non-finite value in row %lld", name, (long long)i);
                return fail(CFR_EINVAL, buf);
            }
        }
    }
    return CFR_OK;
}

// CSR -> CSR of the transpose, every output row in ascending input-row order.
void transpose(int64_t n_rows, int64_t n_cols, const int64_t *ptr, const int32_t *idx,
               const double *val, std::vector<int64_t> &tptr, std::vector<int32_t> &tidx,
               std::vector<double> &tval)
{
    int64_t nnz = ptr[n_rows];
    tptr.assign((size_t)n_cols + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) tptr[(size_t)idx[e] + 1]++;
    for (int64_t c = 0; c < n_cols; ++c) tptr[c + 1] += tptr[c];
    tidx.resize((size_t)nnz);
    tval.resize((size_t)nnz);
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t i = 0; i < n_rows; ++i)
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            int64_t pos = fill[idx[e]]++;
            tidx[pos] = (int32_t)i;
            tval[pos] = val[e];
        }
}

int validate_game(const cfr_game_desc *g, bool check_csc)
{
    if (!g) return fail(CFR_EINVAL, "null game");
    for (int p = 0; p < 2; ++p) {
        int rc = validate_player(g->player[p], p);
        if (rc) return rc;
    }
    if (g->nnz < 0 || g->nnz > std::numeric_limits<int32_t>::max())
        return fail(CFR_EINVAL, "nnz out of range [0, INT32_MAX]");
    int rc = validate_rows("csr", g->player[0].n_seq, g->player[1].n_seq, g->nnz, g->row_ptr,
                           g->col_idx, g->val);
    if (rc) return rc;
    bool any_csc = g->col_ptr || g->row_idx || g->val_csc;
    if (any_csc && !(g->col_ptr && (g->nnz == 0 || (g->row_idx && g->val_csc))))
        return fail(CFR_EINVAL, "csc: give all three arrays or none");
    if (any_csc && check_csc) {
        std::vector<int64_t> tp;
        std::vector<int32_t> ti;
        std::vector<double> tv;
        transpose(g->player[0].n_seq, g->player[1].n_seq, g->row_ptr, g->col_idx, g->val, tp, ti,
                  tv);
        int64_t n2 = g->player[1].n_seq;
        if (std::memcmp(tp.data(), g->col_ptr, sizeof(int64_t) * (size_t)(n2 + 1)) != 0 ||
            (g->nnz > 0 &&
             (std::memcmp(ti.data(), g->row_idx, sizeof(int32_t) * (size_t)g->nnz) != 0 ||
              std::memcmp(tv.data(), g->val_csc, sizeof(double) * (size_t)g->nnz) != 0)))
            return fail(CFR_EINVAL, "csc is not the exact transpose of the csr");
    }
    return CFR_OK;
}

// ---------------------------------------------------------------------------
// Level-order plan of one treeplex
// ---------------------------------------------------------------------------

struct PlayerPlan {
    int32_t n_seq = 1, n_inf = 0, n_levels = 0;
    bool identity = true;
    std::vector<int32_t> new_of_old;  // caller sequence -> internal sequence
    std::vector<int32_t> old_of_new;  // internal sequence -> caller sequence
    std::vector<int32_t> inf_first;   // [n_inf+1]
    std::vector<int32_t> seq_par;     // [n_seq]
    std::vector<int32_t> child_ptr;   // [n_seq+1]
    std::vector<int32_t> child_idx;   // [n_inf]
    std::vector<int32_t> lvl_inf;     // [n_levels+1]
    std::vector<int32_t> lvl_seq;     // [n_levels+1]
    std::vector<uint8_t> lvl_kind;    // [n_levels]
    int32_t top_levels = 0, n_roots = 0;
    std::vector<int32_t> top_off;     // [top_levels*(n_roots+1)]
    std::vector<int32_t> top_list;    // decision points of the shallow levels by level, then root
};

void plan_player(const cfr_player_desc &d, PlayerPlan &pl)
{
    const int32_t n_seq = (int32_t)d.n_seq, n_inf = (int32_t)d.n_inf;
    pl.n_seq = n_seq;
    pl.n_inf = n_inf;
    std::vector<int32_t> seq_inf((size_t)n_seq, -1);
    for (int32_t j = 0; j < n_inf; ++j)
        for (int32_t a = d.inf_first_seq[j]; a < d.inf_first_seq[j + 1]; ++a) seq_inf[a] = j;
    std::vector<int32_t> level((size_t)n_inf, 0);
    int32_t n_levels = 0;
    for (int32_t j = 0; j < n_inf; ++j) {
        int32_t par = d.inf_parent[j];
        level[j] = par == 0 ? 0 : level[seq_inf[par]] + 1;
        n_levels = std::max(n_levels, level[j] + 1);
    }
    pl.n_levels = n_levels;
    // stable bucket by level
    std::vector<int32_t> count((size_t)n_levels + 1, 0);
    for (int32_t j = 0; j < n_inf; ++j) count[level[j] + 1]++;
    for (int32_t lv = 0; lv < n_levels; ++lv) count[lv + 1] += count[lv];
    std::vector<int32_t> old_inf_of_new((size_t)n_inf);
    {
        std::vector<int32_t> fill(count.begin(), count.end() - 1);
        for (int32_t j = 0; j < n_inf; ++j) old_inf_of_new[fill[level[j]]++] = j;
    }
    pl.new_of_old.assign((size_t)n_seq, 0);
    pl.old_of_new.assign((size_t)n_seq, 0);
    pl.inf_first.assign((size_t)n_inf + 1, n_seq);
    pl.lvl_inf.assign((size_t)n_levels + 1, n_inf);
    pl.lvl_seq.assign((size_t)n_levels + 1, n_seq);
    int32_t next = 1;
    for (int32_t k = 0; k < n_inf; ++k) {
        int32_t j = old_inf_of_new[k];
        if (k == count[level[j]]) {
            pl.lvl_inf[level[j]] = k;
            pl.lvl_seq[level[j]] = next;
        }
        pl.inf_first[k] = next;
        for (int32_t a = d.inf_first_seq[j]; a < d.inf_first_seq[j + 1]; ++a) {
            pl.new_of_old[a] = next;
            pl.old_of_new[next] = a;
            ++next;
        }
    }
    pl.identity = true;
    for (int32_t k = 0; k < n_inf; ++k)
        if (old_inf_of_new[k] != k) {
            pl.identity = false;
            break;
        }
    // parent sequence of each decision point / of each sequence, new numbering
    std::vector<int32_t> inf_par((size_t)n_inf);
    pl.seq_par.assign((size_t)n_seq, 0);
    for (int32_t k = 0; k < n_inf; ++k) {
        inf_par[k] = pl.new_of_old[d.inf_parent[old_inf_of_new[k]]];
        for (int32_t a = pl.inf_first[k]; a < pl.inf_first[k + 1]; ++a) pl.seq_par[a] = inf_par[k];
    }
    // decision points below each sequence, ascending
    pl.child_ptr.assign((size_t)n_seq + 1, 0);
    for (int32_t k = 0; k < n_inf; ++k) pl.child_ptr[inf_par[k] + 1]++;
    for (int32_t s = 0; s < n_seq; ++s) pl.child_ptr[s + 1] += pl.child_ptr[s];
    pl.child_idx.assign((size_t)std::max(n_inf, 1), 0);
    {
        std::vector<int32_t> fill(pl.child_ptr.begin(), pl.child_ptr.end() - 1);
        for (int32_t k = 0; k < n_inf; ++k) pl.child_idx[fill[inf_par[k]]++] = k;
    }
    // levels whose decision points fit the fast sweep path (2: and have
    // nothing below them)
    pl.lvl_kind.assign((size_t)n_levels, 2);
    for (int32_t lv = 0; lv < n_levels; ++lv)
        for (int32_t k = pl.lvl_inf[lv]; k < pl.lvl_inf[lv + 1]; ++k) {
            if (pl.inf_first[k + 1] - pl.inf_first[k] > cfr::kFastActs) pl.lvl_kind[lv] = 0;
            for (int32_t a = pl.inf_first[k]; a < pl.inf_first[k + 1]; ++a) {
                const int32_t kids = pl.child_ptr[a + 1] - pl.child_ptr[a];
                if (kids > cfr::kFastKids) pl.lvl_kind[lv] = 0;
                else if (kids > 0 && pl.lvl_kind[lv] == 2) pl.lvl_kind[lv] = 1;
            }
        }
    // One launch per root subtree for the whole sweep, when every root
    // decision point's share of every level is at most kTopMaxGroup decision
    // points (one pass of the block).  The levels of one sweep form a chain
    // of dependent memory accesses either way, so this only pays when it
    // removes every per-level launch; otherwise each level gets a launch
    // over all its decision points.
    pl.top_levels = 0;
    pl.n_roots = n_levels > 0 ? pl.lvl_inf[1] - pl.lvl_inf[0] : 0;
    pl.top_off.clear();
    pl.top_list.clear();
    if (n_levels == 0) return;
    std::vector<int32_t> root((size_t)n_inf, 0);
    std::vector<int32_t> seq_new_inf((size_t)n_seq, 0);
    for (int32_t k = 0; k < n_inf; ++k)
        for (int32_t a = pl.inf_first[k]; a < pl.inf_first[k + 1]; ++a) seq_new_inf[a] = k;
    for (int32_t k = 0; k < n_inf; ++k)
        root[k] = inf_par[k] == 0 ? k : root[seq_new_inf[inf_par[k]]];
    const int32_t R = pl.n_roots;
    std::vector<int32_t> cnt((size_t)R + 1);
    for (int32_t lv = 0; lv < n_levels; ++lv) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int32_t k = pl.lvl_inf[lv]; k < pl.lvl_inf[lv + 1]; ++k) cnt[root[k] + 1]++;
        int32_t mx = *std::max_element(cnt.begin(), cnt.end());
        if (mx > cfr::kTopMaxGroup) break;
        for (int32_t r = 0; r < R; ++r) cnt[r + 1] += cnt[r];
        const int32_t base = (int32_t)pl.top_list.size();
        for (int32_t r = 0; r <= R; ++r) pl.top_off.push_back(base + cnt[r]);
        pl.top_list.resize((size_t)base + (size_t)cnt[R]);
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
        for (int32_t k = pl.lvl_inf[lv]; k < pl.lvl_inf[lv + 1]; ++k)
            pl.top_list[(size_t)base + (size_t)fill[root[k]]++] = k;
        pl.top_levels = lv + 1;
    }
    if (pl.top_levels < n_levels && !CFR_TOP_PARTIAL) {
        pl.top_levels = 0;
        pl.top_off.clear();
        pl.top_list.clear();
    }
}

// Rows of `n_rows` length given by `len(i)` grouped into product blocks.
template <typename Len>
std::vector<int32_t> partition_rows(int32_t n_rows, Len len)
{
    std::vector<int32_t> blk{0};
    int64_t cur_nnz = 0;
    int32_t cur_rows = 0;
    for (int32_t r = 0; r < n_rows; ++r) {
        int64_t l = len(r);
        if (l > cfr::kSpmvCap) {
            if (cur_rows) blk.push_back(r);
            blk.push_back(r + 1);
            cur_nnz = 0;
            cur_rows = 0;
            continue;
        }
        if (cur_rows && (cur_nnz + l > cfr::kSpmvCap || cur_rows == cfr::kSpmvRowCap)) {
            blk.push_back(r);
            cur_nnz = 0;
            cur_rows = 0;
        }
        cur_nnz += l;
        ++cur_rows;
    }
    if (cur_rows) blk.push_back(n_rows);
    return blk;
}

// Workspace layout: every buffer 256-byte aligned, carved in a fixed order.
struct Carver {
    size_t cur = 0;
    char *base = nullptr;
    void *take(size_t bytes)
    {
        cur = (cur + 255) & ~(size_t)255;
        void *p = base ? base + cur : nullptr;
        cur += bytes;
        return p;
    }
};

struct Sizes {
    int64_t nnz;
    int32_t n_seq[2], n_inf[2], n_blk_csr, n_blk_csc;
    int32_t top_off[2], top_list[2];
};

struct Buffers {
    Scalars *sc;
    double *partials;
    DevPlayer dp[2];
    int32_t *csr_ptr, *csr_idx, *csr_blk, *csc_ptr, *csc_idx, *csc_blk;
    void *csr_val, *csc_val;
};

Buffers carve(Carver &c, const Sizes &z, int prec)
{
    const size_t V = cfr::value_bytes(prec), R = cfr::accum_bytes(prec), C = cfr::compute_bytes(prec);
    Buffers b{};
    b.sc = (Scalars *)c.take(sizeof(Scalars));
    b.partials = (double *)c.take(sizeof(double) * cfr::kDotPartials);
    for (int p = 0; p < 2; ++p) {
        DevPlayer &d = b.dp[p];
        size_t n = (size_t)z.n_seq[p], ni = (size_t)z.n_inf[p];
        d.inf_first = (int32_t *)c.take(4 * (ni + 1));
        d.seq_par = (int32_t *)c.take(4 * n);
        d.child_ptr = (int32_t *)c.take(4 * (n + 1));
        d.child_idx = (int32_t *)c.take(4 * (ni > 0 ? ni : 1));
        d.r = c.take(R * n);
        d.m = c.take(R * n);
        d.s = c.take(R * n);
        d.b = c.take(V * n);
        d.x = c.take(V * n);
        d.g = c.take(V * n);
        d.xbar = c.take(V * n);
        d.vinf = c.take(C * (ni > 0 ? ni : 1));
        d.top_off = (int32_t *)c.take(4 * (size_t)std::max(z.top_off[p], 1));
        d.top_list = (int32_t *)c.take(4 * (size_t)std::max(z.top_list[p], 1));
    }
    b.csr_ptr = (int32_t *)c.take(4 * ((size_t)z.n_seq[0] + 1));
    b.csr_idx = (int32_t *)c.take(4 * (size_t)z.nnz);
    b.csr_val = c.take(V * (size_t)z.nnz);
    b.csr_blk = (int32_t *)c.take(8 * ((size_t)z.n_blk_csr + 1));
    b.csc_ptr = (int32_t *)c.take(4 * ((size_t)z.n_seq[1] + 1));
    b.csc_idx = (int32_t *)c.take(4 * (size_t)z.nnz);
    b.csc_val = c.take(V * (size_t)z.nnz);
    b.csc_blk = (int32_t *)c.take(8 * ((size_t)z.n_blk_csc + 1));
    return b;
}

// Column lengths of the caller's CSR.
std::vector<int64_t> column_counts(const cfr_game_desc *g)
{
    std::vector<int64_t> cnt((size_t)g->player[1].n_seq, 0);
    for (int64_t e = 0; e < g->nnz; ++e) cnt[g->col_idx[e]]++;
    return cnt;
}

struct Plan {
    PlayerPlan pl[2];
    std::vector<int32_t> blk_csr, blk_csc;
    Sizes sizes;
};

void make_plan(const cfr_game_desc *g, Plan &P)
{
    for (int p = 0; p < 2; ++p) plan_player(g->player[p], P.pl[p]);
    const PlayerPlan &a = P.pl[0], &b = P.pl[1];
    P.blk_csr = partition_rows(a.n_seq, [&](int32_t r) {
        int32_t o = a.old_of_new[r];
        return g->row_ptr[o + 1] - g->row_ptr[o];
    });
    std::vector<int64_t> cc = column_counts(g);
    P.blk_csc = partition_rows(b.n_seq, [&](int32_t r) { return cc[b.old_of_new[r]]; });

    P.sizes.nnz = g->nnz;
    for (int p = 0; p < 2; ++p) {
        P.sizes.n_seq[p] = P.pl[p].n_seq;
        P.sizes.n_inf[p] = P.pl[p].n_inf;
        P.sizes.top_off[p] = (int32_t)P.pl[p].top_off.size();
        P.sizes.top_list[p] = (int32_t)P.pl[p].top_list.size();
    }
    P.sizes.n_blk_csr = (int32_t)P.blk_csr.size() - 1;
    P.sizes.n_blk_csc = (int32_t)P.blk_csc.size() - 1;
}

int check_options(const cfr_options *o)
{
    if (!o) return fail(CFR_EINVAL, "null options");
    if (o->precision < CFR_FP64 || o->precision > CFR_FP32_ACC64)
        return fail(CFR_EINVAL, "unknown precision");
    if (o->avg_weight < CFR_AVG_DEFAULT || o->avg_weight > CFR_AVG_POW_GAMMA)
        return fail(CFR_EINVAL, "unknown averaging weight");
    if (o->spmv_order < CFR_SPMV_DEFAULT || o->spmv_order > CFR_SPMV_PARALLEL)
        return fail(CFR_EINVAL, "unknown summation order");
    if (!std::isfinite(o->dcfr_alpha) || !std::isfinite(o->dcfr_beta) ||
        !std::isfinite(o->dcfr_gamma))
        return fail(CFR_EINVAL, "DCFR exponents must be finite");
    return CFR_OK;
}

// Restores the caller's current device when a call returns.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// Solver
// ---------------------------------------------------------------------------

struct cfr_solver {
    cfr_options opt{};
    int prec = CFR_FP64;
    hipStream_t st = nullptr;
    hipStream_t cap = nullptr;  // private stream used only to capture graphs
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    Plan plan;
    Buffers buf{};
    DevMatrix csr, csc;
    int64_t t = 0;
    int variant = -1, mode = -1;
    bool failed = false;
    int xcd_remap = 1;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events[2];
    int64_t launches[2] = {0, 0};
    double total_ms[2] = {0, 0};
    double bytes_per_launch[2] = {0, 0};

    int sequential() const
    {
        if (opt.spmv_order == CFR_SPMV_SEQUENTIAL) return 1;
        if (opt.spmv_order == CFR_SPMV_PARALLEL) return 0;
        return prec == CFR_FP64 ? 1 : 0;
    }

    cfr::IterParams iter_params() const
    {
        cfr::IterParams ip;
        ip.variant = variant;
        ip.avg_kind = opt.avg_weight;
        ip.alpha = opt.dcfr_alpha;
        ip.beta = opt.dcfr_beta;
        ip.gamma = opt.dcfr_gamma;
        return ip;
    }

    // Payoff product over the CSR (which = 0) or the CSC (which = 1); with
    // begin set, its first block also advances the iteration scalars.
    hipError_t spmv(int which, const void *xin, void *yout, bool begin, hipStream_t s)
    {
        const DevMatrix &A = which == 0 ? csr : csc;
        Scalars *bsc = begin ? buf.sc : nullptr;
        cfr::IterParams ip = iter_params();
        if (timing && s == st) {
            hipEvent_t a, b;
            hipError_t e = hipEventCreate(&a);
            if (e == hipSuccess) e = hipEventCreate(&b);
            if (e != hipSuccess) return e;
            (void)hipEventRecord(a, s);
            e = cfr::launch_spmv(prec, A, xin, yout, xcd_remap, sequential(), bsc, ip, s);
            (void)hipEventRecord(b, s);
            events[which].emplace_back(a, b);
            launches[which]++;
            return e;
        }
        return cfr::launch_spmv(prec, A, xin, yout, xcd_remap, sequential(), bsc, ip, s);
    }

    // One player's ObserveUtility + NextStrategy: the deep levels one launch
    // each (bottom-up), the shallow levels in one launch (bottom-up, then
    // top-down), then the deep levels again (top-down, with averaging).
    hipError_t sweeps(int p, double usign, hipStream_t s)
    {
        const DevPlayer &d = buf.dp[p];
        hipError_t e;
        if (d.top_levels > 0) {
            // the whole sweep in one launch per root subtree
            for (int lv = d.n_levels - 1; lv >= d.top_levels; --lv)
                if ((e = cfr::launch_up_level(prec, variant, d, lv, usign, d.g, buf.sc, s)) !=
                    hipSuccess)
                    return e;
            if ((e = cfr::launch_top(prec, variant, d, usign, 1, buf.sc, s)) != hipSuccess) return e;
            return down_sweep(p, 1, d.top_levels, s);
        }
        // level 0's launch also does its top-down step
        for (int lv = d.n_levels - 1; lv >= 0; --lv)
            if ((e = cfr::launch_up_level(prec, variant, d, lv, usign, d.g, buf.sc, s)) != hipSuccess)
                return e;
        return down_sweep(p, 1, 1, s);
    }

    hipError_t down_sweep(int p, int average, int from_level, hipStream_t s)
    {
        const DevPlayer &d = buf.dp[p];
        for (int lv = from_level; lv < d.n_levels; ++lv) {
            hipError_t e = cfr::launch_down_level(prec, d, lv, average, buf.sc, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

    // One iteration, enqueued on stream s.
    hipError_t enqueue_iteration(hipStream_t s)
    {
        hipError_t e;
        DevPlayer &P1 = buf.dp[0], &P2 = buf.dp[1];
        if (mode == CFR_SIMULTANEOUS) {
            // both products read the strategies of iteration t before either
            // player moves on
            if ((e = spmv(0, P2.x, P1.g, true, s)) != hipSuccess) return e;
            if ((e = spmv(1, P1.x, P2.g, false, s)) != hipSuccess) return e;
            if ((e = sweeps(0, 1.0, s)) != hipSuccess) return e;
            return sweeps(1, -1.0, s);
        }
        if ((e = spmv(0, P2.x, P1.g, true, s)) != hipSuccess) return e;
        if ((e = sweeps(0, 1.0, s)) != hipSuccess) return e;
        if ((e = spmv(1, P1.x, P2.g, false, s)) != hipSuccess) return e;
        return sweeps(1, -1.0, s);
    }

    hipError_t build_graph()
    {
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t e2 = enqueue_iteration(cap);
        e = hipStreamEndCapture(cap, &graph);
        if (e2 != hipSuccess) return e2;
        if (e != hipSuccess) return e;
        return hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    }

    void release()
    {
        for (int k = 0; k < 2; ++k) {
            for (auto &pr : events[k]) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
            events[k].clear();
        }
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        gexec = nullptr;
        graph = nullptr;
        cap = nullptr;
        if (own_ws && ws) (void)hipFree(ws);
        ws = nullptr;
    }

    int device_error(const char *what, hipError_t e)
    {
        failed = true;
        return fail(CFR_EDEVICE, hip_msg(what, e));
    }

    int sync(const char *what)
    {
        hipError_t e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return device_error(what, e);
        return CFR_OK;
    }
};

namespace {

template <typename T>
hipError_t h2d(void *dst, const T *src, size_t count, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, st);
}

// Converts a double array to the solver's value type into `tmp` and copies it.
hipError_t h2d_values(void *dst, const double *src, size_t count, int prec,
                      std::vector<float> &tmp, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    if (cfr::value_bytes(prec) == 8) return h2d(dst, src, count, st);
    tmp.resize(count);
    for (size_t i = 0; i < count; ++i) tmp[i] = (float)src[i];
    hipError_t e = h2d(dst, tmp.data(), count, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);  // tmp is reused
}

// Builds the internal row-sorted matrix of `rows` in level order.
void permute_rows(int32_t n_rows, const std::vector<int32_t> &old_of_new_row,
                  const std::vector<int32_t> &new_of_old_col, const int64_t *ptr,
                  const int32_t *idx, const double *val, std::vector<int64_t> &optr,
                  std::vector<int32_t> &oidx, std::vector<double> &oval)
{
    optr.assign((size_t)n_rows + 1, 0);
    for (int32_t r = 0; r < n_rows; ++r) {
        int32_t o = old_of_new_row[r];
        optr[r + 1] = optr[r] + (ptr[o + 1] - ptr[o]);
    }
    oidx.resize((size_t)optr[n_rows]);
    oval.resize((size_t)optr[n_rows]);
    std::vector<std::pair<int32_t, double>> row;
    for (int32_t r = 0; r < n_rows; ++r) {
        int32_t o = old_of_new_row[r];
        row.clear();
        for (int64_t e = ptr[o]; e < ptr[o + 1]; ++e) row.emplace_back(new_of_old_col[idx[e]], val[e]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                      return a.first < b.first;
                  });
        int64_t base = optr[r];
        for (size_t k = 0; k < row.size(); ++k) {
            oidx[base + k] = row[k].first;
            oval[base + k] = row[k].second;
        }
    }
}

// (first row, first nonzero) of every row block, interleaved.
std::vector<int32_t> block_extents(const std::vector<int32_t> &blk, const std::vector<int32_t> &ptr)
{
    std::vector<int32_t> out(2 * blk.size());
    for (size_t i = 0; i < blk.size(); ++i) {
        out[2 * i] = blk[i];
        out[2 * i + 1] = ptr[(size_t)blk[i]];
    }
    return out;
}

std::vector<int32_t> narrow_ptr(const int64_t *ptr, size_t n)
{
    std::vector<int32_t> out(n);
    for (size_t i = 0; i < n; ++i) out[i] = (int32_t)ptr[i];
    return out;
}

int create_impl(const cfr_game_desc *g, const cfr_options *o, cfr_solver *s)
{
    s->opt = *o;
    s->prec = o->precision;
    s->st = (hipStream_t)o->stream;
    Plan &P = s->plan;
    make_plan(g, P);
    size_t need = 0;
    {
        Carver c;
        carve(c, P.sizes, s->prec);
        need = c.cur + 256;
    }
    if (o->workspace) {
        if (o->workspace_bytes < need)
            return fail(CFR_ENOMEM, "workspace smaller than cfr_workspace_size");
        s->ws = o->workspace;
        s->ws_bytes = o->workspace_bytes;
        s->own_ws = false;
    } else {
        hipError_t e = hipMalloc(&s->ws, need);
        if (e != hipSuccess) {
            s->ws = nullptr;
            return fail(CFR_ENOMEM, hip_msg("hipMalloc of the workspace", e));
        }
        s->ws_bytes = need;
        s->own_ws = true;
    }
    Carver c;
    c.base = (char *)(((uintptr_t)s->ws + 255) & ~(uintptr_t)255);
    s->buf = carve(c, P.sizes, s->prec);
    Buffers &B = s->buf;
    hipStream_t st = s->st;
    hipError_t e = hipSuccess;
#define CHECK(x)                                              \
    do {                                                      \
        e = (x);                                              \
        if (e != hipSuccess) return s->device_error(#x, e);   \
    } while (0)

    // treeplexes
    for (int p = 0; p < 2; ++p) {
        PlayerPlan &pl = P.pl[p];
        DevPlayer &d = B.dp[p];
        d.n_seq = pl.n_seq;
        d.n_inf = pl.n_inf;
        d.n_levels = pl.n_levels;
        d.lvl_inf = pl.lvl_inf.data();
        d.lvl_seq = pl.lvl_seq.data();
        d.lvl_kind = pl.lvl_kind.data();
        CHECK(h2d(d.inf_first, pl.inf_first.data(), pl.inf_first.size(), st));
        CHECK(h2d(d.seq_par, pl.seq_par.data(), pl.seq_par.size(), st));
        CHECK(h2d(d.child_ptr, pl.child_ptr.data(), pl.child_ptr.size(), st));
        CHECK(h2d(d.child_idx, pl.child_idx.data(), pl.child_idx.size(), st));
        CHECK(h2d(d.top_off, pl.top_off.data(), pl.top_off.size(), st));
        CHECK(h2d(d.top_list, pl.top_list.data(), pl.top_list.size(), st));
        d.top_levels = pl.top_levels;
        d.n_roots = pl.n_roots;
        d.top_fast = 1;
        for (int32_t lv = 0; lv < pl.top_levels; ++lv) d.top_fast &= pl.lvl_kind[lv] != 0;
        size_t R = cfr::accum_bytes(s->prec) * (size_t)pl.n_seq;
        CHECK(hipMemsetAsync(d.r, 0, R, st));
        CHECK(hipMemsetAsync(d.m, 0, R, st));
        CHECK(hipMemsetAsync(d.s, 0, R, st));
    }
    CHECK(hipMemsetAsync(B.sc, 0, sizeof(Scalars), st));

    // payoff matrix, in level order
    const PlayerPlan &p1 = P.pl[0], &p2 = P.pl[1];
    std::vector<int64_t> ptr_buf;
    std::vector<int32_t> idx_buf;
    std::vector<double> val_buf;
    const int64_t *rptr = g->row_ptr;
    const int32_t *ridx = g->col_idx;
    const double *rval = g->val;
    if (!(p1.identity && p2.identity)) {
        permute_rows(p1.n_seq, p1.old_of_new, p2.new_of_old, g->row_ptr, g->col_idx, g->val,
                     ptr_buf, idx_buf, val_buf);
        rptr = ptr_buf.data();
        ridx = idx_buf.data();
        rval = val_buf.data();
    }
    std::vector<float> ftmp;
    std::vector<int32_t> ptr32 = narrow_ptr(rptr, (size_t)p1.n_seq + 1);
    CHECK(h2d(B.csr_ptr, ptr32.data(), ptr32.size(), st));
    CHECK(h2d(B.csr_idx, ridx, (size_t)g->nnz, st));
    CHECK(h2d_values(B.csr_val, rval, (size_t)g->nnz, s->prec, ftmp, st));
    std::vector<int32_t> blk_csr = block_extents(P.blk_csr, ptr32);
    CHECK(h2d(B.csr_blk, blk_csr.data(), blk_csr.size(), st));
    CHECK(hipStreamSynchronize(st));  // host buffers below are rebuilt
    {
        std::vector<int64_t> tptr;
        std::vector<int32_t> tidx;
        std::vector<double> tval;
        const int64_t *cptr;
        const int32_t *cidx;
        const double *cval;
        if (p1.identity && p2.identity && g->col_ptr) {
            cptr = g->col_ptr;  // validated to be the exact transpose
            cidx = g->row_idx;
            cval = g->val_csc;
        } else {
            transpose(p1.n_seq, p2.n_seq, rptr, ridx, rval, tptr, tidx, tval);
            cptr = tptr.data();
            cidx = tidx.data();
            cval = tval.data();
        }
        std::vector<int32_t> cptr32 = narrow_ptr(cptr, (size_t)p2.n_seq + 1);
        CHECK(h2d(B.csc_ptr, cptr32.data(), cptr32.size(), st));
        CHECK(h2d(B.csc_idx, cidx, (size_t)g->nnz, st));
        CHECK(h2d_values(B.csc_val, cval, (size_t)g->nnz, s->prec, ftmp, st));
        std::vector<int32_t> blk_csc = block_extents(P.blk_csc, cptr32);
        CHECK(h2d(B.csc_blk, blk_csc.data(), blk_csc.size(), st));
        CHECK(hipStreamSynchronize(st));
    }
    s->csr = DevMatrix{p1.n_seq, p2.n_seq, g->nnz, P.sizes.n_blk_csr, B.csr_ptr, B.csr_idx,
                       B.csr_val, B.csr_blk};
    s->csc = DevMatrix{p2.n_seq, p1.n_seq, g->nnz, P.sizes.n_blk_csc, B.csc_ptr, B.csc_idx,
                       B.csc_val, B.csc_blk};
    const double V = (double)cfr::value_bytes(s->prec);
    for (int k = 0; k < 2; ++k) {
        const DevMatrix &A = k == 0 ? s->csr : s->csc;
        s->bytes_per_launch[k] = (double)A.nnz * (4.0 + V) + 4.0 * (A.n_rows + 1) +
                                 V * A.n_cols + V * A.n_rows;
    }

    // first strategies: uniform behaviour, then the top-down pass
    for (int p = 0; p < 2; ++p) {
        DevPlayer &d = B.dp[p];
        if (cfr::value_bytes(s->prec) == 8) {
            double one = 1.0;
            CHECK(hipMemcpyAsync(d.x, &one, sizeof one, hipMemcpyHostToDevice, st));
            CHECK(hipStreamSynchronize(st));
        } else {
            float one = 1.0f;
            CHECK(hipMemcpyAsync(d.x, &one, sizeof one, hipMemcpyHostToDevice, st));
            CHECK(hipStreamSynchronize(st));
        }
        CHECK(cfr::launch_uniform_b(s->prec, d, st));
        CHECK(s->down_sweep(p, 0, 0, st));
    }
    CHECK(hipStreamSynchronize(st));
#undef CHECK
    return CFR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

int cfr_options_default(cfr_options *opt)
{
    if (!opt) return fail(CFR_EINVAL, "null options");
    std::memset(opt, 0, sizeof *opt);
    opt->precision = CFR_FP64;
    opt->dcfr_alpha = 1.5;
    opt->dcfr_beta = 0.0;
    opt->dcfr_gamma = 2.0;
    opt->avg_weight = CFR_AVG_DEFAULT;
    opt->use_graph = 1;
    return CFR_OK;
}

int cfr_validate(const cfr_game_desc *game)
{
    try {
        return validate_game(game, true);
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_workspace_size(const cfr_game_desc *game, const cfr_options *opt, size_t *bytes)
{
    if (!bytes) return fail(CFR_EINVAL, "null output");
    try {
        int rc = check_options(opt);
        if (rc) return rc;
        rc = validate_game(game, false);
        if (rc) return rc;
        Plan P;
        make_plan(game, P);
        Carver c;
        carve(c, P.sizes, opt->precision);
        *bytes = c.cur + 256;
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_create(const cfr_game_desc *game, const cfr_options *opt, cfr_solver **out)
{
    if (!out) return fail(CFR_EINVAL, "null output");
    *out = nullptr;
    cfr_solver *s = nullptr;
    try {
        int rc = check_options(opt);
        if (rc) return rc;
        rc = validate_game(game, true);
        if (rc) return rc;
        int n_dev = 0;
        hipError_t e = hipGetDeviceCount(&n_dev);
        if (e != hipSuccess || n_dev <= 0) return fail(CFR_EDEVICE, "no HIP device available");
        if (opt->device < 0 || opt->device >= n_dev) return fail(CFR_EINVAL, "device out of range");
        DeviceGuard guard(opt->device);
        s = new cfr_solver();
        rc = create_impl(game, opt, s);
        if (rc) {
            s->release();
            delete s;
            return rc;
        }
        *out = s;
        return CFR_OK;
    } catch (const std::exception &ex) {
        if (s) {
            s->release();
            delete s;
        }
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_step(cfr_solver *s, int64_t n, int variant, int mode)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (n < 0) return fail(CFR_EINVAL, "negative iteration count");
    if (variant < CFR_VANILLA || variant > CFR_PCFR) return fail(CFR_EINVAL, "unknown variant");
    if (mode != CFR_SIMULTANEOUS && mode != CFR_ALTERNATING) return fail(CFR_EINVAL, "unknown mode");
    if (s->variant >= 0 && (variant != s->variant || mode != s->mode))
        return fail(CFR_ESTATE, "variant and mode are fixed by the first cfr_step");
    if (n == 0) return CFR_OK;
    DeviceGuard guard(s->opt.device);
    s->variant = variant;
    s->mode = mode;
    hipError_t e = hipSuccess;
    if (s->opt.use_graph && !s->timing) {
        if (!s->gexec) {
            e = s->build_graph();
            if (e != hipSuccess) return s->device_error("graph capture of one iteration", e);
        }
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) e = hipGraphLaunch(s->gexec, s->st);
    } else {
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) e = s->enqueue_iteration(s->st);
    }
    if (e != hipSuccess) return s->device_error("iteration launch", e);
    s->t += n;
    return CFR_OK;
}

static int fetch(cfr_solver *s, const void *dev, size_t count, size_t elem, std::vector<char> &host)
{
    host.resize(count * elem);
    if (count == 0) return CFR_OK;
    hipError_t e = hipMemcpyAsync(host.data(), dev, count * elem, hipMemcpyDeviceToHost, s->st);
    if (e != hipSuccess) return s->device_error("device-to-host copy", e);
    return s->sync("device-to-host copy");
}

static double load_elem(const std::vector<char> &h, size_t i, size_t elem)
{
    if (elem == 8) {
        double v;
        std::memcpy(&v, h.data() + i * 8, 8);
        return v;
    }
    float v;
    std::memcpy(&v, h.data() + i * 4, 4);
    return (double)v;
}

int cfr_strategy(cfr_solver *s, int player, int kind, double *out, int64_t len)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (player < 0 || player > 1 || !out) return fail(CFR_EINVAL, "bad player or output");
    if (kind != CFR_CURRENT && kind != CFR_AVERAGE) return fail(CFR_EINVAL, "unknown kind");
    const PlayerPlan &pl = s->plan.pl[player];
    if (len != pl.n_seq) return fail(CFR_EINVAL, "output length must equal n_seq");
    DeviceGuard guard(s->opt.device);
    const DevPlayer &d = s->buf.dp[player];
    std::vector<char> h;
    int rc;
    if (kind == CFR_AVERAGE && s->t > 0) {
        Scalars sc;
        hipError_t e = hipMemcpyAsync(&sc, s->buf.sc, sizeof sc, hipMemcpyDeviceToHost, s->st);
        if (e != hipSuccess) return s->device_error("scalar copy", e);
        size_t el = cfr::accum_bytes(s->prec);
        if ((rc = fetch(s, d.s, (size_t)pl.n_seq, el, h))) return rc;
        for (int32_t i = 0; i < pl.n_seq; ++i)
            out[pl.old_of_new[i]] = i == 0 ? 1.0 : load_elem(h, (size_t)i, el) / sc.W;
        return CFR_OK;
    }
    size_t el = cfr::value_bytes(s->prec);
    if ((rc = fetch(s, d.x, (size_t)pl.n_seq, el, h))) return rc;
    for (int32_t i = 0; i < pl.n_seq; ++i) out[pl.old_of_new[i]] = load_elem(h, (size_t)i, el);
    return CFR_OK;
}

int cfr_regrets(cfr_solver *s, int player, double *out, int64_t len)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (player < 0 || player > 1 || !out) return fail(CFR_EINVAL, "bad player or output");
    const PlayerPlan &pl = s->plan.pl[player];
    if (len != pl.n_seq) return fail(CFR_EINVAL, "output length must equal n_seq");
    DeviceGuard guard(s->opt.device);
    std::vector<char> h;
    size_t el = cfr::accum_bytes(s->prec);
    int rc = fetch(s, s->buf.dp[player].r, (size_t)pl.n_seq, el, h);
    if (rc) return rc;
    for (int32_t i = 0; i < pl.n_seq; ++i)
        out[pl.old_of_new[i]] = i == 0 ? 0.0 : load_elem(h, (size_t)i, el);
    return CFR_OK;
}

int cfr_exploitability(cfr_solver *s, int kind, double *out)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (!out) return fail(CFR_EINVAL, "null output");
    if (kind != CFR_CURRENT && kind != CFR_AVERAGE) return fail(CFR_EINVAL, "unknown kind");
    DeviceGuard guard(s->opt.device);
    hipStream_t st = s->st;
    DevPlayer &P1 = s->buf.dp[0], &P2 = s->buf.dp[1];
    const void *src[2] = {P1.x, P2.x};
    hipError_t e = hipSuccess;
#define CHECK(x)                                                          \
    do {                                                                  \
        e = (x);                                                          \
        if (e != hipSuccess) return s->device_error("exploitability", e); \
    } while (0)
    if (kind == CFR_AVERAGE && s->t > 0) {
        for (int p = 0; p < 2; ++p) {
            CHECK(cfr::launch_normalize(s->prec, s->buf.dp[p], s->buf.sc, st));
            src[p] = s->buf.dp[p].xbar;
        }
    }
    cfr::IterParams ip = s->iter_params();
    CHECK(cfr::launch_spmv(s->prec, s->csr, src[1], P1.g, s->xcd_remap, s->sequential(), nullptr,
                           ip, st));
    CHECK(cfr::launch_spmv(s->prec, s->csc, src[0], P2.g, s->xcd_remap, s->sequential(), nullptr,
                           ip, st));
    for (int p = 0; p < 2; ++p) {
        const DevPlayer &d = s->buf.dp[p];
        double usign = p == 0 ? 1.0 : -1.0;
        for (int lv = d.n_levels - 1; lv >= 0; --lv)
            CHECK(cfr::launch_br_level(s->prec, d, lv, usign, d.g, st));
        CHECK(cfr::launch_root_value(s->prec, d, usign, d.g, &s->buf.sc->out[p], st));
    }
    CHECK(cfr::launch_dot(s->prec, P1.n_seq, src[0], P1.g, s->buf.partials, cfr::kDotPartials,
                          &s->buf.sc->out[2], st));
    double res[3];
    CHECK(hipMemcpyAsync(res, s->buf.sc->out, sizeof res, hipMemcpyDeviceToHost, st));
#undef CHECK
    int rc = s->sync("exploitability");
    if (rc) return rc;
    out[0] = (res[0] + res[1]) / 2.0;
    out[1] = res[0] + res[1];
    out[2] = res[0];
    out[3] = res[1];
    out[4] = res[2];
    return CFR_OK;
}

int cfr_iteration(cfr_solver *s, int64_t *t)
{
    if (!s || !t) return fail(CFR_EINVAL, "null argument");
    *t = s->t;
    return CFR_OK;
}

int cfr_kernel_timing(cfr_solver *s, int enable)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    DeviceGuard guard(s->opt.device);
    int rc = s->sync("kernel timing");
    if (rc) return rc;
    for (int k = 0; k < 2; ++k) {
        for (auto &pr : s->events[k]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        s->events[k].clear();
        s->launches[k] = 0;
        s->total_ms[k] = 0;
    }
    s->timing = enable != 0;
    return CFR_OK;
}

int cfr_kernel_stats(cfr_solver *s, int kernel, int64_t *launches, double *total_ms,
                     double *bytes_per_launch)
{
    if (!s || kernel < 0 || kernel > 1) return fail(CFR_EINVAL, "bad solver or kernel");
    DeviceGuard guard(s->opt.device);
    int rc = s->sync("kernel stats");
    if (rc) return rc;
    for (auto &pr : s->events[kernel]) {
        float ms = 0;
        hipError_t e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess) return s->device_error("event timing", e);
        s->total_ms[kernel] += ms;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    s->events[kernel].clear();
    if (launches) *launches = s->launches[kernel];
    if (total_ms) *total_ms = s->total_ms[kernel];
    if (bytes_per_launch) *bytes_per_launch = s->bytes_per_launch[kernel];
    return CFR_OK;
}

int cfr_destroy(cfr_solver *s)
{
    if (!s) return CFR_OK;
    {
        DeviceGuard guard(s->opt.device);
        (void)hipStreamSynchronize(s->st);
        s->release();
    }
    delete s;
    return CFR_OK;
}

const char *cfr_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
