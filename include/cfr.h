/*
 * cfr.h - C ABI of the MI355X (gfx950) sequence-form CFR library (libcfr.so).
 *
 * One iteration of two-player zero-sum sequence-form counterfactual regret
 * minimisation written as linear algebra (Kim & Sandholm, "Parallelizing
 * Counterfactual Regret Minimization", Algorithm 2 and Section 3):
 *   - the payoff products g1 = A y and g2 = A^T x (the two-player utility
 *     step of Section 2.1, done as sparse matrix-vector products),
 *   - a level-by-level bottom-up sweep over each player's treeplex that turns
 *     sequence utilities into counterfactual values (ObserveUtility),
 *   - the regret update of vanilla CFR, CFR+ (Algorithm 3), DCFR
 *     (Algorithm 4) and the predictive variants (Algorithm 5),
 *   - regret matching at every decision point and a level-by-level top-down
 *     sweep back to sequence form (NextStrategy),
 *   - weighted average strategies and a best-response max-sweep for
 *     exploitability.
 * Everything runs as HIP kernels on one GPU; the host code validates and
 * lays out the input once.
 *
 * Conventions shared by every entry point:
 *   - Pointers inside cfr_game_desc are HOST pointers.  The library copies
 *     what it needs during cfr_create; the caller may free them afterwards.
 *   - Output buffers of cfr_strategy / cfr_regrets / cfr_exploitability are
 *     HOST pointers owned by the caller.
 *   - cfr_options.workspace, when given, is a DEVICE pointer owned by the
 *     caller that must outlive the solver.
 *   - Sequence 0 of each player is the empty sequence.  All vectors indexed
 *     by sequence have n_seq entries in the caller's numbering.
 *   - Every function returns CFR_OK (0) or a negative CFR_E* code; the
 *     message of the last failure on the calling thread is returned by
 *     cfr_last_error().  No C++ exception crosses this boundary.
 *   - Calls on one solver must not overlap (the solver is not thread-safe);
 *     distinct solvers are independent.
 */
#ifndef CFR_H
#define CFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CFR_OK 0
#define CFR_EINVAL (-1)       /* malformed game arrays or arguments          */
#define CFR_ENOMEM (-2)       /* workspace too small or allocation failure   */
#define CFR_EDEVICE (-3)      /* a HIP call or kernel failed                 */
#define CFR_ESTATE (-4)       /* call not valid in the solver's state        */
#define CFR_EUNSUPPORTED (-5) /* option not supported                        */

/* ---- enumerations ------------------------------------------------------ */
/* Arithmetic of the device path.
 *   CFR_FP64:       every stored vector and all arithmetic in double.
 *   CFR_FP32:       payoff values, strategies, utilities, regrets and
 *                   averages in float; final scalar reductions in double.
 *   CFR_FP32_ACC64: payoff values, strategies and utilities in float;
 *                   cumulative regrets, predictions, average accumulators
 *                   and all in-register arithmetic in double.            */
enum { CFR_FP64 = 0, CFR_FP32 = 1, CFR_FP32_ACC64 = 2 };

/* Regret minimiser.
 *   CFR_VANILLA    regret matching on cumulative regrets (Algorithm 1/2);
 *   CFR_PLUS       regrets floored at 0 after each update (Algorithm 3);
 *   CFR_DCFR       positive regrets times t^a/(t^a+1), negative ones times
 *                  t^b/(t^b+1) after each update (Algorithm 4);
 *   CFR_PCFR_PLUS  CFR+ regrets, strategy from regret matching on regrets
 *                  plus the prediction m^t = u^{t-1} (Algorithm 5);
 *   CFR_PCFR       the same without the floor (Algorithm 5, PCFR).       */
enum { CFR_VANILLA = 0, CFR_PLUS = 1, CFR_DCFR = 2, CFR_PCFR_PLUS = 3, CFR_PCFR = 4 };

/* Update schedule (Section 3.5): simultaneous = both players observe the
 * same profile; alternating = player 1 observes A y^t and moves to x^{t+1},
 * then player 2 observes -A^T x^{t+1}.                                    */
enum { CFR_SIMULTANEOUS = 0, CFR_ALTERNATING = 1 };

/* Which profile cfr_strategy / cfr_exploitability read.  CURRENT is the
 * strategy the next iteration plays (regret matching on the regrets after
 * the last completed iteration; uniform before the first one).  AVERAGE is
 * sum_t w_t x^t / sum_t w_t in sequence form (CURRENT before iteration 1). */
enum { CFR_CURRENT = 0, CFR_AVERAGE = 1 };

/* Summation order inside a payoff-product row.  SEQUENTIAL adds a row's
 * products strictly left to right (what a plain loop does; the FP64 path
 * then reproduces a sequential evaluation bit for bit, which matters
 * because regret matching amplifies rounding differences over iterations).
 * PARALLEL lets a group of lanes share a row.  DEFAULT: SEQUENTIAL for
 * CFR_FP64, PARALLEL otherwise.                                            */
enum { CFR_SPMV_DEFAULT = 0, CFR_SPMV_SEQUENTIAL = 1, CFR_SPMV_PARALLEL = 2 };

/* Averaging weight w_t.  DEFAULT: 1 (vanilla, PCFR), t (CFR+), t^gamma
 * (DCFR; the paper's quadratic weighting with gamma = 2), t^2 (PCFR+).   */
enum { CFR_AVG_DEFAULT = 0, CFR_AVG_UNIFORM = 1, CFR_AVG_LINEAR = 2,
       CFR_AVG_QUADRATIC = 3, CFR_AVG_POW_GAMMA = 4 };

/* ---- input description --------------------------------------------------
 * One tree-form sequential decision process per player (Section 2.1):
 *   n_seq          sequences including the empty sequence (index 0), >= 1;
 *   n_inf          decision points, >= 0;
 *   inf_parent     [n_inf]   parent sequence of each decision point;
 *   inf_first_seq  [n_inf+1] decision point j owns the contiguous sequences
 *                  [inf_first_seq[j], inf_first_seq[j+1]); each owns at
 *                  least one; they tile 1..n_seq-1 in order.
 * Observation points are implicit: several decision points may share a
 * parent sequence.  Required order: inf_parent[j] < inf_first_seq[j].     */
typedef struct cfr_player_desc {
    int64_t n_seq;
    int64_t n_inf;
    const int32_t *inf_parent;
    const int32_t *inf_first_seq;
} cfr_player_desc;

/* Player 1's sequence-form payoff matrix A (chance folded in), n_seq[0]
 * rows by n_seq[1] columns: player 1 observes A y, player 2 observes
 * -A^T x.  CSR is required: row_ptr [n_seq0+1] (row_ptr[0] = 0, monotone,
 * row_ptr[n_seq0] = nnz), col_idx [nnz] strictly increasing inside a row,
 * val [nnz] finite.  CSC (col_ptr, row_idx, val_csc) is optional: NULL
 * pointers make the library transpose the CSR; if given it must be exactly
 * the transpose (checked).                                                  */
typedef struct cfr_game_desc {
    cfr_player_desc player[2];
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    const int64_t *col_ptr;
    const int32_t *row_idx;
    const double *val_csc;
} cfr_game_desc;

typedef struct cfr_options {
    int precision;          /* CFR_FP64 | CFR_FP32 | CFR_FP32_ACC64          */
    double dcfr_alpha;      /* DCFR positive-regret exponent (default 1.5)   */
    double dcfr_beta;       /* DCFR negative-regret exponent (default 0)     */
    double dcfr_gamma;      /* DCFR averaging exponent (default 2)           */
    int avg_weight;         /* CFR_AVG_*                                     */
    void *stream;           /* hipStream_t to enqueue on; NULL = null stream */
    int device;             /* HIP device ordinal                            */
    void *workspace;        /* device memory of >= cfr_workspace_size bytes,
                               or NULL to let the library allocate it       */
    size_t workspace_bytes;
    int use_graph;          /* 1: replay a captured HIP graph per iteration  */
    int spmv_order;         /* CFR_SPMV_*                                    */
} cfr_options;

typedef struct cfr_solver cfr_solver;

/* ---- entry points ------------------------------------------------------- */

/* Fills *opt with the defaults above (FP64, DCFR 1.5/0/2, default
 * averaging, null stream, device 0, library-owned workspace, graphs on). */
int cfr_options_default(cfr_options *opt);

/* Host-only structural check of a game (no device needed).  Returns
 * CFR_EINVAL with a message for: n_seq < 1 or > INT32_MAX; nnz < 0 or
 * > INT32_MAX; a decision point with no action; offsets not tiling
 * 1..n_seq-1; a parent out of range or not before its decision point's
 * first sequence; row_ptr not monotone or not ending at nnz; a column index
 * out of range or not strictly increasing in its row; a non-finite value;
 * a CSC that is not the exact transpose of the CSR.                        */
int cfr_validate(const cfr_game_desc *game);

/* Device bytes the solver needs for this game and options (including the
 * 256-byte alignment of every buffer).                                     */
int cfr_workspace_size(const cfr_game_desc *game, const cfr_options *opt, size_t *bytes);

/* Validates the game, lays it out level by level, copies it to the device
 * and sets t = 0, regrets and averages to zero and both current strategies
 * to uniform.  *out receives the solver; on failure *out is NULL.
 * Errors: CFR_EINVAL (game or options), CFR_ENOMEM (workspace too small or
 * hipMalloc failed), CFR_EDEVICE (HIP error).                               */
int cfr_create(const cfr_game_desc *game, const cfr_options *opt, cfr_solver **out);

/* Enqueues n >= 0 iterations on the solver's stream and returns without
 * waiting.  The variant and mode of the first call stay fixed for the life
 * of the solver; a different pair returns CFR_ESTATE.                      */
int cfr_step(cfr_solver *s, int64_t n, int variant, int mode);

/* Copies a sequence-form strategy of `player` (0 or 1) into out[len]
 * (len must equal that player's n_seq), in the caller's numbering, as
 * double.  kind is CFR_CURRENT or CFR_AVERAGE.  Waits for the stream.      */
int cfr_strategy(cfr_solver *s, int player, int kind, double *out, int64_t len);

/* Cumulative regrets of `player` (entry 0 is 0), caller's numbering, as
 * double; waits for the stream.                                            */
int cfr_regrets(cfr_solver *s, int player, double *out, int64_t len);

/* Evaluates the CURRENT or AVERAGE profile (xbar, ybar) on the device:
 *   out[0] exploitability = NashConv / 2
 *   out[1] NashConv = BR1 + BR2
 *   out[2] BR1 = max_x x^T A ybar
 *   out[3] BR2 = max_y -(xbar^T A y)
 *   out[4] value xbar^T A ybar
 * Best responses use a bottom-up max-sweep over each treeplex.  Waits for
 * the stream.  out must hold 5 doubles.                                    */
int cfr_exploitability(cfr_solver *s, int kind, double *out);

/* Iterations completed so far (host counter; the device holds its own).   */
int cfr_iteration(cfr_solver *s, int64_t *t);

/* Enables (1) or disables (0) per-kernel timing with HIP events recorded on
 * the solver's stream around every payoff-product launch, and resets the
 * accumulated statistics.  Graph replay is bypassed while enabled.         */
int cfr_kernel_timing(cfr_solver *s, int enable);

/* Accumulated launches and total milliseconds of one timed kernel class
 * (0: A y over CSR, 1: A^T x over CSC), plus the algorithmic bytes one
 * launch of that class moves (index and value streams, row pointers, the
 * gathered input vector read once and the output vector written once).
 * Waits for the stream.                                                    */
int cfr_kernel_stats(cfr_solver *s, int kernel, int64_t *launches, double *total_ms,
                     double *bytes_per_launch);

/* Releases the solver (and the workspace it allocated, if any).  NULL is
 * accepted.                                                                */
int cfr_destroy(cfr_solver *s);

/* Message of the last failing call on this thread ("" if none).           */
const char *cfr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CFR_H */
