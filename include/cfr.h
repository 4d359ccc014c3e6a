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

/* Top-down pass of NextStrategy.  DEFAULT: below level 0, one launch in
 * which each sequence multiplies the behavioural strategies along its
 * parent chain from the root down (the same products in the same order as
 * the level-by-level pass, so identical results), when no chain is longer
 * than 16; otherwise, and with LEVELS, one launch per level.             */
enum { CFR_DOWN_DEFAULT = 0, CFR_DOWN_LEVELS = 1 };

/* Bottom-up pass of a single solver.  DEFAULT and LEVELS: one launch per
 * level.  PAIRS: two adjacent levels run as one launch wherever the upper
 * level's decision points have at most 4 actions and at most 16 decision
 * points below them and the lower level has at most 4 actions per decision
 * point, 4 decision points below each action and at most 2^18 decision
 * points (the same operations in the same order as two launches, so
 * identical results; it chains more dependent memory rounds than two
 * launches cost, and measured slower on the medium and large games).     */
enum { CFR_UP_DEFAULT = 0, CFR_UP_LEVELS = 1, CFR_UP_PAIRS = 2 };

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
    int down_pass;          /* CFR_DOWN_*                                    */
    int up_pass;            /* CFR_UP_*                                      */
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

/* Validates the game (one tree-form sequential decision process per player
 * and the sequence-form payoff matrix of Section 2.1), lays it out level by
 * level, copies it to the device and sets t = 0, regrets and averages to
 * zero and both current strategies to uniform (regret matching on zero
 * regrets, the arbitrary choice Section 2.1 leaves open).  *out receives the solver; on failure *out is NULL.
 * Errors: CFR_EINVAL (game or options), CFR_ENOMEM (workspace too small or
 * hipMalloc failed), CFR_EDEVICE (HIP error).                               */
int cfr_create(const cfr_game_desc *game, const cfr_options *opt, cfr_solver **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): as
 * cfr_create, but the solver allocates nothing on the device or in
 * page-locked host memory, at creation or later.  Its device state lives
 * in a static array of CFR_STATIC_WORKSPACE_BYTES that the library holds
 * on each GPU it runs on from its first use there until the process ends;
 * every solver made this way on one GPU uses that GPU's array, so at most
 * one lives per GPU at a time (CFR_ESTATE while another does; calls that
 * overlap on one GPU would race on the array, which keeps the last
 * solver's contents: creation initialises everything a solver reads).
 * opt->workspace must be NULL (CFR_EINVAL) and opt->use_graph is ignored
 * (iterations are launched one kernel at a time on opt->stream).  A game
 * whose cfr_workspace_size exceeds the array gets CFR_ENOMEM before any
 * device call.  The solver is used and released with the usual calls
 * (cfr_step, cfr_strategy, cfr_exploitability, cfr_destroy ...) and gives
 * the same results as one made by cfr_create; cfr_tune and
 * cfr_kernel_timing (which create HIP events) and tilings with stream form
 * 3 (whose quad copies are allocated) return CFR_EUNSUPPORTED.           */
#define CFR_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int cfr_create_static(const cfr_game_desc *game, const cfr_options *opt, cfr_solver **out);

/* Enqueues n >= 0 iterations on the solver's stream and returns without
 * waiting.  One iteration is Algorithm 2 (ObserveUtility after the payoff
 * products, then NextStrategy) with the variant's regret update (Algorithms
 * 3-5) and the update schedule of Section 3.5 (alternating: player 1
 * observes A y^t and moves, then player 2 observes -A^T x^{t+1}).  The
 * variant and mode of the first call stay fixed for the life of the
 * solver; a different pair returns CFR_ESTATE.                             */
int cfr_step(cfr_solver *s, int64_t n, int variant, int mode);

/* Copies a sequence-form strategy of `player` (0 or 1) into out[len]
 * (len must equal that player's n_seq), in the caller's numbering, as
 * double: a point of the player's sequence-form polytope (Section 2.1),
 * the current one produced by NextStrategy of Algorithm 2 or the weighted
 * average.  kind is CFR_CURRENT or CFR_AVERAGE.  Waits for the stream.     */
int cfr_strategy(cfr_solver *s, int player, int kind, double *out, int64_t len);

/* Cumulative regrets of `player` (entry 0 is 0), caller's numbering, as
 * double; waits for the stream.                                            */
int cfr_regrets(cfr_solver *s, int player, double *out, int64_t len);

/* Evaluates the CURRENT or AVERAGE profile (xbar, ybar) on the device and
 * writes the first min(len, 5) of:
 *   out[0] exploitability = NashConv / 2
 *   out[1] NashConv = BR1 + BR2
 *   out[2] BR1 = max_x x^T A ybar
 *   out[3] BR2 = max_y -(xbar^T A y)
 *   out[4] value xbar^T A ybar
 * len < 4 is CFR_EINVAL.  Exploitability is the metric of the paper's
 * Experiments section, which does not define it; it is read here as half
 * the NashConv of the profile.  Best responses use the bottom-up pass of
 * Algorithm 2 with the maximum over actions in place of the strategy-
 * weighted sum (best response is named as future work in the paper's
 * conclusions).  Waits for the stream.                                     */
int cfr_exploitability(cfr_solver *s, int kind, double *out, int64_t len);

/* Iterations completed so far (host counter; the device holds its own).   */
int cfr_iteration(cfr_solver *s, int64_t *t);

/* Enables (1) or disables (0) per-kernel timing of every payoff-product
 * launch with a pair of HIP events that the launch itself sets to the
 * kernel's start and end times (hipExtLaunchKernel; the span a profiler's
 * kernel trace reports), and resets the accumulated statistics.  Graph
 * replay is bypassed while enabled.                                        */
int cfr_kernel_timing(cfr_solver *s, int enable);

/* Accumulated launches and total milliseconds of one timed kernel class
 * (0: A y over CSR, 1: A^T x over CSC), plus the algorithmic bytes one
 * launch of that class moves (index and value streams, row pointers, the
 * gathered input vector read once and the output vector written once).
 * Waits for the stream.                                                    */
int cfr_kernel_stats(cfr_solver *s, int kernel, int64_t *launches, double *total_ms,
                     double *bytes_per_launch);

/* Checkpointing.  The state of a solver — iteration counter, averaging
 * weights, and per player the cumulative regrets, predictions, average
 * accumulators and current behavioural and sequence-form strategies — as
 * an opaque byte image: cfr_state_size gives its length, cfr_get_state
 * writes it to a host buffer (waits for the stream), cfr_set_state loads
 * it into a solver created from the same game with the same precision
 * (CFR_EINVAL otherwise; it also fixes the variant and mode recorded in the
 * image).  A restored solver continues exactly as the original would.    */
int cfr_state_size(cfr_solver *s, size_t *bytes);
int cfr_get_state(cfr_solver *s, void *out, size_t len);
int cfr_set_state(cfr_solver *s, const void *in, size_t len);

/* Payoff-product tiling of the A y product (index 0) and of the A^T x
 * product (index 1): nonzeros per thread (4, 8 or 16; a block holds up to
 * 256 times that many less 3), rows per block (64..256), vec (1: the index
 * and value streams are read with 16-byte loads, four elements per lane;
 * 2: the same loads, turned around in LDS so that each gather instruction
 * reads consecutive elements; 0: one 4-byte load per element; 3: quads, a
 * copy of the matrix in which each element is a run of at most four
 * nonzeros of a row whose columns share one aligned group of four, stored
 * as one index and four values and gathered with one 16-byte load (8 or
 * 16 nonzeros per thread: a thread takes items/4 quads); the library
 * allocates this copy itself, on
 * first use, outside any caller workspace, and frees it on destroy) and perm
 * (1: before the product, the
 * gathered strategy is copied into the order in which the rows first use
 * its entries, and the product gathers from that copy, so each row's
 * gathers touch consecutive entries; the index stream is renumbered once
 * when the flag changes) and xcd (the order blocks are launched in, see
 * below).  Rows longer than one block's capacity are summed by a tree in
 * every order; every other row keeps its summation order under every
 * choice (quads add -0.0 at absent positions, which changes no sum).     */
typedef struct cfr_spmv_tiling {
    int items[2];
    int rows[2];
    int vec[2];
    int perm[2];
    int xcd[2]; /* 1: blocks launched so that each XCD takes a contiguous
                   range of them (neighbouring rows share its L2); 0: in
                   table order                                            */
} cfr_spmv_tiling;

/* Reads / sets the solver's tiling (CFR_EINVAL outside the ranges above).  */
int cfr_get_tiling(cfr_solver *s, cfr_spmv_tiling *t);
int cfr_set_tiling(cfr_solver *s, const cfr_spmv_tiling *t);

/* Autotuner: times every supported tiling of each product on this game
 * (reps launches each, HIP events on the solver's stream), keeps the
 * fastest (then times its other block order), and writes it to *chosen
 * (may be NULL).  Overwrites only the
 * products' outputs, which every iteration recomputes first.  Waits for
 * the stream.                                                              */
int cfr_tune(cfr_solver *s, int reps, cfr_spmv_tiling *chosen);

/* Releases the solver (and the workspace it allocated, if any).  NULL is
 * accepted.                                                                */
int cfr_destroy(cfr_solver *s);

/* ---- batches of games ----------------------------------------------------
 * Many independent games solved together (the repeated-game and research
 * use cases of Sections 5 and 6): every launch of an iteration covers all games
 * that are still iterating, and one iteration of the whole batch is one
 * captured HIP graph, so the launch count per iteration does not grow with
 * the number of games.  Each game has its own regret minimiser, iteration
 * counter and stopping rule; no reduction mixes two games, so a game's
 * results do not depend on the other games in the batch.
 *
 * Storage: one device workspace with per-player arenas of sequence and
 * decision-point indices and an arena of payoff nonzeros.  A game takes
 * n_seq + 1 sequence indices rounded up to a multiple of four (so that every
 * game starts at a multiple of four) and n_inf + 1 decision-point indices per
 * player and nnz nonzeros (cfr_batch_game_size); cfr_batch_add fails with
 * CFR_ENOMEM when no free range or slot fits, and cfr_batch_remove returns
 * the ranges.  Checks: every check_every iterations the average strategy
 * of each iterating game is evaluated; a game stops when its
 * exploitability is at most its target or its iteration count has reached
 * its limit.  A game added between two checks starts at the next check, so
 * its iterates and checks are those of the game solved alone with the same
 * check period.                                                           */
typedef struct cfr_batch cfr_batch;

typedef struct cfr_batch_options {
    int precision;             /* CFR_FP64 | CFR_FP32 | CFR_FP32_ACC64           */
    int mode;                  /* CFR_SIMULTANEOUS | CFR_ALTERNATING (all games) */
    int spmv_order;            /* CFR_SPMV_*                                     */
    int64_t max_games;         /* game slots                                     */
    int64_t seq_capacity[2];   /* sequence indices per player                    */
    int64_t inf_capacity[2];   /* decision-point indices per player              */
    int64_t nnz_capacity;      /* payoff nonzeros                                */
    int64_t check_every;       /* iterations between checks (>= 1)              */
    void *stream;              /* hipStream_t; NULL = null stream                */
    int device;                /* HIP device ordinal                             */
    int use_graph;             /* 1: replay a captured graph per iteration       */
    int down_pass;             /* CFR_DOWN_*                                     */
    int async_admission;       /* 1: cfr_batch_add_prepared only enqueues its
                                  copies (on a stream of its own) and returns;
                                  the prepared game must then stay alive until
                                  the game has run or been removed.  A game
                                  added while others iterate joins at the
                                  next check, so its copies overlap one check
                                  period of the others.                     */
    int64_t quad_capacity;     /* quads per product of the store that stream
                                  form 3 uses, allocated at creation outside
                                  the workspace (quad_capacity * (4 + 4 value
                                  bytes) per product, plus a row pointer per
                                  sequence index); 0: allocated when that form
                                  is first used (min(2^26, nnz_capacity)) and
                                  grown by doubling, each growth waiting for
                                  the streams and copying the store.        */
} cfr_batch_options;

typedef struct cfr_game_params {
    int variant;                    /* CFR_VANILLA .. CFR_PCFR                  */
    int avg_weight;                 /* CFR_AVG_*                                */
    double dcfr_alpha, dcfr_beta, dcfr_gamma;
    double target_exploitability;   /* stop at a check with expl <= this (0: never) */
    int64_t max_iterations;         /* stop at a check at or beyond this (0: never) */
} cfr_game_params;

enum { CFR_GAME_ACTIVE = 0, CFR_GAME_WAITING = 1, CFR_GAME_DONE = 2 };

typedef struct cfr_game_status {
    int state;             /* CFR_GAME_*                                        */
    int reached_target;    /* 1 if it stopped on its exploitability target      */
    int64_t iterations;    /* iterations completed                              */
    int64_t evaluated_at;  /* iteration of the last evaluation (-1: none)       */
    double exploitability; /* average-strategy exploitability at that evaluation */
} cfr_game_status;

/* Defaults: FP32_ACC64, alternating, 256 slots, capacities 0 (must be
 * set), check every 10 iterations, null stream, device 0, graphs on; game
 * parameters: PCFR+, default averaging, DCFR 1.5/0/2, no target, no limit. */
int cfr_batch_options_default(cfr_batch_options *opt);
int cfr_game_params_default(cfr_game_params *gp);

/* Index units a game takes in a batch: out[0..1] sequence indices of each
 * player, out[2..3] decision-point indices, out[4] nonzeros.  Host only.  */
int cfr_batch_game_size(const cfr_game_desc *game, int64_t *out);

/* Device bytes of a batch with these capacities.                         */
int cfr_batch_workspace_size(const cfr_batch_options *opt, size_t *bytes);

/* Index limits of a batch with these capacities (host only; no device).
 * Value slots (a decision point's value stored beside its parent sequence,
 * one dependent load fewer per sweep level) hold 4 * sequence + rank in an
 * int32, so they are used only while a player's sequence capacity is at
 * most 2^29; above it every level keeps its values in the plain per
 * decision point array (same results).  A quad word (stream form 3) keeps a
 * column's aligned group of four in 28 bits, so that form is refused
 * (CFR_EINVAL from the tiling calls; skipped by the autotuner) while the
 * column player's sequence capacity exceeds 2^30.  The same limits apply
 * to a single solver, whose capacity is its game's sequence count plus
 * one, rounded up to a multiple of four.
 *   out[0], out[1]  1 if value slots are used for player 1 / player 2
 *   out[2], out[3]  1 if stream form 3 is allowed for A y / for A^T x     */
int cfr_batch_index_limits(const cfr_batch_options *opt, int *out);

/* Allocates the batch's workspace (library-owned) on opt->device.        */
int cfr_batch_create(const cfr_batch_options *opt, cfr_batch **out);

/* Validates and adds a game (copied; the caller may free its arrays).
 * *id receives the game's handle.  CFR_ENOMEM: no free slot or range.    */
int cfr_batch_add(cfr_batch *b, const cfr_game_desc *game, const cfr_game_params *gp,
                  int64_t *id);

/* A game validated, laid out in level order and converted to one
 * precision's value type on the host, ready to be added to batches of that
 * precision: cfr_prepare launches no device work and may run on worker
 * threads while a batch iterates (the serving path prepares arriving
 * requests this way, so that admission is only the copy to the device).
 * Its index and value streams are held in page-locked host memory
 * (hipHostMalloc; ordinary memory if that fails), so those copies are DMA
 * transfers that do not hold up the host.  A prepared game owns copies of
 * everything it needs and may be added any number of times.               */
typedef struct cfr_prepared cfr_prepared;
int cfr_prepare(const cfr_game_desc *game, int precision, cfr_prepared **out);
/* Builds, on the host, the quad copies (stream form 3 of the tiling) of
 * both products of a prepared game, product w in column order perm[w] (0:
 * as numbered, 1: first-touch), in page-locked memory (ordinary memory if
 * that fails).  A batch whose product w is in stream form 3 with that
 * column order then copies them at cfr_batch_add_prepared instead of
 * building them on the device when the game joins.  Host only; may run on
 * a worker thread, but not while the same prepared game is being added.
 * Replaces quads built before.  Errors: CFR_EINVAL (null, perm not 0/1),
 * CFR_ENOMEM (host allocation).                                           */
int cfr_prepare_quads(cfr_prepared *p, const int perm[2]);
/* Index units of a prepared game, as cfr_batch_game_size.                 */
int cfr_prepared_size(const cfr_prepared *p, int64_t *out);
/* As cfr_batch_add; CFR_EINVAL if the batch's precision differs.          */
int cfr_batch_add_prepared(cfr_batch *b, const cfr_prepared *p, const cfr_game_params *gp,
                           int64_t *id);
int cfr_prepared_destroy(cfr_prepared *p);

/* Runs up to n iterations of the iterating games with checks every
 * check_every iterations, stopping early when no game is left; waits for
 * the stream at each check.  *n_active (may be NULL) receives the number
 * of games still iterating or waiting to start.                          */
int cfr_batch_run(cfr_batch *b, int64_t n, int64_t *n_active);

/* One check period of cfr_batch_run without waiting, so that the host (or
 * another batch on another stream) works while the device iterates:
 * cfr_batch_run_begin joins the games due to start, enqueues the
 * iterations up to the next check and that check's evaluation on the
 * batch's stream (results copied to page-locked memory) and returns;
 * cfr_batch_run_end waits for them, applies the check exactly as
 * cfr_batch_run does (same iterates, same stopping) and writes the number
 * of games still iterating or waiting to *n_active (may be NULL).  Between
 * the two calls only cfr_batch_status and cfr_batch_run_ready may be
 * called on the batch (other calls return CFR_ESTATE); run_end without a
 * begun period does nothing.
 * CFR_EUNSUPPORTED if the page-locked staging could not be allocated.   */
int cfr_batch_run_begin(cfr_batch *b);
int cfr_batch_run_end(cfr_batch *b, int64_t *n_active);
/* *ready = 1 when no check period is begun or the begun one has completed
 * on the device (cfr_batch_run_end would not wait), else 0.  Does not
 * wait; may be called between run_begin and run_end.                    */
int cfr_batch_run_ready(cfr_batch *b, int *ready);

int cfr_batch_status(cfr_batch *b, int64_t id, cfr_game_status *out);

/* As cfr_strategy / cfr_exploitability for one game of the batch (the
 * evaluation also becomes the game's last evaluation).                    */
int cfr_batch_strategy(cfr_batch *b, int64_t id, int player, int kind, double *out,
                       int64_t len);
int cfr_batch_exploitability(cfr_batch *b, int64_t id, int kind, double *out,
                             int64_t len);

/* Frees a game's slot and ranges.                                         */
int cfr_batch_remove(cfr_batch *b, int64_t id);

/* Tiling of the batch's products, as for a single solver; cfr_batch_tune
 * times the candidates on the games currently iterating.                  */
int cfr_batch_get_tiling(cfr_batch *b, cfr_spmv_tiling *t);
int cfr_batch_set_tiling(cfr_batch *b, const cfr_spmv_tiling *t);
int cfr_batch_tune(cfr_batch *b, int reps, cfr_spmv_tiling *chosen);

/* Total launches and milliseconds of the products of the last
 * cfr_batch_run while timing was enabled, as cfr_kernel_stats.           */
int cfr_batch_kernel_timing(cfr_batch *b, int enable);
int cfr_batch_kernel_stats(cfr_batch *b, int kernel, int64_t *launches, double *total_ms,
                           double *bytes_per_launch);

/* Host seconds and calls spent so far by the batch's runtime: out[0..6]
 * seconds in table builds, graph captures, evaluations (including their
 * wait for the stream), iteration enqueues, game additions, removals and
 * quad-copy work (stream form 3: device builds, part of the table builds,
 * and copies of prepared quads, part of the additions); out[7..13] the
 * matching call counts.  For reports.                                     */
int cfr_batch_host_stats(cfr_batch *b, double *out);

int cfr_batch_destroy(cfr_batch *b);

/* Message of the last failing call on this thread ("" if none).           */
const char *cfr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CFR_H */
