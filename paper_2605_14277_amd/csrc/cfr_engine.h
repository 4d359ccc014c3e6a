// Host runtime shared by the single-game solver and the batch of games
// (cfr_api.hip): level-order planning of a game, the device arenas that
// hold any set of games, the block tables every launch walks, graph capture
// of one iteration and the evaluation pass.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "cfr.h"
#include "cfr_internal.h"

namespace cfr {

// Records the message of a failing call for cfr_last_error; returns code.
int fail(int code, const std::string &msg);
const char *last_error_message();
std::string hip_msg(const char *what, hipError_t e);

// ---------------------------------------------------------------------------
// Level order of one game (local numbering)
// ---------------------------------------------------------------------------
//
// The level of a decision point is the number of its own earlier decisions:
// 0 under the empty sequence, else one more than the level of its parent
// sequence's decision point.  Decision points are numbered level by level,
// keeping the caller's order inside a level; each one's sequences follow
// consecutively.  The sequences of one level then form one contiguous
// range, so each level of a sweep is one launch over ranges (Algorithm 2
// applies one level graph per step).  The decision points below each
// sequence (the children of the observation point that follows it in
// Algorithm 1) are listed in child_ptr/child_idx, ascending.
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
    std::vector<uint8_t> lvl_kind;    // [n_levels] 0 generic, 1 fast, 2 fast without children
    std::vector<uint8_t> lvl_pair;    // [n_levels] 1: levels L-1 and L fit one two-level launch
    int32_t top_levels = 0, n_roots = 0;
    std::vector<int32_t> top_off;     // [top_levels*(n_roots+1)]
    std::vector<int32_t> top_list;    // decision points of the shallow levels by level, then root
    // levels fuse_lo..fuse_hi in one launch (k_fuse) when fuse_hi > fuse_lo:
    // block b takes the decision points fuse_list[fuse_off[b*(D+1)+l] ..
    // fuse_off[b*(D+1)+l+1]) of level fuse_lo + l (D = fuse_hi - fuse_lo + 1),
    // whole subtrees below a set of level-fuse_lo decision points
    int32_t fuse_lo = 0, fuse_hi = -1, fuse_blocks = 0;
    std::vector<int32_t> fuse_off;    // [fuse_blocks*(D+1)]
    std::vector<int32_t> fuse_list;   // decision points of the fused levels by block, then level
};

// CSR -> CSR of the transpose, every output row in ascending input-row order.
void transpose(int64_t n_rows, int64_t n_cols, const int64_t *ptr, const int32_t *idx,
               const double *val, std::vector<int64_t> &tptr, std::vector<int32_t> &tidx,
               std::vector<double> &tval);

// A validated game in level order, ready for upload: both players' plans
// and the payoff matrix sorted by player-1 rows (csr) and by player-2 rows
// (csc), with local indices.  The index/value pointers refer either to the
// owned vectors or, when no renumbering was needed, to the caller's arrays
// (valid for the duration of the call that prepared the game).
struct HostGame {
    PlayerPlan pl[2];
    int64_t nnz = 0;
    std::vector<int32_t> ptr[2];  // [n_seq+1] row pointers of csr (0) and csc (1)
    const int32_t *idx[2] = {nullptr, nullptr};
    const double *val[2] = {nullptr, nullptr};
    std::vector<int32_t> own_idx[2];
    std::vector<double> own_val[2];
};
// lone: also group the shallow levels for the one-launch sweep (k_top).
// with_matrix = false: plans and row pointers only (for sizing).
void prepare_game(const cfr_game_desc *g, bool lone, bool with_matrix, HostGame &hg);

// Everything an engine copies to the device for one game, with the game's
// own (local) indices: per player the treeplex arrays, the value slots, the
// first strategy and the first-touch order; per product the row pointers
// and the index and value streams.  Admission copies it and shifts the
// indices to the game's global positions on the device.  The arrays live in
// one host buffer (page-locked when asked and possible, so the copies are
// DMA transfers that never hold up the host); with `borrow`, the index and
// FP64 value streams are read from the HostGame's arrays instead.
struct GameImage {
    int prec = CFR_FP64;
    int64_t nnz = 0;
    int32_t n_seq[2] = {0, 0}, n_inf[2] = {0, 0};
    struct Player {
        size_t inf_first, seq_par, child_ptr, child_idx, cslot, ccount, b0, x0, perm, pos;
    } pl[2];
    size_t ptr[2] = {0, 0}, idx[2] = {0, 0}, val[2] = {0, 0};
    const int32_t *idx_src[2] = {nullptr, nullptr};  // index streams
    const void *val_src[2] = {nullptr, nullptr};     // value streams in the value type
    size_t bytes = 0;
    bool locked = false;  // the buffer is page-locked
    char *base = nullptr;
    std::shared_ptr<void> pinned;
    std::vector<char> plain;
    // Quad copies of the products (stream form 3) in the game's local
    // numbering, built on the host for one column order per product: row
    // pointers, quad words (local aligned group | mask << kQuadMaskShift)
    // and four values per quad, in a buffer of their own.
    struct Quads {
        bool built[2] = {false, false};
        int perm[2] = {0, 0};  // column order they were built in
        int64_t nq[2] = {0, 0};
        std::vector<int32_t> qptr[2];  // host row pointers (partitioning)
        size_t ptr[2] = {0, 0}, idx[2] = {0, 0}, val[2] = {0, 0};  // offsets in the buffer
        bool locked = false;
        char *base = nullptr;
        std::shared_ptr<void> pinned;
        std::vector<char> plain;
    } quads;
};
void build_image(const HostGame &hg, int prec, bool pinned, bool borrow, GameImage &img);
// Builds img.quads for both products (perm[w]: 0 identity, 1 first-touch
// column order).
void build_image_quads(const HostGame &hg, const int perm[2], bool pinned, GameImage &img);

// Per-game constants of the regret minimiser and the stopping rule.
struct GameParams {
    int variant = -1;  // fixed at the first step for the single-game solver
    int avg_kind = CFR_AVG_DEFAULT;
    double alpha = 1.5, beta = 0.0, gamma = 2.0;
    double target = 0.0;    // stop when the average's exploitability is at most this
    int64_t max_it = 0;     // stop at the first check at or beyond this many iterations
};

// Index space, storage and table capacities of an engine.
struct Capacity {
    int64_t slots = 1;
    int64_t seq[2] = {0, 0};  // sequence indices per player (a game takes n_seq + 1)
    int64_t inf[2] = {0, 0};  // decision-point indices per player (a game takes n_inf + 1)
    int64_t nnz = 0;
    int64_t t_csr = 0, t_csc = 0;               // product blocks
    int64_t t_up[2] = {0, 0}, t_down[2] = {0, 0}, t_seq[2] = {0, 0};  // range blocks
    int64_t t_dall[2] = {0, 0};  // range blocks of the one-launch top-down pass
    int64_t top_off[2] = {0, 0}, top_list[2] = {0, 0};
    int64_t fuse_off[2] = {0, 0}, fuse_list[2] = {0, 0};
};
// Exact capacity of one game alone (the single-game solver).
Capacity lone_capacity(const HostGame &hg, int items_csr, int rows_csr, int items_csc,
                       int rows_csc);
// Table capacities that hold any set of games fitting the index capacities.
void bound_tables(Capacity &c);
// Device bytes of an engine of this capacity (256-byte aligned buffers).
size_t engine_bytes(const Capacity &c, int prec);

// First-fit allocator of index ranges.
struct RangeAlloc {
    int64_t cap = 0;
    std::map<int64_t, int64_t> free_;  // start -> length
    void init(int64_t c);
    int64_t take(int64_t n);  // start of a free range of n, or -1
    void give(int64_t at, int64_t n);
    int64_t largest() const;
};

// Stream form 3 of one product: a derived copy of every game's matrix in
// quads, in memory the engine allocates itself on first use and grows when
// needed.  Each game owns a range of quads, built on the device from its
// element arrays in their current numbering (and dropped when that
// numbering changes or the game leaves).
struct QuadStore {
    int32_t *ptr = nullptr;   // [row player's sequence capacity] game-local quad row pointers
    uint32_t *idx = nullptr;  // [cap] quad index | presence mask << kQuadMaskShift
    void *val = nullptr;      // [4 * cap] value type
    int64_t cap = 0;
    RangeAlloc alloc;
};

// One game held by an engine.
struct Slot {
    bool live = false;     // holds a game
    bool active = false;   // iterates
    bool pending = false;  // admitted between checks; joins at the next one
    int64_t id = -1;
    GameParams gp;
    int64_t t = 0;
    int32_t n_seq[2] = {0, 0}, n_inf[2] = {0, 0}, n_levels[2] = {0, 0};
    int64_t sb[2] = {0, 0}, ib[2] = {0, 0}, nb = 0, nnz = 0;
    std::vector<int32_t> lvl_inf[2], lvl_seq[2];
    std::vector<uint8_t> lvl_kind[2];
    std::vector<uint8_t> lvl_pair[2];
    std::vector<uint8_t> lvl_slots[2];   // per level: kSlotsWrite | kSlotsRead
    // the game's own sweep structures while it iterates alone: levels in
    // k_top (lone solver only), and its fused levels (checked lists, local
    // decision points; fuse_hi < fuse_lo: none)
    int32_t top_levels[2] = {0, 0};
    int32_t fuse_lo[2] = {0, 0}, fuse_hi[2] = {-1, -1}, fuse_blocks[2] = {0, 0};
    std::vector<int32_t> fuse_off[2], fuse_list[2];
    std::vector<int32_t> ptr[2];         // local row pointers of csr / csc (re-partitioning)
    int64_t qb[2] = {-1, -1};            // first quad of the game's stream-form-3 copy (-1: none)
    int64_t nq[2] = {0, 0};              // quads in it
    std::vector<int32_t> qptr[2];        // its local quad row pointers
    std::vector<int32_t> old_of_new[2];  // internal -> caller numbering
    std::vector<SpmvBlock> blocks[2];    // product blocks (global fields)
    double last[5] = {0, 0, 0, 0, 0};    // last evaluation: expl, NashConv, BR1, BR2, value
    // asynchronous admission: host copies the uploads read, and the event
    // that marks their completion on the upload stream
    std::vector<std::vector<char>> staging;
    hipEvent_t up_ev = nullptr;
    bool up_waited = false;
    int64_t join_after = 0;  // a waiting game joins at a check once `checks` reaches this
    int64_t last_t = -1;                 // iteration of that evaluation
    bool reached = false;
};

// Block tables of one set of games, in device memory, plus the host-side
// launch plan over them.
struct Tables {
    SpmvBlock *csr = nullptr, *csc = nullptr;
    RangeBlock *up[2] = {nullptr, nullptr}, *down[2] = {nullptr, nullptr},
               *seq[2] = {nullptr, nullptr}, *dall[2] = {nullptr, nullptr};
    SlotRef *root[2] = {nullptr, nullptr}, *fin = nullptr;
    int32_t n_csr = 0, n_csc = 0, n_seq[2] = {0, 0}, n_root[2] = {0, 0}, n_fin = 0;
    int32_t n_dall[2] = {0, 0};
    int dall_depth[2] = {0, 0};  // levels of the deepest game (its longest parent chain)
    RangeBlock dall_direct[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};  // hi > lo: one game's range
    struct Up {
        int32_t off, n;
        int variant, kind;
        RangeBlock direct;  // hi > lo: the whole launch is this one range of one game
    };
    std::vector<std::vector<Up>> up_l[2];                      // per level: one launch per variant
    std::vector<std::pair<int32_t, int32_t>> up_level[2];      // per level: all of its entries
    std::vector<std::pair<int32_t, int32_t>> down_l[2];        // per level (level 0 unused)
    // host copies of the last upload (kept until the next one: the copies
    // are asynchronous)
    std::vector<SpmvBlock> h_csr, h_csc;
    std::vector<RangeBlock> h_up[2], h_down[2], h_seq[2], h_dall[2];
    std::vector<SlotRef> h_root[2], h_fin;
    double bytes[2] = {0, 0};  // algorithmic bytes of one product launch over these games
    bool valid = false;
};

// Adds the wall time of its scope to a host-time counter.
struct HostTimer {
    double *acc;
    int64_t *cnt;
    double t0;
    HostTimer(double *a, int64_t *c);
    ~HostTimer();
};

struct Engine {
    int prec = CFR_FP64;
    int mode = -1;  // CFR_SIMULTANEOUS / CFR_ALTERNATING, fixed by the first step
    int spmv_order = CFR_SPMV_DEFAULT;
    int items[2] = {kSpmvItemsDefault, kSpmvItemsDefault};
    int rows[2] = {kSpmvRowCap, kSpmvRowCap};
    int vec[2] = {1, 1};  // 16-byte stream loads in the products
    int perm_on[2] = {0, 0};  // the product gathers a first-touch-ordered copy
    int xcd_remap[2] = {1, 1};  // per product: XCD-contiguous block order
    int device = 0;
    bool use_graph = true;
    bool no_alloc = false;  // allocates no device or page-locked memory (cfr_create_static)
    bool lone = false;  // a single game: shallow levels may run as one launch
    int down_pass = CFR_DOWN_DEFAULT;  // top-down pass: one launch, or one per level
    int up_pass = CFR_UP_DEFAULT;      // bottom-up pass of a lone game: per level, or pairs
    hipStream_t st = nullptr;
    hipStream_t cap_st = nullptr;  // private stream used only to capture graphs
    hipStream_t up_st = nullptr;   // admission copies (asynchronous admission)
    bool async_admission = false;  // cfr_batch_add_prepared returns before its copies finish
    Scalars *scal_stage = nullptr;  // page-locked staging of each slot's first scalars
    Capacity cap;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    bool failed = false;

    // device buffers
    Scalars *sc = nullptr;
    double *partials = nullptr;
    DevPlayer dp[2];
    int32_t *ptr[2] = {nullptr, nullptr}, *idx[2] = {nullptr, nullptr};
    void *val[2] = {nullptr, nullptr};
    char *tab_region[2] = {nullptr, nullptr};  // iteration tables, evaluation tables
    size_t tab_bytes = 0;

    RangeAlloc seq_alloc[2], inf_alloc[2], nnz_alloc;
    QuadStore quad[2];
    std::vector<Slot> slots;
    int64_t next_id = 0;
    Tables it, ev;  // tables of the iterating games / of the last evaluated set
    std::vector<int> ev_set;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // runs launched directly since the graph was dropped: the first short
    // run after the set of games changes is not captured
    int direct_runs = 0;
    int64_t check_every = 0;  // 0: no checks (single-game solver)
    int64_t phase = 0;        // iterations since the last check
    int64_t checks = 0;       // checks done so far
    // an asynchronous check period (run_begin .. run_end): the games of the
    // check it enqueued, the page-locked copy of every slot's scalars the
    // check reads back, and the event that marks the copy's completion
    bool pending = false;
    std::vector<int> pending_set;
    Scalars *eval_stage = nullptr;
    hipEvent_t eval_ev = nullptr;

    // host-side time and calls per activity (kHost* below), for reports
    enum {
        kHostTables = 0,
        kHostGraph,
        kHostEval,
        kHostEnqueue,
        kHostAdd,
        kHostRemove,
        kHostQuads,  // quad-copy work (device builds in table builds, prepared copies in adds)
        kHostN
    };
    double host_s[kHostN] = {0, 0, 0, 0, 0, 0, 0};
    int64_t host_n[kHostN] = {0, 0, 0, 0, 0, 0, 0};

    // per-launch timing of the payoff products (HIP events on st)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events[2];
    int64_t launches[2] = {0, 0};
    double total_ms[2] = {0, 0};

    // Carves the device buffers for `c` out of `workspace` (or allocates).
    int init(const Capacity &c, int precision, int dev, hipStream_t stream, void *workspace,
             size_t workspace_bytes);
    int init_arenas(const Capacity &c);  // host-side range allocators and game slots
    void release();
    int device_error(const char *what, hipError_t e);
    int sync(const char *what);

    int sequential() const;
    // Uploads a prepared game into free ranges and puts it at the uniform
    // strategy; *slot_out receives its slot.  CFR_ENOMEM when it does not fit.
    // async: copies on the upload stream without waiting (the game's host
    // arrays must outlive them: a prepared game's do).
    int add(const HostGame &hg, const GameImage &img, const GameParams &gp, bool join_now,
            bool async, int *slot_out);
    void remove(int slot);
    // Makes the stream wait for the admission copies of these games.
    hipError_t wait_uploads(const std::vector<int> &set);
    // Frees the host copies of finished admissions (all of them with wait).
    void reap_uploads(bool wait);
    int set_params(int slot, const GameParams &gp);  // writes the game's constants to the device
    // Re-partitions every game's product blocks for a new tiling.
    void repartition(int which, int items_, int rows_, int vec_);
    // Switches a product to (or back from) gathering the first-touch-ordered
    // copy of its input: remaps every game's index stream in place.
    int set_perm(int which, int on);
    void partition(Slot &s, int which);
    // Builds the quad copies that products in stream form 3 need for the
    // games of `set` (waits for their admission copies and for the stream).
    int ensure_quads(const std::vector<int> &set);
    void drop_quads(Slot &s, int which);
    int grow_quads(int which, int64_t need);
    // Allocates both products' quad stores with room for n quads each (and
    // their row pointers); growth then starts from there.
    int reserve_quads(int64_t n);
    int64_t quad_reserved = 0;  // 0: first store min(kQuadStoreMin, nonzero capacity)

    std::vector<int> active_set() const;
    int build_tables(Tables &T, char *region, const std::vector<int> &set);
    bool tables_in_bounds(const Tables &T) const;
    int rebuild();  // iteration tables of the active games; drops the graph
    void drop_graph();
    // The one-block shallow pass and the fused levels of the game in slot k
    // when it is the only one iterating (k < 0: none); uploads its fused
    // lists on stream s.
    hipError_t single_plans(int k, hipStream_t s);
    int single_slot = -1;  // the game those structures belong to

    // `gathered`: the permuted copy the product reads is already current
    // (written by the top-down pass just before), so no gather launch
    hipError_t spmv(const Tables &T, int which, const void *xin, void *yout, bool begin,
                    hipStream_t s, bool timed, bool gathered = false);
    // With `fold` non-null, a lone game's top-down pass also writes the
    // permuted copy of x (and sets *fold) when it runs as one launch.
    hipError_t sweeps(const Tables &T, int p, double usign, hipStream_t s, bool *fold = nullptr);
    hipError_t enqueue_iteration(hipStream_t s);
    hipError_t build_graph();
    // n iterations of every active game (no checks).
    int iterate(int64_t n);
    // Evaluates the average (or current) profile of the games in `set`;
    // results land in each slot's `last`.
    int evaluate(const std::vector<int> &set, int kind);
    // The two halves of evaluate: the launches and the copy of every slot's
    // scalars to `out` (host memory of slots.size() records) on the stream;
    // then, once that copy has completed, the set's results from `out`.
    int evaluate_launch(const std::vector<int> &set, int kind, Scalars *out);
    void evaluate_collect(const std::vector<int> &set, const Scalars *out);
    // After a check of `set`: games that met their stopping rule stop.
    void apply_check(const std::vector<int> &set);
    // n iterations with checks every check_every iterations; games that meet
    // their stopping rule at a check stop iterating.
    int run(int64_t n);
    // One check period without waiting: run_begin enqueues the iterations up
    // to the next check and that check's evaluation (with its results copied
    // to page-locked memory) and returns; run_end waits for them and applies
    // the check.  Nothing else may change the engine in between.
    int run_begin();
    int run_end();
    // 1 when no check period is begun or the begun one has completed.
    int run_ready();
    // Times `reps` launches of one product with the current tiling (ms each).
    int time_spmv(int which, int reps, double *ms);

    int fetch_vector(int slot, int player, int what, std::vector<double> &out);
};

}  // namespace cfr
