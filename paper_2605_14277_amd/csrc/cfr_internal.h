// Internal declarations shared by the host runtime (cfr_engine.hip,
// cfr_api.hip) and the kernel launchers (cfr_kernels.hip).  Not part of the
// public ABI.
//
// Device layout.  Every game held by an engine owns, per player, a block of
// consecutive sequence indices (its empty sequence first, then its other
// sequences in level order, then one sentinel) and a block of consecutive
// decision-point indices (in level order, then one sentinel).  All index
// arrays hold these global indices, so one launch can cover any set of
// games: it walks a table of blocks, each naming a game ("slot") and an
// index range, and reads the game's own iteration scalars.  A single game
// is the case of one slot at offset 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace cfr {

// Per-game iteration scalars kept in device memory, so that every kernel
// reads the iteration index and its derived factors at run time and a
// captured graph of one iteration can be replayed unchanged.
struct Scalars {
    double t;      // iterations completed (incremented first thing each iteration)
    double w;      // averaging weight of the current iteration
    double W;      // sum of weights so far
    double dpos;   // DCFR factor for positive regrets, t^a/(t^a+1)
    double dneg;   // DCFR factor for negative regrets, t^b/(t^b+1)
    double alpha, beta, gamma;  // DCFR exponents of this game
    int32_t variant;            // CFR_VANILLA .. CFR_PCFR
    int32_t avg_kind;           // CFR_AVG_*
    int32_t pad[2];
    double out[8];  // evaluation results (BR1, BR2, value)
};

// One block of a payoff product: a run of whole rows of one game.
struct SpmvBlock {
    int32_t row0;   // first row (global sequence index of the row player)
    int32_t nr;     // rows in the block
    int32_t n;      // nonzeros in the block
    int32_t p0;     // row pointer of row0 (offset inside the game's matrix)
    int64_t e0;     // position of the block's first nonzero in the index/value arrays
    int32_t slot;   // game
    int32_t begin;  // 1 on the game's first block: advances the game's scalars
};
static_assert(sizeof(SpmvBlock) == 32, "one scalar load per block");

// A range [lo, hi) of at most one block's worth of decision points or
// sequences of one game.  aux: the game's empty sequence (sequence tables)
// or the value-slot flags (bottom-up tables).
struct RangeBlock {
    int32_t lo, hi, slot, aux;
};

// Per-game entry of the evaluation reductions: value at the empty sequence
// (root = empty sequence, [a, b) = decision points under it) or the final
// stage of a dot product ([a, b) = the game's partial sums).
struct SlotRef {
    int32_t slot, root, a, b;
};

// Device arrays of one player, covering every slot (global indices).
// The shallow levels 0 .. levels-1 of the bottom-up pass of a game
// iterating alone (a lone solver's, or a batch's only active one) in one
// block (k_shallow): each level's values stay in LDS for the level above,
// and only the deepest of them reads its children's values from global
// memory (their value slots).  Levels are taken from the root down while
// all of them together hold at most kShallowMax decision points (one per
// thread: a single block passing several times over a level was measured
// slower than a launch per level), every one on the fast path.
constexpr int kShallowThreads = 1024;
constexpr int kShallowMax = kShallowThreads;
constexpr int kShallowLevels = 8;
struct ShallowPlan {
    int32_t levels = 0;                // 0: not used
    int32_t lo[kShallowLevels + 1] = {};  // global first decision point of each level, and the end
    uint8_t kind[kShallowLevels] = {};    // 1 fast, 2 fast without decision points below
};

// Levels lo .. lo+levels-1 below the shallow ones of a game iterating alone
// (a lone solver's, or a batch's only active one) in one launch (k_fuse),
// from lists of the game's local decision points (base added): each block
// takes whole subtrees below a group of level-lo
// decision points, at most kFuseThreads decision points in all (one per
// thread), every level on the fast path.  Inside a block the levels pass
// their values through vinf, separated by block barriers; the shallowest
// writes its values where the level above reads them (or, as level 0, does
// its top-down step), the deepest reads its children's values as its own
// launch would.  Only small levels are fused
// (the deepest at most kFuseDeepMax decision points): larger ones are bound
// by their bytes, where a launch over the whole level keeps more waves in
// flight.  Blocks of 256 (several per CU) and a deepest level of at most
// 65536 decision points measured best on the medium and large games, against
// blocks of 128, 512 or 1024 and limits of 16384 to 131072.
// A lone game's bottom-up (UP) and top-down (DOWN) launches over one direct
// range: 1 deals each XCD a contiguous eighth of the range (neighbouring
// sequences, which share parents and are read together by the next
// product, stay in one L2), 0 keeps the blocks in order.  Both on measured
// 0.3028 against 0.3100 ms per large-game iteration on one box and within
// noise on another.
#ifndef CFR_SWEEP_XCD_UP
#define CFR_SWEEP_XCD_UP 1
#endif
#ifndef CFR_SWEEP_XCD_DOWN
#define CFR_SWEEP_XCD_DOWN 1
#endif
#ifndef CFR_FUSE_THREADS
#define CFR_FUSE_THREADS 256
#endif
#ifndef CFR_FUSE_DEEP_MAX
#define CFR_FUSE_DEEP_MAX 65536
#endif
constexpr int kFuseThreads = CFR_FUSE_THREADS;
constexpr int kFuseLevels = 4;
constexpr int32_t kFuseDeepMax = CFR_FUSE_DEEP_MAX;  // decision points of any fused level at most
constexpr int64_t kFuseListMax = (int64_t)kFuseLevels * kFuseDeepMax;
struct FusePlan {
    int32_t levels = 0;     // 0: not used
    int32_t lo = 0;         // shallowest fused level
    int32_t base = 0;       // the game's first decision point (the lists are local)
    int32_t blocks = 0;
    int32_t top_slots = 0;  // the shallowest level writes value slots
    int32_t deep_read = 0;  // deepest level: 0 no children, 1 reads slots, 2 reads vinf
};

struct DevPlayer {
    int32_t *inf_first = nullptr;  // [decision points + sentinel] first sequence of each
    int32_t *seq_par = nullptr;    // [sequences] parent sequence of each sequence's decision point
    int32_t *child_ptr = nullptr;  // [sequences] decision points below each sequence:
    int32_t *child_idx = nullptr;  //   child_idx[child_ptr[s] .. child_ptr[s+1])
    void *r = nullptr;             // accumulator type
    void *m = nullptr;             // accumulator type
    void *s = nullptr;             // accumulator type
    void *b = nullptr;             // value type
    void *x = nullptr;             // value type
    void *g = nullptr;             // value type
    void *xbar = nullptr;          // value type
    void *vinf = nullptr;          // [decision points] compute type
    // first-touch order of this player's sequences in the product that
    // gathers them: perm[j] = sequence at permuted position j, pos its
    // inverse (global indices), xp the permuted copy the product reads
    int32_t *perm = nullptr;
    int32_t *pos = nullptr;
    void *xp = nullptr;            // value type
    // values of the decision points below each sequence in slots of four:
    // a decision point whose parent sequence has at most kFastKids of them
    // stores its value at cval[cslot[j]] = 4 * parent + rank (else -1)
    int32_t *cslot = nullptr;      // [decision points]
    uint8_t *ccount = nullptr;     // [sequences] decision points below (<= kFastKids when used)
    void *cval = nullptr;          // [4 * sequences] compute type
    // shallow levels 0 .. top_levels-1 of a lone game in one launch (k_top),
    // one block per root decision point (n_roots of them)
    int32_t top_levels = 0;
    int32_t n_roots = 0;
    int32_t *top_off = nullptr;    // [top_levels*(n_roots+1)]
    int32_t *top_list = nullptr;   // decision points grouped by level, then root
    int top_fast = 0;              // every level in k_top is a fast level
    ShallowPlan shallow;           // shallow levels of a lone game in one block (k_shallow)
    FusePlan fuse;                 // fused levels of a lone game (k_fuse)
    int32_t *fuse_off = nullptr;   // [blocks*(levels+1)] list offsets by block, then level
    int32_t *fuse_list = nullptr;  // decision points of the fused levels by block, then level
};

// Kernel launchers (cfr_kernels.hip).  All enqueue on `st` and return the
// launch status.  Tables and the arrays they index live in device memory.
//
// Payoff product yout = M xin over the blocks of `tab`; with `begin`, the
// first block of each game advances that game's scalars.  items: nonzeros
// per thread of the kernel instance (the block partition must hold at most
// spmv_block_cap(items) nonzeros per block, or one row); vec: 16-byte
// stream loads.  The index and value arrays must be readable three elements
// past the last nonzero.  start/stop (both or neither): events the launch
// sets to the kernel's own start and end times (not to be used under graph
// capture).
hipError_t launch_spmv(int prec, int items, int vec, const SpmvBlock *tab, int32_t n_tab,
                       const int32_t *ptr, const int32_t *idx, const void *val, const void *xin,
                       void *yout, int xcd_remap, int sequential, int begin, Scalars *sc,
                       hipStream_t st, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// ObserveUtility on the decision points of `tab` (one level), fused with the
// variant's post-step and regret matching; kind 0 generic, 1 fast, 2 fast
// without children; root: the level under the empty sequence, whose
// top-down step (with averaging) is done in the same launch.  direct (may be
// null; host memory): one game's whole range [lo, hi) with its slot and aux,
// used instead of the table (blocks of kRangeBlock, no table load).
hipError_t launch_up(int prec, int variant, int kind, int root, const RangeBlock *tab,
                     int32_t n_tab, const RangeBlock *direct, const DevPlayer &p, double usign,
                     const Scalars *sc, hipStream_t st);
// Levels U and U+1 of one game's ObserveUtility in one launch: `upper` is
// level U's range (one game); every decision point of U has at most
// kFastActs actions and at most kPairKids decision points below them, and
// level U+1 is on the fast path (child_kind 1, or 2 with nothing below
// it).  child_reads_slots: level U+1 reads its children's values from
// slots; upper_writes_slots: level U stores its values in slots; root:
// level U is level 0 (its top-down step is done too).
hipError_t launch_up_pair(int prec, int variant, int child_kind, int child_reads_slots,
                          int upper_writes_slots, int root, const RangeBlock &upper,
                          const DevPlayer &p, double usign, const Scalars *sc, hipStream_t st);
// Top-down pass over the sequences of `tab` (one level).
hipError_t launch_down(int prec, const RangeBlock *tab, int32_t n_tab, const DevPlayer &p,
                       int average, const Scalars *sc, hipStream_t st);
// Top-down pass over every level below level 0 in one launch: each sequence
// of `tab` (aux = its game's empty sequence) multiplies the behavioural
// strategies of its at most max_depth (<= kDownAllMaxDepth) ancestors.
// With `fold` (a direct range from one game's empty sequence on) it also
// writes the first-touch copy p.xp[p.pos[i]] = x[i] and averages only the
// sequences from avg_lo on.
hipError_t launch_down_all(int prec, int max_depth, const RangeBlock *tab, int32_t n_tab,
                           const RangeBlock *direct, const DevPlayer &p, int average,
                           const Scalars *sc, hipStream_t st, int fold = 0, int32_t avg_lo = 0);
// ObserveUtility on levels top_levels-1..0, then the top-down pass on levels
// 0..top_levels-1 (with averaging when `average`) of the game in slot 0.
hipError_t launch_top(int prec, int variant, const DevPlayer &p, double usign, int average,
                      const Scalars *sc, hipStream_t st);
// ObserveUtility of the shallow levels p.shallow of a lone game (slot 0),
// deepest first, one block; level 0 also does its top-down step.
// The fused levels of p.fuse (k_fuse), one block per group of subtrees.
hipError_t launch_fuse(int prec, int variant, const DevPlayer &p, double usign,
                       const Scalars *sc, hipStream_t st);
hipError_t launch_shallow(int prec, int variant, const DevPlayer &p, double usign,
                          const Scalars *sc, hipStream_t st);
// xbar = s / W per game (x where W = 0), 1 at each game's empty sequence.
hipError_t launch_normalize(int prec, const RangeBlock *tab, int32_t n_tab, const DevPlayer &p,
                            const Scalars *sc, hipStream_t st);
// One level of the best-response max-sweep (values in vinf).
hipError_t launch_br(int prec, const RangeBlock *tab, int32_t n_tab, const DevPlayer &p,
                     double usign, hipStream_t st);
// Per game: usign*g[root] + sum of vinf over the root decision points,
// into sc[slot].out[out_index].
hipError_t launch_root_value(int prec, const SlotRef *tab, int32_t n_tab, const DevPlayer &p,
                             double usign, Scalars *sc, int out_index, hipStream_t st);
// Per game: sum over its sequences of a[i]*b[i] in double, into
// sc[slot].out[out_index] (partials: one double per entry of `tab`).
hipError_t launch_dot(int prec, const RangeBlock *tab, int32_t n_tab, const void *a,
                      const void *b, double *partials, const SlotRef *fin, int32_t n_fin,
                      Scalars *sc, int out_index, hipStream_t st);
// a[i] += base for i < n (only where a[i] >= 0 for the second form).
hipError_t launch_add_offset(int32_t *a, int64_t n, int32_t base, hipStream_t st);
hipError_t launch_add_offset_nonneg(int32_t *a, int64_t n, int32_t base, hipStream_t st);
// dst[i] = src[perm[i]] over the sequences of `tab` (value type).
hipError_t launch_gather(int prec, const RangeBlock *tab, int32_t n_tab, const int32_t *perm,
                         const void *src, void *dst, hipStream_t st);
// a[i] = map[a[i]] for i < n.
hipError_t launch_remap(int32_t *a, int64_t n, const int32_t *map, hipStream_t st);
// Quad stream of one game's product (rows [row0, row0 + nr) of the global
// row space; element row pointers `ptr` hold game-local offsets into the
// index/value arrays at element base nb).  Count: quads of each row into
// cnt[0 .. nr).  Fill: quads of row r from quad qb + qptr[row0 + r]
// (qptr: game-local quad offsets at the global rows).
hipError_t launch_quad_count(const int32_t *ptr, const int32_t *idx, int64_t nb, int32_t row0,
                             int32_t nr, int32_t *cnt, hipStream_t st);
hipError_t launch_quad_fill(int prec, const int32_t *ptr, const int32_t *idx, const void *val,
                            int64_t nb, int32_t row0, int32_t nr, const int32_t *qptr, int64_t qb,
                            uint32_t *qidx, void *qval, hipStream_t st);

size_t value_bytes(int prec);
size_t accum_bytes(int prec);
size_t compute_bytes(int prec);

// Payoff-product tiling.  The kernel is instantiated for these
// nonzeros-per-thread counts; the runtime picks one per matrix.
#ifndef CFR_SPMV_ITEMS
#define CFR_SPMV_ITEMS 16
#endif
#ifndef CFR_SPMV_NONTEMPORAL
#define CFR_SPMV_NONTEMPORAL 1
#endif
// 1: the FP32 modes stage products in LDS in the value type (float)
#ifndef CFR_SPMV_LDS_VALUE
#define CFR_SPMV_LDS_VALUE 1
#endif
constexpr int kSpmvThreads = 256;
constexpr int kSpmvItemsDefault = CFR_SPMV_ITEMS;
constexpr int kSpmvItemsMax = 16;
constexpr int kSpmvRowCap = 256;  // rows per block at most
static_assert(kSpmvRowCap <= kSpmvThreads, "a block's row pointers are one per thread");
inline bool spmv_items_supported(int items) { return items == 4 || items == 8 || items == 16; }
// Nonzeros one block of the product may hold: the staging area less the up
// to three elements the 16-byte stream loads start before the block.
__host__ __device__ constexpr int spmv_block_cap(int items) { return kSpmvThreads * items - 3; }
constexpr int kStreamPad = 4;  // readable elements past the end of the index/value arrays
// Stream form 3 (quads): element = quad index | presence mask << kQuadMaskShift
constexpr int kQuadMaskShift = 28;
constexpr uint32_t kQuadIndexMask = (1u << kQuadMaskShift) - 1;
// Smallest block capacity (stream elements) of any tiling: quads at 8
// nonzeros per thread (512 a block; stream form 3 takes 8 or 16); element
// tiling caps are larger, and a block never holds more elements than
// nonzeros, so partitions at this cap bound the blocks of every tiling.
constexpr int kQuadItemsMin = 8;
constexpr int kMinBlockCap = kSpmvThreads * kQuadItemsMin / 4;
constexpr int kVecPad = 4;      // readable entries past the end of every gathered vector
// Index limits of the device layout.  A value slot is 4 * sequence + rank in
// an int32, so value slots are used only while a player's whole sequence
// index space (every game of the engine) stays at or below 2^29; a quad word
// keeps a column's aligned group of four in kQuadMaskShift bits, so stream
// form 3 needs the column player's index space at or below 2^30.
constexpr int64_t kSlotSeqLimit = (int64_t)1 << 29;
constexpr int64_t kQuadColLimit = (int64_t)1 << (kQuadMaskShift + 2);
inline bool slots_fit(int64_t seq_space) { return seq_space <= kSlotSeqLimit; }
inline bool quads_fit(int64_t col_space) { return col_space <= kQuadColLimit; }
constexpr int64_t kQuadStoreMin = (int64_t)1 << 26;  // first quad store of a batch (quads)
// A game's block of sequence indices (n_seq + 1 with the sentinel) is
// rounded up to a multiple of four, so every game starts at a multiple of
// four and its local aligned groups of four columns are global ones.
__host__ __device__ constexpr int64_t seq_block(int64_t n_seq) { return (n_seq + 1 + 3) & ~(int64_t)3; }
// Stream elements one block of the product may hold under stream form vec.
__host__ __device__ constexpr int spmv_block_cap_v(int items, int vec)
{
    return vec == 3 ? kSpmvThreads * items / 4 : spmv_block_cap(items);
}
constexpr int kRangeBlock = 256;  // decision points or sequences per sweep block
// 1: run the shallow levels in one launch (k_top) even when deeper levels
// remain as per-level launches
#ifndef CFR_TOP_PARTIAL
#define CFR_TOP_PARTIAL 0
#endif
constexpr int kDownAllMaxDepth = 16;  // longest parent chain of the one-launch top-down pass
// value-slot flags of a bottom-up table entry (RangeBlock::aux)
constexpr int kSlotsWrite = 1;  // the level's decision points store values in parent slots
constexpr int kSlotsRead = 2;   // the level reads its children's values from slots
constexpr int32_t kSlotLevelMax = 262144;  // largest level (per game) that writes slots
constexpr int kPairKids = 16;       // two-level launch: decision points below an upper one
constexpr int32_t kPairLevelMax = 262144;  // largest lower level (per game) of a two-level launch
constexpr int kFastActs = 4;        // fast sweep path: actions per decision point
constexpr int kFastKids = 4;        // fast sweep path: decision points below a sequence
constexpr int kTopThreads = 1024;   // threads of the shallow-level block
constexpr int kTopMaxGroup = 1024;  // decision points per root and level it takes

}  // namespace cfr
