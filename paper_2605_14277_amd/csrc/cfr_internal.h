// Internal declarations shared by the host runtime (cfr_api.hip) and the
// kernel launchers (cfr_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace cfr {

// Per-iteration scalars kept in device memory, so that every kernel reads
// the iteration index and its derived factors at run time and a captured
// graph of one iteration can be replayed unchanged.
struct Scalars {
    double t;      // iterations completed (incremented first thing each iteration)
    double w;      // averaging weight of the current iteration
    double W;      // sum of weights so far
    double dpos;   // DCFR factor for positive regrets, t^a/(t^a+1)
    double dneg;   // DCFR factor for negative regrets, t^b/(t^b+1)
    double pad[3];
    double out[8]; // scalar results of the evaluation kernels
};

// Constants of the iteration that the first product launch uses to advance
// the device-side scalars.
struct IterParams {
    int variant = 0;
    int avg_kind = 0;
    double alpha = 1.5, beta = 0.0, gamma = 2.0;
};

// Payoff matrix sorted along one player's sequences: CSR of A (player 1
// rows) or CSR of A^T (player 2 rows), with the row-block partition the
// product kernel walks.
struct DevMatrix {
    int32_t n_rows = 0;
    int32_t n_cols = 0;
    int64_t nnz = 0;
    int32_t n_blk = 0;
    const int32_t *ptr = nullptr;  // [n_rows+1]
    const int32_t *idx = nullptr;  // [nnz]
    const void *val = nullptr;     // [nnz] value type
    const int32_t *blk = nullptr;  // [2*(n_blk+1)] (first row, first nonzero) of each block
};

// One player's treeplex in level order (see the runtime for the layout).
struct DevPlayer {
    int32_t n_seq = 0;
    int32_t n_inf = 0;
    int32_t n_levels = 0;
    const int32_t *lvl_inf = nullptr;  // host array [n_levels+1]
    const int32_t *lvl_seq = nullptr;  // host array [n_levels+1]
    const uint8_t *lvl_kind = nullptr; // host array [n_levels]: 1 if every decision point of
                                       // the level has <= kFastActs actions, each with
                                       // <= kFastKids decision points below it; 2 if in
                                       // addition nothing lies below the level; else 0
    int32_t *inf_first = nullptr;      // [n_inf+1]
    int32_t *seq_par = nullptr;        // [n_seq] parent sequence of each sequence's decision point
    int32_t *child_ptr = nullptr;      // [n_seq+1] decision points below each sequence:
    int32_t *child_idx = nullptr;      //   child_idx[child_ptr[s] .. child_ptr[s+1])
    void *r = nullptr;                 // [n_seq] accumulator type
    void *m = nullptr;                 // [n_seq] accumulator type
    void *s = nullptr;                 // [n_seq] accumulator type
    void *b = nullptr;                 // [n_seq] value type
    void *x = nullptr;                 // [n_seq] value type
    void *g = nullptr;                 // [n_seq] value type
    void *xbar = nullptr;              // [n_seq] value type
    void *vinf = nullptr;              // [n_inf] compute type
    // shallow levels 0 .. top_levels-1 run in one launch (k_top), one block
    // per root decision point (n_roots of them)
    int32_t top_levels = 0;
    int32_t n_roots = 0;
    int32_t *top_off = nullptr;        // [top_levels*(n_roots+1)]
    int32_t *top_list = nullptr;       // decision points grouped by level, then root
    int top_fast = 0;                  // every level in k_top is a fast level
};

// Kernel launchers (cfr_kernels.hip).  All enqueue on `st` and return the
// launch status.
hipError_t launch_uniform_b(int prec, const DevPlayer &p, hipStream_t st);
// begin_sc != nullptr: the first block also advances the iteration scalars.
hipError_t launch_spmv(int prec, const DevMatrix &A, const void *xin, void *yout,
                       int xcd_remap, int sequential, Scalars *begin_sc, const IterParams &ip,
                       hipStream_t st);
hipError_t launch_up_level(int prec, int variant, const DevPlayer &p, int level, double usign,
                           const void *g, const Scalars *sc, hipStream_t st);
hipError_t launch_down_level(int prec, const DevPlayer &p, int level, int average,
                             const Scalars *sc, hipStream_t st);
// launch_up_level on level 0 also runs that level's top-down step.
// ObserveUtility on levels top_levels-1..0, then the top-down pass on levels
// 0..top_levels-1 (with averaging when `average`).
hipError_t launch_top(int prec, int variant, const DevPlayer &p, double usign, int average,
                      const Scalars *sc, hipStream_t st);
hipError_t launch_normalize(int prec, const DevPlayer &p, const Scalars *sc, hipStream_t st);
hipError_t launch_br_level(int prec, const DevPlayer &p, int level, double usign,
                           const void *g, hipStream_t st);
hipError_t launch_root_value(int prec, const DevPlayer &p, double usign, const void *g,
                             double *out, hipStream_t st);
hipError_t launch_dot(int prec, int32_t n, const void *a, const void *b, double *partials,
                      int n_partials, double *out, hipStream_t st);

size_t value_bytes(int prec);
size_t accum_bytes(int prec);
size_t compute_bytes(int prec);

// Payoff-product tiling (overridable at build time for tuning sweeps).
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
constexpr int kSpmvItems = CFR_SPMV_ITEMS;
constexpr int kSpmvCap = kSpmvThreads * kSpmvItems;  // nonzeros staged per block
constexpr int kSpmvRowCap = 256;                     // rows per block
static_assert(kSpmvRowCap <= kSpmvThreads, "a block's row pointers are one per thread");
constexpr int kDotPartials = 512;
// 1: run the shallow levels in one launch (k_top) even when deeper levels
// remain as per-level launches
#ifndef CFR_TOP_PARTIAL
#define CFR_TOP_PARTIAL 0
#endif
constexpr int kFastActs = 4;        // fast sweep path: actions per decision point
constexpr int kFastKids = 4;        // fast sweep path: decision points below a sequence
constexpr int kTopThreads = 1024;   // threads of the shallow-level block
constexpr int kTopMaxGroup = 1024;  // decision points per root and level it takes

}  // namespace cfr
