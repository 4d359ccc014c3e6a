// HIP kernels for one iteration of sequence-form CFR on gfx950.
//
// The path is sparse and bandwidth-bound (about 0.25 flop per byte), so
// nothing here uses MFMA.  Every launch walks a table of blocks; each entry
// names a game and a range of it, so one launch serves one game or a whole
// batch of games (global indices, per-game scalars).  Kernels:
//   k_spmv      payoff product over a row-sorted matrix (A y over the CSR,
//               A^T x over the CSC): each 256-thread block owns a run of
//               whole rows of one game, streams their index/value pairs with
//               coalesced loads, gathers the input vector, stages the
//               products in LDS, and sums every row.  A row longer than one
//               block's capacity gets a block of its own and a tree
//               reduction.
//   k_up        one treeplex level of ObserveUtility (Algorithm 2, bottom-up
//               part and regret update) fused with the variant's post-step
//               and with regret matching for the next strategy: one thread
//               per decision point.
//   k_down      one treeplex level of NextStrategy's top-down pass, fused
//               with the average-strategy accumulation of the strategy it
//               overwrites: one thread per sequence.
//   k_down_all  the whole top-down pass below level 0 in one launch: each
//               sequence multiplies its parent chain from the root down.
//   k_top       the shallow levels of a lone game, bottom-up then top-down,
//               in one launch: one block per root decision point's subtree.
//   k_shallow   the shallow levels of a game iterating alone, bottom-up, in
//               one 1024-thread block, values passed between levels in LDS.
//   k_fuse      the small levels below those in one launch, a block per
//               group of whole subtrees from a host-built list.
//   k_br        one level of the best-response max-sweep.
//   k_normalize / k_root / k_dot   average normalisation and deterministic
//               per-game scalar reductions.  The per-iteration scalars (t,
//               the averaging weight, the DCFR factors) of each game are
//               advanced by that game's first block of the iteration's first
//               payoff product.
// Precision modes select the value type (payoffs, strategies, utilities),
// the accumulator type (regrets, predictions, averages) and the compute
// type (in-register arithmetic).  No kernel uses atomics, so every result
// is run-to-run reproducible, and no reduction mixes two games, so a game's
// iterates do not depend on which other games share its launches.
#include "cfr_internal.h"

#include <hip/hip_ext.h>

#include <cfloat>
#include <type_traits>

#include "cfr.h"

namespace cfr {

template <int P>
struct Types;
template <>
struct Types<CFR_FP64> {
    using V = double;
    using R = double;
    using C = double;
};
template <>
struct Types<CFR_FP32> {
    using V = float;
    using R = float;
    using C = float;
};
template <>
struct Types<CFR_FP32_ACC64> {
    using V = float;
    using R = double;
    using C = double;
};

size_t value_bytes(int prec) { return prec == CFR_FP64 ? 8 : 4; }
size_t accum_bytes(int prec) { return prec == CFR_FP32 ? 4 : 8; }
size_t compute_bytes(int prec) { return prec == CFR_FP32 ? 4 : 8; }

namespace {

constexpr int kThreads = 256;
constexpr int kMaxActs = 8;  // decision points up to this size keep their actions in registers

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// Four consecutive stream elements with 16-byte loads (the address is a
// multiple of four elements).
__device__ __forceinline__ v4i load4(const int32_t *p)
{
#if CFR_SPMV_NONTEMPORAL
    return __builtin_nontemporal_load((const v4i *)p);
#else
    return *(const v4i *)p;
#endif
}
__device__ __forceinline__ void load4(const float *p, float (&o)[4])
{
#if CFR_SPMV_NONTEMPORAL
    const v4f t = __builtin_nontemporal_load((const v4f *)p);
#else
    const v4f t = *(const v4f *)p;
#endif
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
}
__device__ __forceinline__ void load4(const double *p, double (&o)[4])
{
#if CFR_SPMV_NONTEMPORAL
    const v2d a = __builtin_nontemporal_load((const v2d *)p);
    const v2d b = __builtin_nontemporal_load((const v2d *)p + 1);
#else
    const v2d a = *(const v2d *)p, b = *((const v2d *)p + 1);
#endif
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}
// Four entries of a gathered vector (aligned to four), through the caches.
__device__ __forceinline__ void load4_cached(const float *p, float (&o)[4])
{
    const v4f t = *(const v4f *)p;
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
}
__device__ __forceinline__ void load4_cached(const double *p, double (&o)[4])
{
    const v2d a = *(const v2d *)p, b = *((const v2d *)p + 1);
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}
__device__ __forceinline__ void store4(float *p, const float (&o)[4])
{
    *(v4f *)p = v4f{o[0], o[1], o[2], o[3]};
}
__device__ __forceinline__ void store4(double *p, const double (&o)[4])
{
    *(v2d *)p = v2d{o[0], o[1]};
    *((v2d *)p + 1) = v2d{o[2], o[3]};
}

// ---------------------------------------------------------------------------
// Per-iteration scalars
// ---------------------------------------------------------------------------

__device__ __forceinline__ void begin_iteration(Scalars *sc)
{
    double t = sc->t + 1.0;
    sc->t = t;
    int kind = sc->avg_kind;
    const int variant = sc->variant;
    if (kind == CFR_AVG_DEFAULT) {
        kind = variant == CFR_PLUS        ? CFR_AVG_LINEAR
               : variant == CFR_DCFR      ? CFR_AVG_POW_GAMMA
               : variant == CFR_PCFR_PLUS ? CFR_AVG_QUADRATIC
                                          : CFR_AVG_UNIFORM;
    }
    double w = 1.0;
    if (kind == CFR_AVG_LINEAR) w = t;
    else if (kind == CFR_AVG_QUADRATIC) w = t * t;
    else if (kind == CFR_AVG_POW_GAMMA) w = pow(t, sc->gamma);
    sc->w = w;
    sc->W = sc->W + w;
    double ta = pow(t, sc->alpha), tb = pow(t, sc->beta);
    sc->dpos = ta / (ta + 1.0);
    sc->dneg = tb / (tb + 1.0);
}

// Out of line, one copy per product kernel family: a called function is
// compiled under its callers' register budget only when they all share it.
template <bool QUADS>
__device__ __noinline__ void begin_iteration_in(Scalars *sc)
{
    begin_iteration(sc);
}

// ---------------------------------------------------------------------------
// Payoff product y = M x over a row-sorted matrix
// ---------------------------------------------------------------------------

// SEQ: every row is summed strictly left to right (the order of a plain
// sequential loop), which the FP64 path needs to reproduce a sequential
// evaluation bit for bit; otherwise a power-of-two group of lanes shares
// each row and combines its partial sums with cross-lane shuffles.
//
// VEC 1: the index and value streams are read four elements per lane with
// 16-byte loads from the block's first element rounded down to a multiple
// of four (the block partition leaves room for the up to three elements
// before it); products are staged at their offset from that aligned start.
// Elements outside the block gather entry 0 and stage a zero that no row
// reads.  One gather instruction then reads every fourth element.
// VEC 2: the same 16-byte loads, after which each wave turns its own
// 256-element chunks around through LDS, so that one gather instruction
// reads 64 consecutive elements (whose column indices lie close together).
// VEC 0: every element is its own 4-byte load, consecutive across lanes.
// VEC 3: the stream is in quads (a derived copy of the matrix): each element
// is a run of at most four nonzeros of one row, in row order, whose columns
// lie in one aligned group of four (quad index | presence mask << 28), with
// four values (any value where the mask is clear); one aligned 16-byte
// gather fetches the four input entries.  Absent positions stage -0.0,
// which leaves every sum unchanged (x + -0.0 == x exactly, signed zeros
// included), so the row sums are exactly those of the nonzeros in row
// order.  Row pointers and block extents count quads.  In the sequential
// order staging slot 4*q + k holds position k of quad q; otherwise slot q
// holds quad q's sum (its positions added in order), so rows are reduced
// over a quarter of the slots.
//
// Each table entry gives a block's rows, nonzeros and game in one scalar
// load.  The loads of a block are all issued
// unconditionally (lanes past the end read the block's first entry and
// ignore it): index/value stream and row pointers in one round, gathers in
// the next; the reduction then reads only LDS.
template <int P, bool SEQ, int ITEMS, int VEC>
__device__ __forceinline__ void spmv_blocks(
    int32_t n_blk, const SpmvBlock *__restrict__ tab, const int32_t *__restrict__ ptr,
    const int32_t *__restrict__ idx, const typename Types<P>::V *__restrict__ val,
    const typename Types<P>::V *__restrict__ xin, typename Types<P>::V *__restrict__ yout,
    int xcd_remap, int begin, Scalars *sc)
{
    using V = typename Types<P>::V;
    using C = typename Types<P>::C;
    // products staged in LDS: the compute type, or the value type when the
    // FP32 modes are built to stage them compactly
    using L = typename std::conditional<(CFR_SPMV_LDS_VALUE != 0) && P != CFR_FP64, V, C>::type;
    // staged products per block; summed quads take one slot each, so that
    // form needs a quarter of the space (and leaves LDS out of the
    // occupancy limit)
    constexpr int kCap = VEC == 3 && !SEQ ? kSpmvThreads * ITEMS / 4 : kSpmvThreads * ITEMS;
    __shared__ L prod[kCap];
    __shared__ int32_t s_ptr[kSpmvRowCap + 1];
    __shared__ C red[kSpmvThreads];

    int32_t bid = (int32_t)blockIdx.x;
    if (xcd_remap) {
        // Workgroups are dealt round-robin over the 8 XCDs; give each XCD a
        // contiguous range of row blocks so neighbouring rows (which gather
        // neighbouring input entries) share one L2.
        int32_t per = (n_blk + 7) / 8;
        bid = (int32_t)(blockIdx.x % 8) * per + (int32_t)(blockIdx.x / 8);
    }
    if (bid >= n_blk) return;
    const int tid = threadIdx.x;
    const SpmvBlock bk = tab[bid];
    if (begin && bk.begin && tid == 0)
        begin_iteration_in<VEC == 3 && !SEQ && P != CFR_FP64>(sc + bk.slot);
    const int32_t rb = bk.row0, nr = bk.nr, n = bk.n, p0 = bk.p0;
    const int64_t e0 = bk.e0;

    constexpr int32_t kBlockCap = VEC == 3 ? kSpmvThreads * ITEMS / 4 : spmv_block_cap(ITEMS);
    if (n > kBlockCap) {
        // a single long row: strided partial sums, then a fixed-order tree
        C acc = 0;
        if (VEC == 3) {
            for (int32_t i = tid; i < n; i += kSpmvThreads) {
                const uint32_t qd = (uint32_t)idx[e0 + i];
                const int64_t c0 = 4 * (int64_t)(qd & kQuadIndexMask);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if ((qd >> (kQuadMaskShift + k)) & 1u)
                        acc = acc + (C)val[4 * (e0 + i) + k] * (C)xin[c0 + k];
            }
        } else {
            for (int32_t i = tid; i < n; i += kSpmvThreads)
                acc = acc + (C)val[e0 + i] * (C)xin[idx[e0 + i]];
        }
        red[tid] = acc;
        __syncthreads();
        for (int w = kSpmvThreads / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] = red[tid] + red[tid + w];
            __syncthreads();
        }
        if (tid == 0) yout[rb] = (V)red[0];
        return;
    }

    // this block's row pointers: one per thread (a block has at most
    // kSpmvRowCap = kSpmvThreads rows)
    const int32_t pr = ptr[rb + (tid < nr ? tid : 0)];
    int32_t sh = 0;  // staging offset of the block's first element
    int32_t per = 1;  // staging slots per stream element
    if (VEC == 3) {
        constexpr int NQ = ITEMS / 4;
        // the sequential (FP64) order stages every position; otherwise a
        // quad's positions (one row, in order) are summed here and the
        // quad is staged as one value
        per = SEQ ? 4 : 1;
        if (n > 0) {
            uint32_t qd[NQ];
            V v4[NQ][4];
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                const int32_t qi = j * kSpmvThreads + tid;
                const int64_t at = e0 + (qi < n ? qi : 0);
                qd[j] = (uint32_t)__builtin_nontemporal_load(idx + at);
                load4(val + 4 * at, v4[j]);
            }
            V gx[NQ][4];
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                load4_cached(xin + 4 * (int64_t)(qd[j] & kQuadIndexMask), gx[j]);
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                const int32_t qi = j * kSpmvThreads + tid;
                if (SEQ) {
                    L o[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        o[k] = (qi < n && ((qd[j] >> (kQuadMaskShift + k)) & 1u))
                                   ? (L)((C)v4[j][k] * (C)gx[j][k])
                                   : (L)(-0.0);
                    store4(&prod[4 * qi], o);
                } else {
                    C qs = (C)(-0.0);
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if ((qd[j] >> (kQuadMaskShift + k)) & 1u)
                            qs = qs + (C)v4[j][k] * (C)gx[j][k];
                    prod[qi] = (L)qs;  // lanes past the block stage a value no row reads
                }
            }
        }
    } else if (VEC == 2) {
        constexpr int NV = ITEMS / 4;
        const int64_t e_al = e0 & ~(int64_t)3;
        sh = (int32_t)(e0 - e_al);
        const int32_t n_al = n + sh;
        if (n > 0) {
            v4i c4[NV];
            V v4[NV][4];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int32_t vi = j * kSpmvThreads + tid;
                const int64_t at = e_al + 4 * (int64_t)(4 * vi < n_al ? vi : 0);
                c4[j] = load4(idx + at);
                load4(val + at, v4[j]);
            }
            // Staging slot 4*vi + e holds element e of lane vi's load; a
            // wave's loads of round j fill slots [4*(j*256 + w0), +256), w0
            // its first thread, and it reads them back as slot
            // 4*(j*256 + w0) + 64*e + lane.  The chunks of different waves
            // are disjoint and the LDS serves one wave's accesses in order,
            // so a wave-level code-motion barrier is all the ordering needed.
            const int lane = tid & 63;
            const int32_t w0 = tid & ~63;
            constexpr int IS = (int)(sizeof(L) / sizeof(int32_t));  // index view: ints per slot
            int32_t *ti = reinterpret_cast<int32_t *>(prod);
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int32_t vi = j * kSpmvThreads + tid;
#pragma unroll
                for (int e = 0; e < 4; ++e) ti[IS * (4 * vi + e)] = c4[j][e];
            }
            __builtin_amdgcn_wave_barrier();
            // all index reads first, then all gathers (one round)
            int32_t ct[NV][4];
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int32_t sl = 4 * (j * kSpmvThreads + w0) + 64 * e + lane;
                    const int32_t q = sl - sh;
                    const int32_t c = ti[IS * sl];
                    ct[j][e] = (q >= 0 && q < n) ? c : 0;
                }
            V gx[NV][4];
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) gx[j][e] = xin[ct[j][e]];
            __builtin_amdgcn_wave_barrier();
            // the values take the same way round while the gathers fly
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int32_t vi = j * kSpmvThreads + tid;
                L o[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = (L)v4[j][e];
                store4(&prod[4 * vi], o);
            }
            __builtin_amdgcn_wave_barrier();
            L vt[NV][4];
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    vt[j][e] = prod[4 * (j * kSpmvThreads + w0) + 64 * e + lane];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int32_t sl = 4 * (j * kSpmvThreads + w0) + 64 * e + lane;
                    const int32_t q = sl - sh;
                    prod[sl] = (q >= 0 && q < n) ? (L)((C)vt[j][e] * (C)gx[j][e]) : (L)0;
                }
        }
    } else if (VEC == 1) {
        constexpr int NV = ITEMS / 4;
        const int64_t e_al = e0 & ~(int64_t)3;
        sh = (int32_t)(e0 - e_al);
        const int32_t n_al = n + sh;
        if (n > 0) {
            v4i c4[NV];
            V v4[NV][4];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int32_t vi = j * kSpmvThreads + tid;
                const int64_t at = e_al + 4 * (int64_t)(4 * vi < n_al ? vi : 0);
                c4[j] = load4(idx + at);
                load4(val + at, v4[j]);
            }
            V gx[NV][4];
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int32_t q = 4 * (j * kSpmvThreads + tid) + e - sh;
                    gx[j][e] = xin[(q >= 0 && q < n) ? c4[j][e] : 0];
                }
            // every lane stores its four slots (zeros outside the block):
            // no branch the loads above could be moved into
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int32_t vi = j * kSpmvThreads + tid;
                L o[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int32_t q = 4 * vi + e - sh;
                    o[e] = (q >= 0 && q < n) ? (L)((C)v4[j][e] * (C)gx[j][e]) : (L)0;
                }
                store4(&prod[4 * vi], o);
            }
        }
    } else if (n > 0) {
        int32_t c[ITEMS];
        V v[ITEMS];
        V gx[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int32_t i = k * kSpmvThreads + tid;
            const int64_t at = e0 + (i < n ? i : 0);
#if CFR_SPMV_NONTEMPORAL
            c[k] = __builtin_nontemporal_load(idx + at);
            v[k] = __builtin_nontemporal_load(val + at);
#else
            c[k] = idx[at];
            v[k] = val[at];
#endif
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) gx[k] = xin[c[k]];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int32_t i = k * kSpmvThreads + tid;
            if (i < n) prod[i] = (L)((C)v[k] * (C)gx[k]);
        }
    }
    if (tid < nr) s_ptr[tid] = per * (pr - p0) + sh;
    if (tid == 0) s_ptr[nr] = per * n + sh;
    __syncthreads();
    if (SEQ) {
        if (tid < nr) {
            int32_t i = s_ptr[tid];
            const int32_t z = s_ptr[tid + 1];
            C acc = 0;
            for (; i + 4 <= z; i += 4) {
                C q0 = prod[i], q1 = prod[i + 1], q2 = prod[i + 2], q3 = prod[i + 3];
                acc = acc + q0;
                acc = acc + q1;
                acc = acc + q2;
                acc = acc + q3;
            }
            for (; i < z; ++i) acc = acc + (C)prod[i];
            yout[rb + tid] = (V)acc;
        }
        return;
    }
    // lanes per row: the largest power of two (<= 64) that still gives every
    // row of the block its own group, and not far above the mean row length
    int Lr = 64;
    while (Lr > 1 && Lr * nr > kSpmvThreads) Lr >>= 1;
    while (Lr > 1 && Lr > 2 * (per * n / nr + 1)) Lr >>= 1;
    const int lane = tid & (Lr - 1);
    const int groups = kSpmvThreads / Lr;
    for (int32_t r = tid / Lr; r < nr; r += groups) {
        const int32_t a = s_ptr[r], z = s_ptr[r + 1];
        C acc = 0;
        for (int32_t i = a + lane; i < z; i += Lr) acc = acc + (C)prod[i];
        for (int off = Lr >> 1; off > 0; off >>= 1) acc = acc + __shfl_xor(acc, off, Lr);
        if (lane == 0) yout[rb + r] = (V)acc;
    }
}

#define CFR_SPMV_PARAMS(P)                                                                    \
    int32_t n_blk, const SpmvBlock *__restrict__ tab, const int32_t *__restrict__ ptr,        \
        const int32_t *__restrict__ idx, const typename Types<P>::V *__restrict__ val,        \
        const typename Types<P>::V *__restrict__ xin, typename Types<P>::V *__restrict__ yout, \
        int xcd_remap, int begin, Scalars *sc

template <int P, bool SEQ, int ITEMS, int VEC>
__global__ __launch_bounds__(kSpmvThreads) void k_spmv(CFR_SPMV_PARAMS(P))
{
    spmv_blocks<P, SEQ, ITEMS, VEC>(n_blk, tab, ptr, idx, val, xin, yout, xcd_remap, begin, sc);
}

// Summed quads with FP32 values.  Left to itself the compiler gives this
// form more than 100 SGPRs, which allows seven waves per SIMD; it fits in
// eight (at most 64 VGPRs, a few SGPRs kept in VGPR lanes), which keeps more
// of the stream in flight, so the bound asks for eight.  The other forms
// keep the compiler's choice (eight would spill VGPRs to memory there).
template <int P, int ITEMS>
__global__ __launch_bounds__(kSpmvThreads, 8) void k_spmv_quads(CFR_SPMV_PARAMS(P))
{
    spmv_blocks<P, false, ITEMS, 3>(n_blk, tab, ptr, idx, val, xin, yout, xcd_remap, begin, sc);
}
#undef CFR_SPMV_PARAMS

// ---------------------------------------------------------------------------
// ObserveUtility for one level, fused with the variant and regret matching
// ---------------------------------------------------------------------------

template <int P, int VAR>
__device__ __forceinline__ typename Types<P>::C post_step(typename Types<P>::C r,
                                                          typename Types<P>::C dpos,
                                                          typename Types<P>::C dneg)
{
    if (VAR == CFR_PLUS || VAR == CFR_PCFR_PLUS) return r > 0 ? r : 0;
    if (VAR == CFR_DCFR) {
        if (r > 0) return r * dpos;
        if (r < 0) return r * dneg;
    }
    return r;
}

// Values of the decision points below each sequence, in slots: on a level
// flagged to write slots (SL & kSlotsWrite), a decision point whose parent
// sequence has at most kFastKids of them stores its value at
// cval[4 * parent + (its rank among them)] instead of vinf, and the parent's
// level (SL & kSlotsRead) reads them with its own action data instead of
// through child_idx.  Only small levels write slots (their writes scatter);
// the flags come with each block of the table and select a compiled copy
// of the level's code, so that each copy issues its loads in as few
// dependent rounds as it can.
template <int P>
struct Kids {
    const int32_t *__restrict__ cslot;   // [decision points] slot, or -1
    const uint8_t *__restrict__ ccount;  // [sequences] decision points below (if <= kFastKids)
    typename Types<P>::C *__restrict__ cval;  // [4 * sequences]
};

// The value of decision point j for its parent's level.
template <int P>
__device__ __forceinline__ void store_value(const Kids<P> &kd, int32_t cs, int32_t j,
                                            typename Types<P>::C *__restrict__ vinf,
                                            typename Types<P>::C v)
{
    if (cs >= 0) kd.cval[cs] = v;
    else vinf[j] = v;
}

// One decision point of ObserveUtility: counterfactual utilities of its
// actions (own utility plus the values of the decision points below), its
// value, the regret update with the variant's post-step, and regret
// matching for the next strategy.
// acc plus the values of the child decision points [c0, c1) of one sequence,
// added one by one in ascending order.  The loop takes the children eight at
// a time and issues
// all eight index loads, then all eight value loads (clamped to the last
// child, the extra ones discarded), before the additions: a wide sequence
// waits for two memory rounds per eight children instead of two per child.
// The sum is the one a child-by-child loop gives.
template <int P>
__device__ __forceinline__ typename Types<P>::C child_sum(
    typename Types<P>::C acc, int32_t c0, int32_t c1, const int32_t *__restrict__ child_idx,
    const typename Types<P>::C *__restrict__ vals)
{
    using C = typename Types<P>::C;
    constexpr int kChunk = 8;
    for (int32_t c = c0; c < c1; c += kChunk) {
        int32_t ci[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) ci[k] = child_idx[c + k < c1 ? c + k : c1 - 1];
        C cv[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) cv[k] = vals[ci[k]];
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            if (c + k < c1) acc = acc + cv[k];
    }
    return acc;
}

template <int P, int VAR, int SL>
__device__ __forceinline__ void up_infoset(
    int32_t j, const int32_t *__restrict__ inf_first, const int32_t *__restrict__ child_ptr,
    const int32_t *__restrict__ child_idx, const typename Types<P>::V *__restrict__ g,
    typename Types<P>::C usign, typename Types<P>::C *__restrict__ vinf,
    typename Types<P>::V *__restrict__ b, typename Types<P>::R *__restrict__ r,
    typename Types<P>::R *__restrict__ m, typename Types<P>::C dpos, typename Types<P>::C dneg,
    const Kids<P> &kd)
{
    using V = typename Types<P>::V;
    using R = typename Types<P>::R;
    using C = typename Types<P>::C;
    constexpr bool kPred = VAR == CFR_PCFR_PLUS || VAR == CFR_PCFR;
    const int32_t a0 = inf_first[j], a1 = inf_first[j + 1];
    const int32_t n = a1 - a0;
    const int32_t cs = (SL & kSlotsWrite) ? kd.cslot[j] : -1;

    // Counterfactual values of the actions g0 .. g0 + kGroup - 1 below a1
    // (q[k]): the payoff plus the child decision points' values, added in
    // order, from the action's value slots when it has at most kFastKids
    // children, else from its child list.  The group's per-action loads
    // (payoff, slot count, child range) are issued together before the
    // child sums, instead of one action after another.
    constexpr int kGroup = 4;
    auto group_q = [&](int32_t g0, C *q) {
        int32_t cnt[kGroup], c0[kGroup], c1[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            const int32_t a = g0 + k < a1 ? g0 + k : a1 - 1;
            q[k] = usign * (C)g[a];
            cnt[k] = (SL & kSlotsRead) ? (int)kd.ccount[a] : kFastKids + 1;
            c0[k] = child_ptr[a];
            c1[k] = child_ptr[a + 1];
        }
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            const int32_t a = g0 + k;
            if (a >= a1) continue;
            if (cnt[k] <= kFastKids) {
                for (int i = 0; i < cnt[k]; ++i) q[k] = q[k] + kd.cval[4 * (int64_t)a + i];
            } else {
                q[k] = child_sum<P>(q[k], c0[k], c1[k], child_idx, vinf);
            }
        }
    };

    if (n <= kMaxActs) {
        static_assert(kMaxActs == 2 * kGroup, "two groups");
        C q[kMaxActs];
        group_q(a0, q);
        if (n > kGroup) group_q(a0 + kGroup, q + kGroup);
        C V_ = 0;
#pragma unroll
        for (int k = 0; k < kMaxActs; ++k)
            if (k < n) V_ = V_ + (C)b[a0 + k] * q[k];
        store_value(kd, cs, j, vinf, V_);
        C z[kMaxActs];
        C Z = 0;
#pragma unroll
        for (int k = 0; k < kMaxActs; ++k) {
            if (k < n) {
                const int32_t a = a0 + k;
                C inst = q[k] - V_;
                C rr = post_step<P, VAR>((C)r[a] + inst, dpos, dneg);
                r[a] = (R)rr;
                C zz = (C)(R)rr;
                if (kPred) {
                    m[a] = (R)inst;
                    zz = zz + (C)(R)inst;
                }
                zz = zz > 0 ? zz : 0;
                z[k] = zz;
                Z = Z + zz;
            }
        }
#pragma unroll
        for (int k = 0; k < kMaxActs; ++k) {
            if (k < n) b[a0 + k] = (V)(Z > 0 ? z[k] / Z : (C)1 / (C)n);
        }
        return;
    }

    // large decision points: recompute instead of holding every action,
    // a group of actions at a time (strategies and regrets loaded together
    // too); the arithmetic is the same, in the same order.
    C V_ = 0;
    for (int32_t g0 = a0; g0 < a1; g0 += kGroup) {
        C q[kGroup], bb[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k) bb[k] = (C)b[g0 + k < a1 ? g0 + k : a1 - 1];
        group_q(g0, q);
#pragma unroll
        for (int k = 0; k < kGroup; ++k)
            if (g0 + k < a1) V_ = V_ + bb[k] * q[k];
    }
    store_value(kd, cs, j, vinf, V_);
    C Z = 0;
    for (int32_t g0 = a0; g0 < a1; g0 += kGroup) {
        C q[kGroup], rv[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k) rv[k] = (C)r[g0 + k < a1 ? g0 + k : a1 - 1];
        group_q(g0, q);
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            const int32_t a = g0 + k;
            if (a >= a1) continue;
            C inst = q[k] - V_;
            C rr = post_step<P, VAR>(rv[k] + inst, dpos, dneg);
            r[a] = (R)rr;
            C zz = (C)(R)rr;
            if (kPred) {
                m[a] = (R)inst;
                zz = zz + (C)(R)inst;
            }
            Z = Z + (zz > 0 ? zz : 0);
        }
    }
    for (int32_t g0 = a0; g0 < a1; g0 += kGroup) {
        C zz[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            const int32_t a = g0 + k < a1 ? g0 + k : a1 - 1;
            zz[k] = (C)r[a];
            if (kPred) zz[k] = zz[k] + (C)m[a];
        }
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            if (g0 + k >= a1) continue;
            const C z = zz[k] > 0 ? zz[k] : 0;
            b[g0 + k] = (V)(Z > 0 ? z / Z : (C)1 / (C)n);
        }
    }
}

// The fast path of up_infoset below (up_infoset_fast) split in two, for
// the one-block pass over the shallow levels, which issues every level's
// loads before computing any level.  The loads of one fast-path decision
// point (at most kFastActs actions, each with at most kFastKids decision
// points below it): its action range, each
// action's payoff, strategy and regret (and prediction), and the child
// counts with either the child values (from value slots, SL & kSlotsRead)
// or the child ids (the caller then reads the values).  Every load is
// issued unconditionally (lanes past the end read a valid clamped address
// and ignore the value), so one dependent round serves each of: action
// range; action data with child pointers, or with child counts and values
// when the level reads slots; otherwise child ids.
template <int P, int NC>
struct FastLoads {
    static constexpr int NCA = NC > 0 ? NC : 1;
    int32_t a0, n;
    typename Types<P>::V gv[kFastActs], bv[kFastActs];
    typename Types<P>::R rv[kFastActs], mv[kFastActs];
    int cnt[kFastActs];
    typename Types<P>::C cv[kFastActs][NCA];
    int32_t cid[kFastActs][NCA];
};

template <int P, int VAR, int NC, int SL>
__device__ __forceinline__ void fast_load(int32_t j, const int32_t *__restrict__ inf_first,
                                          const int32_t *__restrict__ child_ptr,
                                          const int32_t *__restrict__ child_idx,
                                          const typename Types<P>::V *__restrict__ g,
                                          const typename Types<P>::V *__restrict__ b,
                                          const typename Types<P>::R *__restrict__ r,
                                          const typename Types<P>::R *__restrict__ m,
                                          const Kids<P> &kd, FastLoads<P, NC> &L)
{
    static_assert(NC == 0 || NC == 4, "child values are read as slots of four");
    constexpr int NA = kFastActs;
    constexpr bool kPred = VAR == CFR_PCFR_PLUS || VAR == CFR_PCFR;
    L.a0 = inf_first[j];
    L.n = inf_first[j + 1] - L.a0;
    if (NC > 0 && (SL & kSlotsRead)) {
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int32_t a = L.a0 + (k < L.n ? k : 0);
            L.gv[k] = g[a];
            L.bv[k] = b[a];
            L.rv[k] = r[a];
            if (kPred) L.mv[k] = m[a];
            L.cnt[k] = kd.ccount[a];
#pragma unroll
            for (int i = 0; i < NC; ++i) L.cv[k][i] = kd.cval[4 * (int64_t)a + i];
        }
    } else {
        int32_t c0[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int32_t a = L.a0 + (k < L.n ? k : 0);
            L.gv[k] = g[a];
            L.bv[k] = b[a];
            L.rv[k] = r[a];
            if (kPred) L.mv[k] = m[a];
            if (NC > 0) {
                c0[k] = child_ptr[a];
                L.cnt[k] = child_ptr[a + 1] - c0[k];
            } else {
                c0[k] = 0;
                L.cnt[k] = 0;
            }
        }
        if (NC > 0) {
#pragma unroll
            for (int k = 0; k < NA; ++k)
#pragma unroll
                for (int i = 0; i < NC; ++i)
                    L.cid[k][i] = child_idx[i < L.cnt[k] ? c0[k] + i : 0];
        }
    }
}

// The arithmetic of one fast-path decision point from its loads (child
// values in L.cv): counterfactual values q (own payoff, then the children in
// ascending order), the value V = sum_a b q, the regret update with the
// variant's post-step, and regret matching.  Writes r (and m) and the next
// strategy b; returns V.  The arithmetic and its order are exactly those
// of up_infoset and up_infoset_fast (a one-block pass equals a launch per
// level bit for bit, which the tests check).
template <int P, int VAR, int NC>
__device__ __forceinline__ typename Types<P>::C fast_apply(
    const FastLoads<P, NC> &L, typename Types<P>::C usign, typename Types<P>::V *__restrict__ b,
    typename Types<P>::R *__restrict__ r, typename Types<P>::R *__restrict__ m,
    typename Types<P>::C dpos, typename Types<P>::C dneg)
{
    using V = typename Types<P>::V;
    using R = typename Types<P>::R;
    using C = typename Types<P>::C;
    constexpr int NA = kFastActs;
    constexpr bool kPred = VAR == CFR_PCFR_PLUS || VAR == CFR_PCFR;
    const int32_t a0 = L.a0, n = L.n;
    C q[NA];
    C V_ = 0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        if (k < n) {
            C acc = usign * (C)L.gv[k];
#pragma unroll
            for (int i = 0; i < NC; ++i)
                if (i < L.cnt[k]) acc = acc + L.cv[k][i];
            q[k] = acc;
            V_ = V_ + (C)L.bv[k] * acc;
        }
    }
    C z[NA];
    C Z = 0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        if (k < n) {
            const int32_t a = a0 + k;
            C inst = q[k] - V_;
            C rr = post_step<P, VAR>((C)L.rv[k] + inst, dpos, dneg);
            r[a] = (R)rr;
            C zz = (C)(R)rr;
            if (kPred) {
                m[a] = (R)inst;
                zz = zz + (C)(R)inst;
            }
            zz = zz > 0 ? zz : 0;
            z[k] = zz;
            Z = Z + zz;
        }
    }
#pragma unroll
    for (int k = 0; k < NA; ++k)
        if (k < n) b[a0 + k] = (V)(Z > 0 ? z[k] / Z : (C)1 / (C)n);
    return V_;
}

// Fast path of up_infoset for a decision point with at most kFastActs
// actions, each with at most kFastKids decision points below it.  Every
// load is issued unconditionally (lanes past the end read a valid clamped
// address and ignore the value), so one dependent round serves each of:
// action range (and own slot); action data with child pointers, or with
// child counts and values when the block reads slots; otherwise child ids;
// child values.  The arithmetic and its order are exactly those of
// up_infoset (children in ascending order).
template <int P, int VAR, int NC, int SL, bool STORE = true>
__device__ __forceinline__ typename Types<P>::C up_infoset_fast(
    int32_t j, const int32_t *__restrict__ inf_first, const int32_t *__restrict__ child_ptr,
    const int32_t *__restrict__ child_idx, const typename Types<P>::V *__restrict__ g,
    typename Types<P>::C usign, typename Types<P>::C *__restrict__ vinf,
    typename Types<P>::V *__restrict__ b, typename Types<P>::R *__restrict__ r,
    typename Types<P>::R *__restrict__ m, typename Types<P>::C dpos, typename Types<P>::C dneg,
    const Kids<P> &kd)
{
    using V = typename Types<P>::V;
    using R = typename Types<P>::R;
    using C = typename Types<P>::C;
    // NC = 0: a level without children below it (no child loads at all)
    constexpr int NA = kFastActs, NCA = NC > 0 ? NC : 1;
    static_assert(NC == 0 || NC == 4, "child values are read as slots of four");
    constexpr bool kPred = VAR == CFR_PCFR_PLUS || VAR == CFR_PCFR;
    const int32_t a0 = inf_first[j], a1 = inf_first[j + 1];
    const int32_t cs = (STORE && (SL & kSlotsWrite)) ? kd.cslot[j] : -1;
    const int32_t n = a1 - a0;
    V gv[NA], bv[NA];
    R rv[NA], mv[NA];
    int cnt[NA];
    C cv[NA][NCA];
    if (NC > 0 && (SL & kSlotsRead)) {
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int32_t a = a0 + (k < n ? k : 0);
            gv[k] = g[a];
            bv[k] = b[a];
            rv[k] = r[a];
            if (kPred) mv[k] = m[a];
            cnt[k] = kd.ccount[a];
#pragma unroll
            for (int i = 0; i < NC; ++i) cv[k][i] = kd.cval[4 * (int64_t)a + i];
        }
    } else {
        int32_t c0[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int32_t a = a0 + (k < n ? k : 0);
            gv[k] = g[a];
            bv[k] = b[a];
            rv[k] = r[a];
            if (kPred) mv[k] = m[a];
            if (NC > 0) {
                c0[k] = child_ptr[a];
                cnt[k] = child_ptr[a + 1] - c0[k];
            } else {
                c0[k] = 0;
                cnt[k] = 0;
            }
        }
        if (NC > 0) {
            int32_t cid[NA][NCA];
#pragma unroll
            for (int k = 0; k < NA; ++k)
#pragma unroll
                for (int i = 0; i < NC; ++i) cid[k][i] = child_idx[i < cnt[k] ? c0[k] + i : 0];
#pragma unroll
            for (int k = 0; k < NA; ++k)
#pragma unroll
                for (int i = 0; i < NC; ++i) cv[k][i] = vinf[cid[k][i]];
        }
    }
    C q[NA];
    C V_ = 0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        if (k < n) {
            C acc = usign * (C)gv[k];
#pragma unroll
            for (int i = 0; i < NC; ++i)
                if (i < cnt[k]) acc = acc + cv[k][i];
            q[k] = acc;
            V_ = V_ + (C)bv[k] * acc;
        }
    }
    if (STORE) store_value(kd, cs, j, vinf, V_);
    C z[NA];
    C Z = 0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        if (k < n) {
            const int32_t a = a0 + k;
            C inst = q[k] - V_;
            C rr = post_step<P, VAR>((C)rv[k] + inst, dpos, dneg);
            r[a] = (R)rr;
            C zz = (C)(R)rr;
            if (kPred) {
                m[a] = (R)inst;
                zz = zz + (C)(R)inst;
            }
            zz = zz > 0 ? zz : 0;
            z[k] = zz;
            Z = Z + zz;
        }
    }
#pragma unroll
    for (int k = 0; k < NA; ++k)
        if (k < n) b[a0 + k] = (V)(Z > 0 ? z[k] / Z : (C)1 / (C)n);
    return V_;
}

// One decision point of NextStrategy's top-down pass, accumulating the
// strategy it overwrites into the average first.
template <int P>
__device__ __forceinline__ void down_infoset(int32_t j, const int32_t *__restrict__ inf_first,
                                             const int32_t *__restrict__ seq_par,
                                             const typename Types<P>::V *__restrict__ b,
                                             typename Types<P>::V *__restrict__ x,
                                             typename Types<P>::R *__restrict__ s,
                                             typename Types<P>::R w, int average,
                                             bool parent_is_root = false)
{
    using V = typename Types<P>::V;
    using R = typename Types<P>::R;
    const int32_t a0 = inf_first[j], a1 = inf_first[j + 1];
    const int32_t n = a1 - a0;
    if (n <= kFastActs) {
        // all loads at once (clamped addresses), then the stores; under the
        // empty sequence the parent's realisation weight is exactly 1
        V bv[kFastActs], xv[kFastActs];
        R sv[kFastActs];
        const V xp = parent_is_root ? (V)1 : x[seq_par[a0]];
#pragma unroll
        for (int k = 0; k < kFastActs; ++k) {
            const int32_t a = a0 + (k < n ? k : 0);
            bv[k] = b[a];
            xv[k] = x[a];
            sv[k] = s[a];
        }
#pragma unroll
        for (int k = 0; k < kFastActs; ++k) {
            if (k < n) {
                if (average) s[a0 + k] = sv[k] + w * (R)xv[k];
                x[a0 + k] = xp * bv[k];
            }
        }
        return;
    }
    const V xp = parent_is_root ? (V)1 : x[seq_par[a0]];
    for (int32_t a = a0; a < a1; ++a) {
        if (average) s[a] = s[a] + w * (R)x[a];
        x[a] = xp * b[a];
    }
}

// The range of one block of a sweep launch: the table's entry, or with a
// direct range (hi > lo: one game's contiguous range, passed by value) the
// block's share of it, which saves the dependent load of the entry.
template <bool XCD>
__device__ __forceinline__ RangeBlock block_range(const RangeBlock *__restrict__ tab,
                                                  const RangeBlock &dr)
{
    if (dr.hi > dr.lo) {
        int32_t bid = (int32_t)blockIdx.x;
        if (XCD) {
            // workgroups are dealt round-robin over the 8 XCDs: each XCD
            // takes a contiguous eighth of the range (the grid is a multiple
            // of 8; blocks past the end get an empty range)
            const int32_t n = (dr.hi - dr.lo + kRangeBlock - 1) / kRangeBlock;
            const int32_t per = (n + 7) / 8;
            bid = (int32_t)(blockIdx.x % 8) * per + (int32_t)(blockIdx.x / 8);
        }
        const int32_t lo = dr.lo + bid * kRangeBlock;
        return RangeBlock{lo, min(lo + kRangeBlock, dr.hi), dr.slot, dr.aux};
    }
    return tab[blockIdx.x];
}

// One level of ObserveUtility over the decision points of the table's
// ranges.  KIND 0: any shape; 1: fast path; 2: fast path for a level with
// no decision points below it.  ROOT: the level under the empty sequence,
// whose top-down step (x = 1 * b, averaging the old x) needs nothing but
// this thread's own new strategy, so it is done here too.
template <int P, int VAR, int KIND, bool ROOT>
__global__ __launch_bounds__(kThreads) void k_up(
    const RangeBlock *__restrict__ tab, const int32_t *__restrict__ inf_first,
    const int32_t *__restrict__ child_ptr, const int32_t *__restrict__ child_idx,
    const typename Types<P>::V *__restrict__ g, typename Types<P>::C usign,
    typename Types<P>::C *__restrict__ vinf, typename Types<P>::V *__restrict__ b,
    typename Types<P>::R *__restrict__ r, typename Types<P>::R *__restrict__ m,
    const Scalars *__restrict__ sc, const int32_t *__restrict__ seq_par,
    typename Types<P>::V *__restrict__ x, typename Types<P>::R *__restrict__ s, Kids<P> kd,
    RangeBlock dr)
{
    using R = typename Types<P>::R;
    using C = typename Types<P>::C;
    const RangeBlock rb = block_range<CFR_SWEEP_XCD_UP>(tab, dr);
    const int32_t j = rb.lo + (int32_t)threadIdx.x;
    if (j >= rb.hi) return;
    const Scalars *gs = sc + rb.slot;
    C dpos = 1, dneg = 1;
    if (VAR == CFR_DCFR) {
        dpos = (C)gs->dpos;
        dneg = (C)gs->dneg;
    }
    auto level = [&](auto sl) {
        constexpr int SL = decltype(sl)::value;
        if (KIND == 1)
            up_infoset_fast<P, VAR, kFastKids, SL>(j, inf_first, child_ptr, child_idx, g, usign,
                                                   vinf, b, r, m, dpos, dneg, kd);
        else if (KIND == 2)
            up_infoset_fast<P, VAR, 0, SL & kSlotsWrite>(j, inf_first, child_ptr, child_idx, g,
                                                         usign, vinf, b, r, m, dpos, dneg, kd);
        else
            up_infoset<P, VAR, SL>(j, inf_first, child_ptr, child_idx, g, usign, vinf, b, r, m,
                                   dpos, dneg, kd);
    };
    // the flags are the same for the whole block (one scalar branch); the
    // level under the empty sequence never writes slots
    switch (ROOT ? rb.aux & kSlotsRead : rb.aux) {
    case 0: level(std::integral_constant<int, 0>()); break;
    case kSlotsWrite: level(std::integral_constant<int, kSlotsWrite>()); break;
    case kSlotsRead: level(std::integral_constant<int, kSlotsRead>()); break;
    default: level(std::integral_constant<int, kSlotsWrite | kSlotsRead>()); break;
    }
    if (ROOT) down_infoset<P>(j, inf_first, seq_par, b, x, s, (R)gs->w, 1, true);
}

// Two adjacent levels of ObserveUtility in one launch (one game's levels U
// and U+1, every decision point of U with at most kFastActs actions and at
// most kPairKids decision points below them, level U+1 on the fast path).
// A group of kPairKids lanes, four groups to a wave, owns one decision point
// j of level U: lane i takes the i-th decision point below j (its actions'
// child lists one after another, ascending) and runs its ObserveUtility,
// regret update and regret matching exactly as level U+1's own launch
// would, keeping its value in a register instead of storing it.  The group
// then reads its lanes' values across lanes in ascending order, and every
// lane of the group computes j: each action's own utility plus the values
// below it added in that order, the value, the regret update and regret
// matching; the group's first lane stores.  The sums and their order are
// those of two separate launches, so every result is bit for bit the same;
// the launch between the two levels is gone.  Control flow is uniform over
// a group, so every lane a cross-lane read takes from is active.
constexpr int kPairGroups = kThreads / kPairKids;  // decision points of level U per block
static_assert(64 % kPairKids == 0, "a group lies inside one wave");

template <int P, int VAR, int NC, int SLC, int SLU, bool ROOT>
__global__ __launch_bounds__(kThreads) void k_up_pair(
    const int32_t *__restrict__ inf_first, const int32_t *__restrict__ child_ptr,
    const int32_t *__restrict__ child_idx, const typename Types<P>::V *__restrict__ g,
    typename Types<P>::C usign, typename Types<P>::C *__restrict__ vinf,
    typename Types<P>::V *__restrict__ b, typename Types<P>::R *__restrict__ r,
    typename Types<P>::R *__restrict__ m, const Scalars *__restrict__ sc,
    const int32_t *__restrict__ seq_par, typename Types<P>::V *__restrict__ x,
    typename Types<P>::R *__restrict__ s, Kids<P> kd, RangeBlock dr)
{
    using V = typename Types<P>::V;
    using R = typename Types<P>::R;
    using C = typename Types<P>::C;
    constexpr int NA = kFastActs;
    constexpr bool kPred = VAR == CFR_PCFR_PLUS || VAR == CFR_PCFR;
    const int lane = (int)(threadIdx.x % kPairKids);
    const int first_lane = (int)(threadIdx.x % 64) - lane;
    const int32_t j = dr.lo + (int32_t)(blockIdx.x * kPairGroups + threadIdx.x / kPairKids);
    if (j >= dr.hi) return;  // a whole group
    const Scalars *gs = sc + dr.slot;
    C dpos = 1, dneg = 1;
    if (VAR == CFR_DCFR) {
        dpos = (C)gs->dpos;
        dneg = (C)gs->dneg;
    }
    const int32_t a0 = inf_first[j], a1 = inf_first[j + 1];
    const int32_t n = a1 - a0;
    // child list bounds of j's actions (kb[k] .. kb[k+1]: action k's)
    int32_t kb[NA + 1];
#pragma unroll
    for (int k = 0; k <= NA; ++k) kb[k] = child_ptr[a0 + (k < n ? k : n)];
    const int32_t cp0 = kb[0], nk = kb[NA] - cp0;
    // level U+1: this lane's decision point
    C vc = 0;
    if (lane < nk)
        vc = up_infoset_fast<P, VAR, NC, SLC, false>(child_idx[cp0 + lane], inf_first, child_ptr,
                                                     child_idx, g, usign, vinf, b, r, m, dpos,
                                                     dneg, kd);
    // level U: decision point j, in every lane of the group
    V gv[NA], bv[NA];
    R rv[NA], mv[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int32_t a = a0 + (k < n ? k : 0);
        gv[k] = g[a];
        bv[k] = b[a];
        rv[k] = r[a];
        if (kPred) mv[k] = m[a];
    }
    C q[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) q[k] = usign * (C)gv[k];
#pragma unroll
    for (int i = 0; i < kPairKids; ++i) {
        const C v = __shfl(vc, first_lane + i, 64);
#pragma unroll
        for (int k = 0; k < NA; ++k)
            if (k < n && cp0 + i >= kb[k] && cp0 + i < kb[k + 1]) q[k] = q[k] + v;
    }
    C V_ = 0;
#pragma unroll
    for (int k = 0; k < NA; ++k)
        if (k < n) V_ = V_ + (C)bv[k] * q[k];
    if (lane != 0) return;
    store_value(kd, (SLU & kSlotsWrite) ? kd.cslot[j] : -1, j, vinf, V_);
    C z[NA];
    C Z = 0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        if (k < n) {
            const int32_t a = a0 + k;
            C inst = q[k] - V_;
            C rr = post_step<P, VAR>((C)rv[k] + inst, dpos, dneg);
            r[a] = (R)rr;
            C zz = (C)(R)rr;
            if (kPred) {
                m[a] = (R)inst;
                zz = zz + (C)(R)inst;
            }
            zz = zz > 0 ? zz : 0;
            z[k] = zz;
            Z = Z + zz;
        }
    }
#pragma unroll
    for (int k = 0; k < NA; ++k)
        if (k < n) b[a0 + k] = (V)(Z > 0 ? z[k] / Z : (C)1 / (C)n);
    if (ROOT) down_infoset<P>(j, inf_first, seq_par, b, x, s, (R)gs->w, 1, true);
}

// The shallow levels of one player in one launch: block `root` owns the
// subtree below root decision point `root` (subtrees are disjoint and the
// sweeps never cross them).  It runs ObserveUtility on levels
// top_levels-1 .. 0 of its subtree, then the top-down pass on levels
// 0 .. top_levels-1, with a block barrier between levels.  The decision
// points of level l under root r are top_list[top_off[l*(n_roots+1) + r] ..
// top_off[l*(n_roots+1) + r + 1]).
template <int P, int VAR>
__global__ __launch_bounds__(kTopThreads) void k_top(
    int32_t top_levels, int32_t n_roots, const int32_t *__restrict__ top_off,
    const int32_t *__restrict__ top_list, const int32_t *__restrict__ inf_first,
    const int32_t *__restrict__ child_ptr, const int32_t *__restrict__ child_idx,
    const int32_t *__restrict__ seq_par, const typename Types<P>::V *__restrict__ g,
    typename Types<P>::C usign, typename Types<P>::C *__restrict__ vinf,
    typename Types<P>::V *__restrict__ b, typename Types<P>::R *__restrict__ r,
    typename Types<P>::R *__restrict__ m, typename Types<P>::V *__restrict__ x,
    typename Types<P>::R *__restrict__ s, const Scalars *__restrict__ sc, int average,
    int all_fast, Kids<P> kd)
{
    using R = typename Types<P>::R;
    using C = typename Types<P>::C;
    const int32_t root = (int32_t)blockIdx.x;
    C dpos = 1, dneg = 1;
    if (VAR == CFR_DCFR) {
        dpos = (C)sc->dpos;
        dneg = (C)sc->dneg;
    }
    const R w = average ? (R)sc->w : (R)0;
    for (int lv = top_levels - 1; lv >= 0; --lv) {
        const int32_t *off = top_off + (size_t)lv * (n_roots + 1);
        for (int32_t i = off[root] + (int32_t)threadIdx.x; i < off[root + 1]; i += kTopThreads) {
            if (all_fast)
                up_infoset_fast<P, VAR, kFastKids, 0>(top_list[i], inf_first, child_ptr,
                                                      child_idx, g, usign, vinf, b, r, m, dpos,
                                                      dneg, kd);
            else
                up_infoset<P, VAR, 0>(top_list[i], inf_first, child_ptr, child_idx, g, usign,
                                      vinf, b, r, m, dpos, dneg, kd);
        }
        __syncthreads();
    }
    for (int lv = 0; lv < top_levels; ++lv) {
        const int32_t *off = top_off + (size_t)lv * (n_roots + 1);
        for (int32_t i = off[root] + (int32_t)threadIdx.x; i < off[root + 1]; i += kTopThreads)
            down_infoset<P>(top_list[i], inf_first, seq_par, b, x, s, w, average);
        __syncthreads();
    }
}

// The shallow levels of a game iterating alone in one block: the values of each level's
// decision points stay in LDS, where the level above reads them through its
// child lists, so consecutive levels are separated by a block barrier
// instead of a kernel boundary and a round trip through global memory.  The
// deepest of these levels reads its children's values (written by the
// launch of the level below) from their value slots, as its own launch
// would.  Each thread owns one decision point of the shallow levels (at
// most kShallowThreads in all) and issues all of its loads before any level
// is computed, so every level's dependent load rounds overlap those of the
// levels below it; the levels are then computed deepest first, each from
// registers and LDS.  Every decision point runs the fast path of
// ObserveUtility with the same operations in the same order as in a launch
// per level, so every result is the same bit for bit.  Only LDS is shared
// between threads here (the global stores are each thread's own decision
// point's regrets and strategies).
template <int P, int VAR>
__global__ __launch_bounds__(kShallowThreads) void k_shallow(
    ShallowPlan sp, const int32_t *__restrict__ inf_first, const int32_t *__restrict__ child_ptr,
    const int32_t *__restrict__ child_idx, const typename Types<P>::V *__restrict__ g,
    typename Types<P>::C usign, typename Types<P>::V *__restrict__ b,
    typename Types<P>::R *__restrict__ r, typename Types<P>::R *__restrict__ m,
    const Scalars *__restrict__ sc, const int32_t *__restrict__ seq_par,
    typename Types<P>::V *__restrict__ x, typename Types<P>::R *__restrict__ s, Kids<P> kd)
{
    using R = typename Types<P>::R;
    using C = typename Types<P>::C;
    __shared__ C lv[kShallowMax];
    const int32_t base = sp.lo[0];
    C *const lvb = lv - base;  // lvb[j]: value of shallow decision point j
    C dpos = 1, dneg = 1;
    if (VAR == CFR_DCFR) {
        dpos = (C)sc->dpos;
        dneg = (C)sc->dneg;
    }
    const R w = (R)sc->w;
    const int32_t j = base + (int32_t)threadIdx.x;
    const bool own = j < sp.lo[sp.levels];
    int lvl = 0;
    for (int l = 1; l < sp.levels; ++l)
        if (j >= sp.lo[l]) lvl = l;
    // the deepest level reads slots unless it has no decision points below
    // it (then every child count is zero and the child loads are unused)
    const bool slots = lvl == sp.levels - 1 && sp.kind[lvl] != 2;
    FastLoads<P, kFastKids> L;
    if (own) {
        if (slots)
            fast_load<P, VAR, kFastKids, kSlotsRead>(j, inf_first, child_ptr, child_idx, g, b, r,
                                                     m, kd, L);
        else
            fast_load<P, VAR, kFastKids, 0>(j, inf_first, child_ptr, child_idx, g, b, r, m, kd,
                                            L);
    }
    for (int l = sp.levels - 1; l >= 0; --l) {
        if (own && lvl == l) {
            if (l < sp.levels - 1) {
                // only the children that exist: the clamped ids of the
                // others need not be in this block's LDS (the value of a
                // missing child is never added)
#pragma unroll
                for (int k = 0; k < kFastActs; ++k)
#pragma unroll
                    for (int i = 0; i < kFastKids; ++i)
                        L.cv[k][i] = i < L.cnt[k] ? lvb[L.cid[k][i]] : (C)0;
            }
            lvb[j] = fast_apply<P, VAR, kFastKids>(L, usign, b, r, m, dpos, dneg);
            if (l == 0) down_infoset<P>(j, inf_first, seq_par, b, x, s, w, 1, true);
        }
        __syncthreads();
    }
}

// Levels lo .. lo+D-1 of a game iterating alone (below its shallow levels) in one
// launch.  Block b takes the decision points fuse_list[off[l] .. off[l+1])
// of level lo+l (off = fuse_off + b*(D+1)): whole subtrees below some of
// level lo's decision points, so every child a block's decision point reads
// is the block's own or below the fused levels.  Each thread owns one of
// them and issues all of its loads before any level is computed (the
// deepest level also its children's values: from value slots, or by child
// id from vinf, both written by the launch of the level below).  The levels
// are then computed deepest first; each stores its values in vinf and a
// block barrier passes them to the level above, except the shallowest,
// which stores them where its parents' level reads them (slot or vinf), or,
// when it is level 0, also does its top-down step, as level 0's own launch
// would (ROOT: the fused levels start at level 0).  The arithmetic is that
// of a launch per level, bit for bit.
template <int P, int VAR, bool ROOT>
__global__ __launch_bounds__(kFuseThreads) void k_fuse(
    FusePlan fp, const int32_t *__restrict__ fuse_off, const int32_t *__restrict__ fuse_list,
    const int32_t *__restrict__ inf_first, const int32_t *__restrict__ child_ptr,
    const int32_t *__restrict__ child_idx, const typename Types<P>::V *__restrict__ g,
    typename Types<P>::C usign, typename Types<P>::C *vinf, typename Types<P>::V *__restrict__ b,
    typename Types<P>::R *__restrict__ r, typename Types<P>::R *__restrict__ m,
    const Scalars *__restrict__ sc, const int32_t *__restrict__ seq_par,
    typename Types<P>::V *__restrict__ x, typename Types<P>::R *__restrict__ s, Kids<P> kd)
{
    using R = typename Types<P>::R;
    using C = typename Types<P>::C;
    const int D = fp.levels;
    const int32_t *off = fuse_off + (size_t)blockIdx.x * (size_t)(D + 1);
    C dpos = 1, dneg = 1;
    if (VAR == CFR_DCFR) {
        dpos = (C)sc->dpos;
        dneg = (C)sc->dneg;
    }
    const int32_t pos = off[0] + (int32_t)threadIdx.x;
    const bool own = pos < off[D];
    int lvl = 0;
    for (int l = 1; l < D; ++l)
        if (pos >= off[l]) lvl = l;
    const bool deepest = lvl == D - 1;
    FastLoads<P, kFastKids> L;
    int32_t j = 0, cs = -1;
    if (own) {
        j = fp.base + fuse_list[pos];
        if (deepest && fp.deep_read == 1)
            fast_load<P, VAR, kFastKids, kSlotsRead>(j, inf_first, child_ptr, child_idx, g, b, r,
                                                     m, kd, L);
        else
            fast_load<P, VAR, kFastKids, 0>(j, inf_first, child_ptr, child_idx, g, b, r, m, kd,
                                            L);
        if (deepest && fp.deep_read == 2) {
#pragma unroll
            for (int k = 0; k < kFastActs; ++k)
#pragma unroll
                for (int i = 0; i < kFastKids; ++i) L.cv[k][i] = vinf[L.cid[k][i]];
        }
        if (lvl == 0 && fp.top_slots) cs = kd.cslot[j];
    }
    for (int l = D - 1; l >= 0; --l) {
        if (own && lvl == l) {
            if (l < D - 1) {
                // the values the level below stored before the barrier
#pragma unroll
                for (int k = 0; k < kFastActs; ++k)
#pragma unroll
                    for (int i = 0; i < kFastKids; ++i) L.cv[k][i] = vinf[L.cid[k][i]];
            }
            const C V = fast_apply<P, VAR, kFastKids>(L, usign, b, r, m, dpos, dneg);
            store_value(kd, l == 0 ? cs : -1, j, vinf, V);
            if (ROOT && l == 0)
                down_infoset<P>(j, inf_first, seq_par, b, x, s, (R)sc->w, 1, true);
        }
        if (l > 0) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// NextStrategy top-down pass for one level, fused with averaging
// ---------------------------------------------------------------------------

template <int P>
__global__ __launch_bounds__(kThreads) void k_down(const RangeBlock *__restrict__ tab,
                                                   const int32_t *__restrict__ seq_par,
                                                   const typename Types<P>::V *__restrict__ b,
                                                   typename Types<P>::V *__restrict__ x,
                                                   typename Types<P>::R *__restrict__ s,
                                                   const Scalars *__restrict__ sc, int average)
{
    using R = typename Types<P>::R;
    const RangeBlock rb = tab[blockIdx.x];
    const int32_t i = rb.lo + (int32_t)threadIdx.x;
    if (i >= rb.hi) return;
    if (average) {
        R w = (R)sc[rb.slot].w;
        s[i] = s[i] + w * (R)x[i];
    }
    x[i] = x[seq_par[i]] * b[i];
}

// The whole top-down pass below level 0 in one launch: each sequence walks
// its parent chain up to the game's empty sequence (aux), collecting the
// behavioural strategies on the way, then multiplies them from the root
// down: x = ((1 * b_0) * b_1) ... * b_own, the same products in the same
// order as the level-by-level pass, so the result is bit for bit the same.
// It reads only b and the parent links, which the bottom-up pass has
// finished, never another thread's x.  MAXD bounds the chain length.
// With FOLD (one game, range from its empty sequence on) the launch also
// writes the copy in first-touch order that the next product reads,
// xp[pos[i]] = x[i], so no gather launch is needed; the sequences below
// avg_lo (the empty sequence and level 0's, whose x the bottom-up pass
// already wrote: the chain gives the same products) are rewritten with the
// same values and not averaged again.
template <int P, int MAXD, bool FOLD>
__global__ __launch_bounds__(kThreads) void k_down_all(const RangeBlock *__restrict__ tab,
                                                       const int32_t *__restrict__ seq_par,
                                                       const typename Types<P>::V *__restrict__ b,
                                                       typename Types<P>::V *__restrict__ x,
                                                       typename Types<P>::R *__restrict__ s,
                                                       const Scalars *__restrict__ sc, int average,
                                                       RangeBlock dr, const int32_t *__restrict__ pos,
                                                       typename Types<P>::V *__restrict__ xp,
                                                       int32_t avg_lo)
{
    using V = typename Types<P>::V;
    using R = typename Types<P>::R;
    const RangeBlock rb = block_range<CFR_SWEEP_XCD_DOWN>(tab, dr);
    const int32_t i = rb.lo + (int32_t)threadIdx.x;
    if (i >= rb.hi) return;
    const int32_t root = rb.aux;
    V chain[MAXD];
    int d = 0;
    int32_t q = i;
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
        if (q != root) {
            chain[k] = b[q];
            q = seq_par[q];
            d = k + 1;
        }
    }
    V xv = (V)1;
#pragma unroll
    for (int k = MAXD - 1; k >= 0; --k)
        if (k < d) xv = xv * chain[k];
    if (average && (!FOLD || i >= avg_lo)) {
        R w = (R)sc[rb.slot].w;
        s[i] = s[i] + w * (R)x[i];
    }
    x[i] = xv;
    if (FOLD) xp[pos[i]] = xv;
}

// ---------------------------------------------------------------------------
// Evaluation: average normalisation, best-response sweep, reductions
// ---------------------------------------------------------------------------

// xbar = s / W of the sequence's game, 1 at the game's empty sequence (the
// table's aux); the current strategy for a game with no iteration yet.
template <int P>
__global__ __launch_bounds__(kThreads) void k_normalize(const RangeBlock *__restrict__ tab,
                                                        const typename Types<P>::R *s,
                                                        const typename Types<P>::V *x,
                                                        const Scalars *__restrict__ sc,
                                                        typename Types<P>::V *__restrict__ xbar)
{
    using V = typename Types<P>::V;
    const RangeBlock rb = tab[blockIdx.x];
    const int32_t i = rb.lo + (int32_t)threadIdx.x;
    if (i >= rb.hi) return;
    const double W = sc[rb.slot].W;
    xbar[i] = i == rb.aux ? (V)1 : W > 0 ? (V)((double)s[i] / W) : x[i];
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_br(const RangeBlock *__restrict__ tab,
                                                 const int32_t *__restrict__ inf_first,
                                                 const int32_t *__restrict__ child_ptr,
                                                 const int32_t *__restrict__ child_idx,
                                                 const typename Types<P>::V *__restrict__ g,
                                                 typename Types<P>::C usign,
                                                 typename Types<P>::C *__restrict__ vmax)
{
    using C = typename Types<P>::C;
    const RangeBlock rb = tab[blockIdx.x];
    const int32_t j = rb.lo + (int32_t)threadIdx.x;
    if (j >= rb.hi) return;
    const int32_t a0 = inf_first[j], a1 = inf_first[j + 1];
    C best = 0;
    for (int32_t a = a0; a < a1; ++a) {
        const C acc =
            child_sum<P>(usign * (C)g[a], child_ptr[a], child_ptr[a + 1], child_idx, vmax);
        if (a == a0 || acc > best) best = acc;
    }
    vmax[j] = best;
}

// value at each game's empty sequence: own utility there plus the values of
// the decision points directly below it, summed in ascending order
template <int P>
__global__ __launch_bounds__(kThreads) void k_root(int32_t n_tab, const SlotRef *__restrict__ tab,
                                                   const typename Types<P>::V *__restrict__ g,
                                                   typename Types<P>::C usign,
                                                   const typename Types<P>::C *__restrict__ v,
                                                   Scalars *sc, int out_index)
{
    using C = typename Types<P>::C;
    const int32_t k = (int32_t)(blockIdx.x * kThreads + threadIdx.x);
    if (k >= n_tab) return;
    const SlotRef e = tab[k];
    double acc = (double)(usign * (C)g[e.root]);
    for (int32_t j = e.a; j < e.b; ++j) acc = acc + (double)v[j];
    sc[e.slot].out[out_index] = acc;
}

// deterministic two-stage dot product in double: one partial per table
// entry (a fixed tree over its at most kThreads terms), then one block per
// game adding its partials in a fixed order
template <int P>
__global__ __launch_bounds__(kThreads) void k_dot_partial(const RangeBlock *__restrict__ tab,
                                                          const typename Types<P>::V *__restrict__ a,
                                                          const typename Types<P>::V *__restrict__ b,
                                                          double *partials)
{
    __shared__ double red[kThreads];
    const RangeBlock rb = tab[blockIdx.x];
    const int32_t i = rb.lo + (int32_t)threadIdx.x;
    red[threadIdx.x] = i < rb.hi ? (double)a[i] * (double)b[i] : 0.0;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void k_dot_final(const SlotRef *__restrict__ fin,
                                                        const double *partials, Scalars *sc,
                                                        int out_index)
{
    __shared__ double red[kThreads];
    const SlotRef e = fin[blockIdx.x];
    double acc = 0;
    for (int32_t i = e.a + (int32_t)threadIdx.x; i < e.b; i += kThreads) acc = acc + partials[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sc[e.slot].out[out_index] = red[0];
}

__global__ __launch_bounds__(kThreads) void k_add_offset(int32_t *a, int64_t n, int32_t base)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) a[i] += base;
}

__global__ __launch_bounds__(kThreads) void k_add_offset_nonneg(int32_t *a, int64_t n,
                                                                int32_t base)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n && a[i] >= 0) a[i] += base;
}

// The permuted copy of a strategy vector that a product gathers from.
template <int P>
__global__ __launch_bounds__(kThreads) void k_gather(const RangeBlock *__restrict__ tab,
                                                     const int32_t *__restrict__ perm,
                                                     const typename Types<P>::V *__restrict__ src,
                                                     typename Types<P>::V *__restrict__ dst)
{
    const RangeBlock rb = tab[blockIdx.x];
    const int32_t i = rb.lo + (int32_t)threadIdx.x;
    if (i >= rb.hi) return;
    dst[i] = src[perm[i]];
}

__global__ __launch_bounds__(kThreads) void k_remap(int32_t *a, int64_t n,
                                                    const int32_t *__restrict__ map)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) a[i] = map[a[i]];
}

// ---------------------------------------------------------------------------
// Quad stream construction (stream form 3)
// ---------------------------------------------------------------------------

// A row's quads: maximal runs of consecutive nonzeros (in row order) whose
// columns increase and share one aligned group of four.  One wave per row
// (four rows per block): the wave reads 64 consecutive nonzeros at a time,
// each lane decides whether its nonzero starts a quad (the previous one is
// in another group, does not precede it, or belongs to another row), and
// the quads are counted and ranked with ballots.
constexpr int kQuadRowsPerBlock = kThreads / 64;

__device__ __forceinline__ bool starts_quad(int32_t col, int32_t prev, bool first)
{
    return first || (col >> 2) != (prev >> 2) || col <= prev;
}

__global__ __launch_bounds__(kThreads) void k_quad_count(const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ idx,
                                                         int64_t nb, int32_t row0, int32_t nr,
                                                         int32_t *__restrict__ cnt)
{
    const int lane = (int)(threadIdx.x & 63);
    const int32_t r = (int32_t)(blockIdx.x * kQuadRowsPerBlock + (threadIdx.x >> 6));
    if (r >= nr) return;  // the whole wave
    const int32_t a = ptr[row0 + r], z = ptr[row0 + r + 1];
    int32_t c = 0;
    for (int32_t base = a; base < z; base += 64) {
        const int32_t e = base + lane;
        bool st = false;
        if (e < z) {
            const int32_t col = idx[nb + e];
            const int32_t prev = e > a ? idx[nb + e - 1] : -1;
            st = starts_quad(col, prev, e == a);
        }
        c += __popcll(__ballot(st));
    }
    if (lane == 0) cnt[r] = c;
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_quad_fill(
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
    const typename Types<P>::V *__restrict__ val, int64_t nb, int32_t row0, int32_t nr,
    const int32_t *__restrict__ qptr, int64_t qb, uint32_t *__restrict__ qidx,
    typename Types<P>::V *__restrict__ qval)
{
    using V = typename Types<P>::V;
    const int lane = (int)(threadIdx.x & 63);
    const int32_t r = (int32_t)(blockIdx.x * kQuadRowsPerBlock + (threadIdx.x >> 6));
    if (r >= nr) return;  // the whole wave
    const int32_t a = ptr[row0 + r], z = ptr[row0 + r + 1];
    int64_t q0 = qb + qptr[row0 + r];  // first quad of this pass
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int32_t base = a; base < z; base += 64) {
        const int32_t e = base + lane;
        bool st = false;
        int32_t col = 0;
        if (e < z) {
            col = idx[nb + e];
            const int32_t prev = e > a ? idx[nb + e - 1] : -1;
            st = starts_quad(col, prev, e == a);
        }
        const uint64_t ball = __ballot(st);
        if (st) {
            // this quad: the nonzeros from e while none starts a new one
            const int64_t q = q0 + __popcll(ball & below);
            V v[4] = {0, 0, 0, 0};
            uint32_t mask = 1u << (col & 3);
            v[col & 3] = val[nb + e];
            int32_t prev = col;
            for (int k = 1; k < 4 && e + k < z; ++k) {
                const int32_t c2 = idx[nb + e + k];
                if (starts_quad(c2, prev, false)) break;
                mask |= 1u << (c2 & 3);
                v[c2 & 3] = val[nb + e + k];
                prev = c2;
            }
            qidx[q] = (uint32_t)(col >> 2) | (mask << kQuadMaskShift);
#pragma unroll
            for (int k = 0; k < 4; ++k) qval[4 * q + k] = v[k];
        }
        q0 += __popcll(ball);
    }
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------

template <int P>
Kids<P> kids(const DevPlayer &p)
{
    return Kids<P>{p.cslot, p.ccount, (typename Types<P>::C *)p.cval};
}

template <int P, bool SEQ, int ITEMS, int VEC>
hipError_t spmv_launch(const SpmvBlock *tab, int32_t n_tab, const int32_t *ptr, const int32_t *idx,
                       const void *val, const void *xin, void *yout, int xcd_remap, int begin,
                       Scalars *sc, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    using V = typename Types<P>::V;
    unsigned grid = xcd_remap ? (unsigned)(((n_tab + 7) / 8) * 8) : (unsigned)n_tab;
    // With events, the launch itself sets them to the kernel's start and end
    // (what a profiler's kernel trace reads), not the stream's progress
    // around it.
#define CFR_SPMV_GO(KERNEL)                                                                   \
    do {                                                                                      \
        if (ev0)                                                                              \
            hipExtLaunchKernelGGL(KERNEL, dim3(grid), dim3(kSpmvThreads), 0, st, ev0, ev1, 0u, \
                                  n_tab, tab, ptr, idx, (const V *)val, (const V *)xin,       \
                                  (V *)yout, xcd_remap, begin, sc);                           \
        else                                                                                  \
            hipLaunchKernelGGL(KERNEL, dim3(grid), dim3(kSpmvThreads), 0, st, n_tab, tab, ptr, \
                               idx, (const V *)val, (const V *)xin, (V *)yout, xcd_remap,     \
                               begin, sc);                                                    \
    } while (0)
    if constexpr (VEC == 3 && !SEQ && P != CFR_FP64)
        CFR_SPMV_GO((k_spmv_quads<P, ITEMS>));
    else
        CFR_SPMV_GO((k_spmv<P, SEQ, ITEMS, VEC>));
#undef CFR_SPMV_GO
    return hipGetLastError();
}

template <int P, bool SEQ, int VEC>
hipError_t spmv_items(int items, const SpmvBlock *tab, int32_t n_tab, const int32_t *ptr,
                      const int32_t *idx, const void *val, const void *xin, void *yout,
                      int xcd_remap, int begin, Scalars *sc, hipStream_t st, hipEvent_t ev0,
                      hipEvent_t ev1)
{
    switch (items) {
    case 4:
        return spmv_launch<P, SEQ, 4, VEC>(tab, n_tab, ptr, idx, val, xin, yout, xcd_remap, begin,
                                           sc, st, ev0, ev1);
    case 8:
        return spmv_launch<P, SEQ, 8, VEC>(tab, n_tab, ptr, idx, val, xin, yout, xcd_remap, begin,
                                           sc, st, ev0, ev1);
    case 16:
        return spmv_launch<P, SEQ, 16, VEC>(tab, n_tab, ptr, idx, val, xin, yout, xcd_remap, begin,
                                            sc, st, ev0, ev1);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
hipError_t spmv_t(int items, int vec, const SpmvBlock *tab, int32_t n_tab, const int32_t *ptr,
                  const int32_t *idx, const void *val, const void *xin, void *yout, int xcd_remap,
                  int sequential, int begin, Scalars *sc, hipStream_t st, hipEvent_t ev0,
                  hipEvent_t ev1)
{
    if (n_tab <= 0) {
        // nothing to launch: the events still mark this point of the stream
        if (ev0 && hipEventRecord(ev0, st) == hipSuccess) return hipEventRecord(ev1, st);
        return hipSuccess;
    }
#define CFR_SPMV_VEC(SQ)                                                                      \
    switch (vec) {                                                                            \
    case 0:                                                                                   \
        return spmv_items<P, SQ, 0>(items, tab, n_tab, ptr, idx, val, xin, yout, xcd_remap,   \
                                    begin, sc, st, ev0, ev1);                                 \
    case 1:                                                                                   \
        return spmv_items<P, SQ, 1>(items, tab, n_tab, ptr, idx, val, xin, yout, xcd_remap,   \
                                    begin, sc, st, ev0, ev1);                                 \
    case 2:                                                                                   \
        return spmv_items<P, SQ, 2>(items, tab, n_tab, ptr, idx, val, xin, yout, xcd_remap,   \
                                    begin, sc, st, ev0, ev1);                                 \
    case 3:                                                                                   \
        return spmv_items<P, SQ, 3>(items, tab, n_tab, ptr, idx, val, xin, yout, xcd_remap,   \
                                    begin, sc, st, ev0, ev1);                                 \
    default: return hipErrorInvalidValue;                                                     \
    }
    if (sequential) {
        CFR_SPMV_VEC(true)
    }
    CFR_SPMV_VEC(false)
#undef CFR_SPMV_VEC
}

// Blocks of a sweep launch: the table's entries, or those of the direct range.
inline unsigned sweep_grid(int32_t n_tab, const RangeBlock &dr)
{
    if (dr.hi > dr.lo) {
        const unsigned n = (unsigned)((dr.hi - dr.lo + kRangeBlock - 1) / kRangeBlock);
        return CFR_SWEEP_XCD_UP || CFR_SWEEP_XCD_DOWN ? (n + 7) / 8 * 8 : n;
    }
    return (unsigned)n_tab;
}

template <int P, int VAR, int KIND, bool ROOT>
hipError_t up_launch(const RangeBlock *tab, int32_t n_tab, const RangeBlock &dr,
                     const DevPlayer &p, double usign, const Scalars *sc, hipStream_t st)
{
    using T = Types<P>;
    hipLaunchKernelGGL((k_up<P, VAR, KIND, ROOT>), dim3(sweep_grid(n_tab, dr)), dim3(kThreads), 0,
                       st, tab, p.inf_first, p.child_ptr, p.child_idx, (const typename T::V *)p.g,
                       (typename T::C)usign, (typename T::C *)p.vinf, (typename T::V *)p.b,
                       (typename T::R *)p.r, (typename T::R *)p.m, sc, p.seq_par,
                       (typename T::V *)p.x, (typename T::R *)p.s, kids<P>(p), dr);
    return hipGetLastError();
}

template <int P, int VAR>
hipError_t up_t(int kind, int root, const RangeBlock *tab, int32_t n_tab, const RangeBlock &dr,
                const DevPlayer &p, double usign, const Scalars *sc, hipStream_t st)
{
    if (sweep_grid(n_tab, dr) == 0) return hipSuccess;
    if (root) {
        if (kind == 1) return up_launch<P, VAR, 1, true>(tab, n_tab, dr, p, usign, sc, st);
        if (kind == 2) return up_launch<P, VAR, 2, true>(tab, n_tab, dr, p, usign, sc, st);
        return up_launch<P, VAR, 0, true>(tab, n_tab, dr, p, usign, sc, st);
    }
    if (kind == 1) return up_launch<P, VAR, 1, false>(tab, n_tab, dr, p, usign, sc, st);
    if (kind == 2) return up_launch<P, VAR, 2, false>(tab, n_tab, dr, p, usign, sc, st);
    return up_launch<P, VAR, 0, false>(tab, n_tab, dr, p, usign, sc, st);
}

template <int P>
hipError_t up_dispatch(int variant, int kind, int root, const RangeBlock *tab, int32_t n_tab,
                       const RangeBlock &dr, const DevPlayer &p, double usign, const Scalars *sc,
                       hipStream_t st)
{
    switch (variant) {
    case CFR_VANILLA: return up_t<P, CFR_VANILLA>(kind, root, tab, n_tab, dr, p, usign, sc, st);
    case CFR_PLUS: return up_t<P, CFR_PLUS>(kind, root, tab, n_tab, dr, p, usign, sc, st);
    case CFR_DCFR: return up_t<P, CFR_DCFR>(kind, root, tab, n_tab, dr, p, usign, sc, st);
    case CFR_PCFR_PLUS:
        return up_t<P, CFR_PCFR_PLUS>(kind, root, tab, n_tab, dr, p, usign, sc, st);
    case CFR_PCFR: return up_t<P, CFR_PCFR>(kind, root, tab, n_tab, dr, p, usign, sc, st);
    default: return hipErrorInvalidValue;
    }
}

template <int P, int VAR, int NC, int SLC, int SLU, bool ROOT>
hipError_t pair_launch(const RangeBlock &dr, const DevPlayer &p, double usign, const Scalars *sc,
                       hipStream_t st)
{
    using T = Types<P>;
    const unsigned grid = (unsigned)((dr.hi - dr.lo + kPairGroups - 1) / kPairGroups);
    hipLaunchKernelGGL((k_up_pair<P, VAR, NC, SLC, SLU, ROOT>), dim3(grid), dim3(kThreads), 0, st,
                       p.inf_first, p.child_ptr, p.child_idx, (const typename T::V *)p.g,
                       (typename T::C)usign, (typename T::C *)p.vinf, (typename T::V *)p.b,
                       (typename T::R *)p.r, (typename T::R *)p.m, sc, p.seq_par,
                       (typename T::V *)p.x, (typename T::R *)p.s, kids<P>(p), dr);
    return hipGetLastError();
}

template <int P, int VAR, int NC>
hipError_t pair_flags(int child_reads_slots, int upper_writes_slots, int root,
                      const RangeBlock &dr, const DevPlayer &p, double usign, const Scalars *sc,
                      hipStream_t st)
{
    const int f = (child_reads_slots ? 1 : 0) | (upper_writes_slots && !root ? 2 : 0);
    if (root) {
        if (f & 1) return pair_launch<P, VAR, NC, kSlotsRead, 0, true>(dr, p, usign, sc, st);
        return pair_launch<P, VAR, NC, 0, 0, true>(dr, p, usign, sc, st);
    }
    switch (f) {
    case 0: return pair_launch<P, VAR, NC, 0, 0, false>(dr, p, usign, sc, st);
    case 1: return pair_launch<P, VAR, NC, kSlotsRead, 0, false>(dr, p, usign, sc, st);
    case 2: return pair_launch<P, VAR, NC, 0, kSlotsWrite, false>(dr, p, usign, sc, st);
    default: return pair_launch<P, VAR, NC, kSlotsRead, kSlotsWrite, false>(dr, p, usign, sc, st);
    }
}

template <int P, int VAR>
hipError_t pair_t(int child_kind, int child_reads_slots, int upper_writes_slots, int root,
                  const RangeBlock &dr, const DevPlayer &p, double usign, const Scalars *sc,
                  hipStream_t st)
{
    if (dr.hi <= dr.lo) return hipSuccess;
    // NC = 0 only for a lower level with nothing below it, whose decision
    // points read no child values (so no slot flag applies)
    if (child_kind == 2)
        return pair_flags<P, VAR, 0>(0, upper_writes_slots, root, dr, p, usign, sc, st);
    return pair_flags<P, VAR, kFastKids>(child_reads_slots, upper_writes_slots, root, dr, p, usign,
                                         sc, st);
}

template <int P>
hipError_t pair_dispatch(int variant, int child_kind, int child_reads_slots,
                         int upper_writes_slots, int root, const RangeBlock &dr,
                         const DevPlayer &p, double usign, const Scalars *sc, hipStream_t st)
{
#define CFR_PAIR_ARGS child_kind, child_reads_slots, upper_writes_slots, root, dr, p, usign, sc, st
    switch (variant) {
    case CFR_VANILLA: return pair_t<P, CFR_VANILLA>(CFR_PAIR_ARGS);
    case CFR_PLUS: return pair_t<P, CFR_PLUS>(CFR_PAIR_ARGS);
    case CFR_DCFR: return pair_t<P, CFR_DCFR>(CFR_PAIR_ARGS);
    case CFR_PCFR_PLUS: return pair_t<P, CFR_PCFR_PLUS>(CFR_PAIR_ARGS);
    case CFR_PCFR: return pair_t<P, CFR_PCFR>(CFR_PAIR_ARGS);
    default: return hipErrorInvalidValue;
    }
#undef CFR_PAIR_ARGS
}

template <int P, int VAR>
hipError_t top_t(const DevPlayer &p, double usign, int average, const Scalars *sc, hipStream_t st)
{
    using T = Types<P>;
    if (p.top_levels == 0 || p.n_roots == 0) return hipSuccess;
    hipLaunchKernelGGL((k_top<P, VAR>), dim3(p.n_roots), dim3(kTopThreads), 0, st, p.top_levels,
                       p.n_roots, p.top_off, p.top_list, p.inf_first, p.child_ptr, p.child_idx,
                       p.seq_par, (const typename T::V *)p.g, (typename T::C)usign,
                       (typename T::C *)p.vinf, (typename T::V *)p.b, (typename T::R *)p.r,
                       (typename T::R *)p.m, (typename T::V *)p.x, (typename T::R *)p.s, sc,
                       average, p.top_fast, kids<P>(p));
    return hipGetLastError();
}

template <int P, int VAR>
hipError_t shallow_t(const DevPlayer &p, double usign, const Scalars *sc, hipStream_t st)
{
    using T = Types<P>;
    if (p.shallow.levels <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_shallow<P, VAR>), dim3(1), dim3(kShallowThreads), 0, st, p.shallow,
                       p.inf_first, p.child_ptr, p.child_idx, (const typename T::V *)p.g,
                       (typename T::C)usign, (typename T::V *)p.b, (typename T::R *)p.r,
                       (typename T::R *)p.m, sc, p.seq_par, (typename T::V *)p.x,
                       (typename T::R *)p.s, kids<P>(p));
    return hipGetLastError();
}

template <int P, int VAR>
hipError_t fuse_t(const DevPlayer &p, double usign, const Scalars *sc, hipStream_t st)
{
    using T = Types<P>;
    if (p.fuse.levels < 2 || p.fuse.blocks <= 0) return hipSuccess;
    auto kern = p.fuse.lo == 0 ? k_fuse<P, VAR, true> : k_fuse<P, VAR, false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)p.fuse.blocks), dim3(kFuseThreads), 0, st, p.fuse,
                       p.fuse_off, p.fuse_list, p.inf_first, p.child_ptr, p.child_idx,
                       (const typename T::V *)p.g, (typename T::C)usign, (typename T::C *)p.vinf,
                       (typename T::V *)p.b, (typename T::R *)p.r, (typename T::R *)p.m, sc,
                       p.seq_par, (typename T::V *)p.x, (typename T::R *)p.s, kids<P>(p));
    return hipGetLastError();
}

template <int P>
hipError_t fuse_dispatch(int variant, const DevPlayer &p, double usign, const Scalars *sc,
                         hipStream_t st)
{
    switch (variant) {
    case CFR_VANILLA: return fuse_t<P, CFR_VANILLA>(p, usign, sc, st);
    case CFR_PLUS: return fuse_t<P, CFR_PLUS>(p, usign, sc, st);
    case CFR_DCFR: return fuse_t<P, CFR_DCFR>(p, usign, sc, st);
    case CFR_PCFR_PLUS: return fuse_t<P, CFR_PCFR_PLUS>(p, usign, sc, st);
    case CFR_PCFR: return fuse_t<P, CFR_PCFR>(p, usign, sc, st);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
hipError_t shallow_dispatch(int variant, const DevPlayer &p, double usign, const Scalars *sc,
                            hipStream_t st)
{
    switch (variant) {
    case CFR_VANILLA: return shallow_t<P, CFR_VANILLA>(p, usign, sc, st);
    case CFR_PLUS: return shallow_t<P, CFR_PLUS>(p, usign, sc, st);
    case CFR_DCFR: return shallow_t<P, CFR_DCFR>(p, usign, sc, st);
    case CFR_PCFR_PLUS: return shallow_t<P, CFR_PCFR_PLUS>(p, usign, sc, st);
    case CFR_PCFR: return shallow_t<P, CFR_PCFR>(p, usign, sc, st);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
hipError_t top_dispatch(int variant, const DevPlayer &p, double usign, int average,
                        const Scalars *sc, hipStream_t st)
{
    switch (variant) {
    case CFR_VANILLA: return top_t<P, CFR_VANILLA>(p, usign, average, sc, st);
    case CFR_PLUS: return top_t<P, CFR_PLUS>(p, usign, average, sc, st);
    case CFR_DCFR: return top_t<P, CFR_DCFR>(p, usign, average, sc, st);
    case CFR_PCFR_PLUS: return top_t<P, CFR_PCFR_PLUS>(p, usign, average, sc, st);
    case CFR_PCFR: return top_t<P, CFR_PCFR>(p, usign, average, sc, st);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
hipError_t down_t(const RangeBlock *tab, int32_t n_tab, const DevPlayer &p, int average,
                  const Scalars *sc, hipStream_t st)
{
    using T = Types<P>;
    if (n_tab <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_down<P>), dim3((unsigned)n_tab), dim3(kThreads), 0, st, tab, p.seq_par,
                       (const typename T::V *)p.b, (typename T::V *)p.x, (typename T::R *)p.s, sc,
                       average);
    return hipGetLastError();
}

template <int P, int MAXD, bool FOLD>
void down_all_launch(unsigned grid, const RangeBlock *tab, const RangeBlock &dr, const DevPlayer &p,
                     int average, const Scalars *sc, int32_t avg_lo, hipStream_t st)
{
    using T = Types<P>;
    hipLaunchKernelGGL((k_down_all<P, MAXD, FOLD>), dim3(grid), dim3(kThreads), 0, st, tab,
                       p.seq_par, (const typename T::V *)p.b, (typename T::V *)p.x,
                       (typename T::R *)p.s, sc, average, dr, FOLD ? p.pos : nullptr,
                       FOLD ? (typename T::V *)p.xp : nullptr, avg_lo);
}

template <int P>
hipError_t down_all_t(int maxd, const RangeBlock *tab, int32_t n_tab, const RangeBlock &dr,
                      const DevPlayer &p, int average, const Scalars *sc, int fold,
                      int32_t avg_lo, hipStream_t st)
{
    const unsigned grid = sweep_grid(n_tab, dr);
    if (grid == 0) return hipSuccess;
    // the fold needs one game's direct range, from its empty sequence on
    if (fold && (dr.hi <= dr.lo || dr.lo != dr.aux || avg_lo < dr.lo || avg_lo > dr.hi))
        return hipErrorInvalidValue;
    if (maxd <= 8) {
        if (fold)
            down_all_launch<P, 8, true>(grid, tab, dr, p, average, sc, avg_lo, st);
        else
            down_all_launch<P, 8, false>(grid, tab, dr, p, average, sc, avg_lo, st);
    } else if (maxd <= kDownAllMaxDepth) {
        if (fold)
            down_all_launch<P, kDownAllMaxDepth, true>(grid, tab, dr, p, average, sc, avg_lo, st);
        else
            down_all_launch<P, kDownAllMaxDepth, false>(grid, tab, dr, p, average, sc, avg_lo, st);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int P>
hipError_t normalize_t(const RangeBlock *tab, int32_t n_tab, const DevPlayer &p, const Scalars *sc,
                       hipStream_t st)
{
    using T = Types<P>;
    if (n_tab <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_normalize<P>), dim3((unsigned)n_tab), dim3(kThreads), 0, st, tab,
                       (const typename T::R *)p.s, (const typename T::V *)p.x, sc,
                       (typename T::V *)p.xbar);
    return hipGetLastError();
}

template <int P>
hipError_t br_t(const RangeBlock *tab, int32_t n_tab, const DevPlayer &p, double usign,
                hipStream_t st)
{
    using T = Types<P>;
    if (n_tab <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_br<P>), dim3((unsigned)n_tab), dim3(kThreads), 0, st, tab, p.inf_first,
                       p.child_ptr, p.child_idx, (const typename T::V *)p.g, (typename T::C)usign,
                       (typename T::C *)p.vinf);
    return hipGetLastError();
}

template <int P>
hipError_t root_t(const SlotRef *tab, int32_t n_tab, const DevPlayer &p, double usign,
                  Scalars *sc, int out_index, hipStream_t st)
{
    using T = Types<P>;
    if (n_tab <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_root<P>), dim3(grid_for(n_tab)), dim3(kThreads), 0, st, n_tab, tab,
                       (const typename T::V *)p.g, (typename T::C)usign,
                       (const typename T::C *)p.vinf, sc, out_index);
    return hipGetLastError();
}

template <int P>
hipError_t dot_t(const RangeBlock *tab, int32_t n_tab, const void *a, const void *b,
                 double *partials, const SlotRef *fin, int32_t n_fin, Scalars *sc, int out_index,
                 hipStream_t st)
{
    using T = Types<P>;
    if (n_tab <= 0 || n_fin <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_dot_partial<P>), dim3((unsigned)n_tab), dim3(kThreads), 0, st, tab,
                       (const typename T::V *)a, (const typename T::V *)b, partials);
    hipLaunchKernelGGL(k_dot_final, dim3((unsigned)n_fin), dim3(kThreads), 0, st, fin, partials,
                       sc, out_index);
    return hipGetLastError();
}

}  // namespace

#define CFR_DISPATCH(prec, call)                                   \
    switch (prec) {                                                \
    case CFR_FP64: { constexpr int P = CFR_FP64; return call; }    \
    case CFR_FP32: { constexpr int P = CFR_FP32; return call; }    \
    case CFR_FP32_ACC64: { constexpr int P = CFR_FP32_ACC64; return call; } \
    default: return hipErrorInvalidValue;                          \
    }

hipError_t launch_spmv(int prec, int items, int vec, const SpmvBlock *tab, int32_t n_tab,
                       const int32_t *ptr, const int32_t *idx, const void *val, const void *xin,
                       void *yout, int xcd_remap, int sequential, int begin, Scalars *sc,
                       hipStream_t st, hipEvent_t start, hipEvent_t stop)
{
    CFR_DISPATCH(prec, spmv_t<P>(items, vec, tab, n_tab, ptr, idx, val, xin, yout, xcd_remap,
                                 sequential, begin, sc, st, start, stop));
}

hipError_t launch_up(int prec, int variant, int kind, int root, const RangeBlock *tab,
                     int32_t n_tab, const RangeBlock *direct, const DevPlayer &p, double usign,
                     const Scalars *sc, hipStream_t st)
{
    const RangeBlock dr = direct ? *direct : RangeBlock{0, 0, 0, 0};
    CFR_DISPATCH(prec, up_dispatch<P>(variant, kind, root, tab, n_tab, dr, p, usign, sc, st));
}

hipError_t launch_up_pair(int prec, int variant, int child_kind, int child_reads_slots,
                          int upper_writes_slots, int root, const RangeBlock &upper,
                          const DevPlayer &p, double usign, const Scalars *sc, hipStream_t st)
{
    CFR_DISPATCH(prec, pair_dispatch<P>(variant, child_kind, child_reads_slots,
                                        upper_writes_slots, root, upper, p, usign, sc, st));
}

hipError_t launch_top(int prec, int variant, const DevPlayer &p, double usign, int average,
                      const Scalars *sc, hipStream_t st)
{
    CFR_DISPATCH(prec, top_dispatch<P>(variant, p, usign, average, sc, st));
}

hipError_t launch_fuse(int prec, int variant, const DevPlayer &p, double usign,
                       const Scalars *sc, hipStream_t st)
{
    CFR_DISPATCH(prec, fuse_dispatch<P>(variant, p, usign, sc, st));
}

hipError_t launch_shallow(int prec, int variant, const DevPlayer &p, double usign,
                          const Scalars *sc, hipStream_t st)
{
    CFR_DISPATCH(prec, shallow_dispatch<P>(variant, p, usign, sc, st));
}

hipError_t launch_down(int prec, const RangeBlock *tab, int32_t n_tab, const DevPlayer &p,
                       int average, const Scalars *sc, hipStream_t st)
{
    CFR_DISPATCH(prec, down_t<P>(tab, n_tab, p, average, sc, st));
}

hipError_t launch_down_all(int prec, int max_depth, const RangeBlock *tab, int32_t n_tab,
                           const RangeBlock *direct, const DevPlayer &p, int average,
                           const Scalars *sc, hipStream_t st, int fold, int32_t avg_lo)
{
    const RangeBlock dr = direct ? *direct : RangeBlock{0, 0, 0, 0};
    CFR_DISPATCH(prec, down_all_t<P>(max_depth, tab, n_tab, dr, p, average, sc, fold, avg_lo, st));
}

hipError_t launch_normalize(int prec, const RangeBlock *tab, int32_t n_tab, const DevPlayer &p,
                            const Scalars *sc, hipStream_t st)
{
    CFR_DISPATCH(prec, normalize_t<P>(tab, n_tab, p, sc, st));
}

hipError_t launch_br(int prec, const RangeBlock *tab, int32_t n_tab, const DevPlayer &p,
                     double usign, hipStream_t st)
{
    CFR_DISPATCH(prec, br_t<P>(tab, n_tab, p, usign, st));
}

hipError_t launch_root_value(int prec, const SlotRef *tab, int32_t n_tab, const DevPlayer &p,
                             double usign, Scalars *sc, int out_index, hipStream_t st)
{
    CFR_DISPATCH(prec, root_t<P>(tab, n_tab, p, usign, sc, out_index, st));
}

hipError_t launch_dot(int prec, const RangeBlock *tab, int32_t n_tab, const void *a,
                      const void *b, double *partials, const SlotRef *fin, int32_t n_fin,
                      Scalars *sc, int out_index, hipStream_t st)
{
    CFR_DISPATCH(prec, dot_t<P>(tab, n_tab, a, b, partials, fin, n_fin, sc, out_index, st));
}

template <int P>
hipError_t gather_t(const RangeBlock *tab, int32_t n_tab, const int32_t *perm, const void *src,
                    void *dst, hipStream_t st)
{
    using V = typename Types<P>::V;
    if (n_tab <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_gather<P>), dim3((unsigned)n_tab), dim3(kThreads), 0, st, tab, perm,
                       (const V *)src, (V *)dst);
    return hipGetLastError();
}

hipError_t launch_gather(int prec, const RangeBlock *tab, int32_t n_tab, const int32_t *perm,
                         const void *src, void *dst, hipStream_t st)
{
    CFR_DISPATCH(prec, gather_t<P>(tab, n_tab, perm, src, dst, st));
}

hipError_t launch_quad_count(const int32_t *ptr, const int32_t *idx, int64_t nb, int32_t row0,
                             int32_t nr, int32_t *cnt, hipStream_t st)
{
    if (nr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_quad_count,
                       dim3((unsigned)((nr + kQuadRowsPerBlock - 1) / kQuadRowsPerBlock)),
                       dim3(kThreads), 0, st, ptr, idx, nb, row0, nr, cnt);
    return hipGetLastError();
}

template <int P>
hipError_t quad_fill_t(const int32_t *ptr, const int32_t *idx, const void *val, int64_t nb,
                       int32_t row0, int32_t nr, const int32_t *qptr, int64_t qb, uint32_t *qidx,
                       void *qval, hipStream_t st)
{
    using V = typename Types<P>::V;
    if (nr <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_quad_fill<P>),
                       dim3((unsigned)((nr + kQuadRowsPerBlock - 1) / kQuadRowsPerBlock)),
                       dim3(kThreads), 0, st, ptr, idx, (const V *)val, nb, row0, nr, qptr, qb,
                       qidx, (V *)qval);
    return hipGetLastError();
}

hipError_t launch_quad_fill(int prec, const int32_t *ptr, const int32_t *idx, const void *val,
                            int64_t nb, int32_t row0, int32_t nr, const int32_t *qptr, int64_t qb,
                            uint32_t *qidx, void *qval, hipStream_t st)
{
    CFR_DISPATCH(prec, quad_fill_t<P>(ptr, idx, val, nb, row0, nr, qptr, qb, qidx, qval, st));
}

hipError_t launch_remap(int32_t *a, int64_t n, const int32_t *map, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_remap, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       st, a, n, map);
    return hipGetLastError();
}

hipError_t launch_add_offset_nonneg(int32_t *a, int64_t n, int32_t base, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_offset_nonneg, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, a, n, base);
    return hipGetLastError();
}

hipError_t launch_add_offset(int32_t *a, int64_t n, int32_t base, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_offset, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, a, n, base);
    return hipGetLastError();
}

}  // namespace cfr
