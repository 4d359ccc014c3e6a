// Host runtime shared by the single-game solver and the batch of games.
//
// An engine owns one device workspace holding per-player arenas of
// sequence and decision-point indices, an arena of payoff nonzeros, one
// Scalars record per game slot and two regions of block tables (one for the
// iterating games, one for the last evaluated set).  Adding a game takes
// free ranges of each arena, uploads the game with its indices shifted to
// the global positions and sets it to the uniform strategy; every launch of
// an iteration then covers all iterating games at once, and one iteration
// is captured as a HIP graph that is replayed until the set of iterating
// games changes.
#include "cfr_engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

namespace cfr {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

const char *last_error_message() { return g_last_error.c_str(); }

std::string hip_msg(const char *what, hipError_t e)
{
    return std::string(what) + ": " + hipGetErrorString(e);
}

// ---------------------------------------------------------------------------
// Planning
// ---------------------------------------------------------------------------

namespace {

// The fused levels of a game iterating alone (k_fuse): from the first level
// below the shallow ones (the levels the one-block pass would take; level 0
// when there are none, whose top-down step the launch then does too) down
// while every level is on the fast path and holds at most kFuseDeepMax
// decision points (so the lists of any game fit kFuseListMax) and each
// subtree below one decision point of the first level holds at most
// kFuseThreads of them.  Blocks take consecutive such
// subtrees while they hold at most kFuseThreads decision points.
void plan_fuse(PlayerPlan &pl, const std::vector<int32_t> &inf_par,
               const std::vector<int32_t> &seq_new_inf)
{
    pl.fuse_lo = 0;
    pl.fuse_hi = -1;
    pl.fuse_blocks = 0;
    pl.fuse_off.clear();
    pl.fuse_list.clear();
    const int32_t L = pl.n_levels;
    int32_t S = 0;
    while (S < L && S < kShallowLevels && pl.lvl_kind[S] != 0 && pl.lvl_inf[S + 1] <= kShallowMax)
        ++S;
    if (S < 2) S = 0;
    const int32_t T0 = S;
    if (T0 + 1 >= L || pl.lvl_kind[T0] == 0 || pl.lvl_inf[T0 + 1] - pl.lvl_inf[T0] > kFuseDeepMax)
        return;
    const int32_t k0 = pl.lvl_inf[T0], nA = pl.lvl_inf[T0 + 1] - k0;
    // subtree (index of its level-T0 decision point) of every decision point
    // at level T0 and below; parents come before children in level order
    std::vector<int32_t> anc((size_t)pl.n_inf, -1);
    for (int32_t k = k0; k < pl.n_inf; ++k)
        anc[k] = k < k0 + nA ? k - k0 : anc[seq_new_inf[inf_par[k]]];
    std::vector<int32_t> sub((size_t)nA, 1), next;
    int32_t T1 = T0;
    for (int32_t l = T0 + 1; l < L && l - T0 < kFuseLevels; ++l) {
        if (pl.lvl_kind[l] == 0 || pl.lvl_inf[l + 1] - pl.lvl_inf[l] > kFuseDeepMax) break;
        next = sub;
        for (int32_t k = pl.lvl_inf[l]; k < pl.lvl_inf[l + 1]; ++k) next[anc[k]]++;
        if (*std::max_element(next.begin(), next.end()) > kFuseThreads) break;
        sub.swap(next);
        T1 = l;
    }
    if (T1 == T0) return;
    const int32_t D = T1 - T0 + 1;
    std::vector<int32_t> blk((size_t)nA);
    int32_t nb = 0, fill = 0;
    for (int32_t a = 0; a < nA; ++a) {
        if (fill + sub[a] > kFuseThreads) {
            ++nb;
            fill = 0;
        }
        blk[a] = nb;
        fill += sub[a];
    }
    ++nb;
    std::vector<int32_t> cnt((size_t)nb * D, 0);
    for (int32_t l = T0; l <= T1; ++l)
        for (int32_t k = pl.lvl_inf[l]; k < pl.lvl_inf[l + 1]; ++k)
            cnt[(size_t)blk[anc[k]] * D + (l - T0)]++;
    pl.fuse_off.assign((size_t)nb * (D + 1), 0);
    std::vector<int32_t> at((size_t)nb * D);
    int32_t pos = 0;
    for (int32_t bk = 0; bk < nb; ++bk) {
        for (int32_t l = 0; l < D; ++l) {
            pl.fuse_off[(size_t)bk * (D + 1) + l] = pos;
            at[(size_t)bk * D + l] = pos;
            pos += cnt[(size_t)bk * D + l];
        }
        pl.fuse_off[(size_t)bk * (D + 1) + D] = pos;
    }
    pl.fuse_list.assign((size_t)pos, 0);
    for (int32_t l = T0; l <= T1; ++l)
        for (int32_t k = pl.lvl_inf[l]; k < pl.lvl_inf[l + 1]; ++k)
            pl.fuse_list[(size_t)at[(size_t)blk[anc[k]] * D + (l - T0)]++] = k;
    pl.fuse_lo = T0;
    pl.fuse_hi = T1;
    pl.fuse_blocks = nb;
}

// The fused plan's lists index only decision points of their own levels,
// each once, and no block holds more than kFuseThreads (what k_fuse
// indexes and launches).
bool fuse_plan_ok(const PlayerPlan &pl)
{
    const int32_t D = pl.fuse_hi - pl.fuse_lo + 1;
    if (pl.fuse_lo < 0 || D < 2 || D > kFuseLevels || pl.fuse_hi >= pl.n_levels ||
        pl.fuse_blocks < 1 || pl.fuse_off.size() != (size_t)pl.fuse_blocks * (D + 1))
        return false;
    std::vector<uint8_t> seen((size_t)pl.n_inf, 0);
    int32_t prev = 0;
    for (int32_t bk = 0; bk < pl.fuse_blocks; ++bk) {
        const int32_t *off = pl.fuse_off.data() + (size_t)bk * (D + 1);
        if (off[0] != prev || off[D] - off[0] > kFuseThreads) return false;
        for (int32_t l = 0; l < D; ++l) {
            if (off[l + 1] < off[l]) return false;
            for (int32_t i = off[l]; i < off[l + 1]; ++i) {
                const int32_t k = pl.fuse_list[(size_t)i];
                if (k < pl.lvl_inf[pl.fuse_lo + l] || k >= pl.lvl_inf[pl.fuse_lo + l + 1] || seen[k])
                    return false;
                seen[k] = 1;
            }
        }
        prev = off[D];
    }
    return (size_t)prev == pl.fuse_list.size() &&
           prev == pl.lvl_inf[pl.fuse_hi + 1] - pl.lvl_inf[pl.fuse_lo];
}

void plan_player(const cfr_player_desc &d, bool lone, PlayerPlan &pl)
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
            if (pl.inf_first[k + 1] - pl.inf_first[k] > kFastActs) pl.lvl_kind[lv] = 0;
            for (int32_t a = pl.inf_first[k]; a < pl.inf_first[k + 1]; ++a) {
                const int32_t kids = pl.child_ptr[a + 1] - pl.child_ptr[a];
                if (kids > kFastKids) pl.lvl_kind[lv] = 0;
                else if (kids > 0 && pl.lvl_kind[lv] == 2) pl.lvl_kind[lv] = 1;
            }
        }
    // levels that can share a launch with the level above them: the lower
    // level on the fast path and at most kPairLevelMax decision points, every
    // upper decision point with at most kFastActs actions and kPairKids
    // decision points below them
    pl.lvl_pair.assign((size_t)n_levels, 0);
    for (int32_t lv = 1; lv < n_levels; ++lv) {
        bool ok = pl.lvl_kind[lv] != 0 && pl.lvl_inf[lv + 1] - pl.lvl_inf[lv] <= kPairLevelMax;
        for (int32_t k = pl.lvl_inf[lv - 1]; k < pl.lvl_inf[lv] && ok; ++k) {
            const int32_t a0 = pl.inf_first[k], a1 = pl.inf_first[k + 1];
            ok = a1 - a0 <= kFastActs && pl.child_ptr[a1] - pl.child_ptr[a0] <= kPairKids;
        }
        pl.lvl_pair[lv] = ok ? 1 : 0;
    }
    // A lone game may run its whole sweep as one launch per root subtree,
    // when every root decision point's share of every level is at most
    // kTopMaxGroup decision points (one pass of the block).  The levels of
    // one sweep form a chain of dependent memory accesses either way, so
    // this only pays when it removes every per-level launch; otherwise each
    // level gets a launch over all its decision points.
    pl.top_levels = 0;
    pl.n_roots = n_levels > 0 ? pl.lvl_inf[1] - pl.lvl_inf[0] : 0;
    pl.top_off.clear();
    pl.top_list.clear();
    pl.fuse_lo = 0;
    pl.fuse_hi = -1;
    pl.fuse_blocks = 0;
    pl.fuse_off.clear();
    pl.fuse_list.clear();
    if (n_levels == 0) return;
    std::vector<int32_t> seq_new_inf((size_t)n_seq, 0);
    for (int32_t k = 0; k < n_inf; ++k)
        for (int32_t a = pl.inf_first[k]; a < pl.inf_first[k + 1]; ++a) seq_new_inf[a] = k;
    if (!lone) {
        // a batch's game: its fused levels serve while it iterates alone
        plan_fuse(pl, inf_par, seq_new_inf);
        return;
    }
    std::vector<int32_t> root((size_t)n_inf, 0);
    for (int32_t k = 0; k < n_inf; ++k)
        root[k] = inf_par[k] == 0 ? k : root[seq_new_inf[inf_par[k]]];
    const int32_t R = pl.n_roots;
    std::vector<int32_t> cnt((size_t)R + 1);
    for (int32_t lv = 0; lv < n_levels; ++lv) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int32_t k = pl.lvl_inf[lv]; k < pl.lvl_inf[lv + 1]; ++k) cnt[root[k] + 1]++;
        int32_t mx = *std::max_element(cnt.begin(), cnt.end());
        if (mx > kTopMaxGroup) break;
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
    if (pl.top_levels == 0) plan_fuse(pl, inf_par, seq_new_inf);
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

std::vector<int32_t> narrow_ptr(const int64_t *ptr, size_t n)
{
    std::vector<int32_t> out(n);
    for (size_t i = 0; i < n; ++i) out[i] = (int32_t)ptr[i];
    return out;
}

// Row boundaries of product blocks: runs of whole rows with at most
// cap_nnz nonzeros and cap_rows rows; a longer row gets a block of its own.
std::vector<int32_t> partition_rows(const std::vector<int32_t> &ptr, int32_t cap_nnz,
                                    int32_t cap_rows)
{
    const int32_t n_rows = (int32_t)ptr.size() - 1;
    std::vector<int32_t> blk{0};
    int64_t cur_nnz = 0;
    int32_t cur_rows = 0;
    for (int32_t r = 0; r < n_rows; ++r) {
        int64_t l = ptr[r + 1] - ptr[r];
        if (l > cap_nnz) {
            if (cur_rows) blk.push_back(r);
            blk.push_back(r + 1);
            cur_nnz = 0;
            cur_rows = 0;
            continue;
        }
        if (cur_rows && (cur_nnz + l > cap_nnz || cur_rows == cap_rows)) {
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

inline int64_t chunks(int64_t n) { return (n + kRangeBlock - 1) / kRangeBlock; }

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

// Offsets of the block tables inside one table region.
struct TableLayout {
    size_t csr, csc, up[2], down[2], seq[2], dall[2], root[2], fin, bytes;
};

TableLayout table_layout(const Capacity &c)
{
    TableLayout L{};
    Carver k;
    L.csr = (size_t)k.cur;
    k.take(sizeof(SpmvBlock) * (size_t)std::max<int64_t>(c.t_csr, 1));
    L.csc = (k.cur + 255) & ~(size_t)255;
    k.take(sizeof(SpmvBlock) * (size_t)std::max<int64_t>(c.t_csc, 1));
    for (int p = 0; p < 2; ++p) {
        L.up[p] = (k.cur + 255) & ~(size_t)255;
        k.take(sizeof(RangeBlock) * (size_t)std::max<int64_t>(c.t_up[p], 1));
        L.down[p] = (k.cur + 255) & ~(size_t)255;
        k.take(sizeof(RangeBlock) * (size_t)std::max<int64_t>(c.t_down[p], 1));
        L.seq[p] = (k.cur + 255) & ~(size_t)255;
        k.take(sizeof(RangeBlock) * (size_t)std::max<int64_t>(c.t_seq[p], 1));
        L.dall[p] = (k.cur + 255) & ~(size_t)255;
        k.take(sizeof(RangeBlock) * (size_t)std::max<int64_t>(c.t_dall[p], 1));
        L.root[p] = (k.cur + 255) & ~(size_t)255;
        k.take(sizeof(SlotRef) * (size_t)c.slots);
    }
    L.fin = (k.cur + 255) & ~(size_t)255;
    k.take(sizeof(SlotRef) * (size_t)c.slots);
    L.bytes = (k.cur + 255) & ~(size_t)255;
    return L;
}

struct Layout {
    Scalars *sc;
    double *partials;
    DevPlayer dp[2];
    int32_t *ptr[2], *idx[2];
    void *val[2];
    char *tab[2];
    size_t tab_bytes;
};

Layout carve(Carver &k, const Capacity &c, int prec)
{
    const size_t V = value_bytes(prec), R = accum_bytes(prec), C = compute_bytes(prec);
    Layout L{};
    L.sc = (Scalars *)k.take(sizeof(Scalars) * (size_t)c.slots);
    L.partials = (double *)k.take(sizeof(double) * (size_t)std::max<int64_t>(c.t_seq[0], 1));
    for (int p = 0; p < 2; ++p) {
        DevPlayer &d = L.dp[p];
        const size_t n = (size_t)std::max<int64_t>(c.seq[p], 1);
        const size_t ni = (size_t)std::max<int64_t>(c.inf[p], 1);
        d.inf_first = (int32_t *)k.take(4 * ni);
        d.seq_par = (int32_t *)k.take(4 * n);
        d.child_ptr = (int32_t *)k.take(4 * n);
        d.child_idx = (int32_t *)k.take(4 * ni);
        d.r = k.take(R * n);
        d.m = k.take(R * n);
        d.s = k.take(R * n);
        d.b = k.take(V * n);
        d.x = k.take(V * (n + kVecPad));
        d.g = k.take(V * n);
        d.xbar = k.take(V * (n + kVecPad));
        d.vinf = k.take(C * ni);
        d.perm = (int32_t *)k.take(4 * n);
        d.pos = (int32_t *)k.take(4 * n);
        d.xp = k.take(V * (n + kVecPad));
        d.cslot = (int32_t *)k.take(4 * ni);
        d.ccount = (uint8_t *)k.take(n);
        d.cval = k.take(C * 4 * n);
        d.top_off = (int32_t *)k.take(4 * (size_t)std::max<int64_t>(c.top_off[p], 1));
        d.top_list = (int32_t *)k.take(4 * (size_t)std::max<int64_t>(c.top_list[p], 1));
        d.fuse_off = (int32_t *)k.take(4 * (size_t)std::max<int64_t>(c.fuse_off[p], 1));
        d.fuse_list = (int32_t *)k.take(4 * (size_t)std::max<int64_t>(c.fuse_list[p], 1));
    }
    for (int w = 0; w < 2; ++w) {
        L.ptr[w] = (int32_t *)k.take(4 * (size_t)std::max<int64_t>(c.seq[w], 1));
        // kStreamPad readable elements past the last nonzero (16-byte stream loads)
        L.idx[w] = (int32_t *)k.take(4 * (size_t)(c.nnz + kStreamPad));
        L.val[w] = k.take(V * (size_t)(c.nnz + kStreamPad));
    }
    const TableLayout T = table_layout(c);
    L.tab_bytes = T.bytes;
    for (int r = 0; r < 2; ++r) L.tab[r] = (char *)k.take(T.bytes);
    return L;
}

template <typename V, typename C>
void initial_strategy_t(const PlayerPlan &pl, std::vector<char> &bb, std::vector<char> &xb)
{
    // uniform behaviour at every decision point, then the top-down pass in
    // ascending sequence order (a parent sequence precedes its children)
    const size_t n = (size_t)pl.n_seq + 1;
    bb.assign(n * sizeof(V), 0);
    xb.assign(n * sizeof(V), 0);
    V *b = (V *)bb.data();
    V *x = (V *)xb.data();
    x[0] = (V)1;
    for (int32_t k = 0; k < pl.n_inf; ++k) {
        const int32_t a0 = pl.inf_first[k], a1 = pl.inf_first[k + 1];
        for (int32_t a = a0; a < a1; ++a) b[a] = (V)((C)1 / (C)(a1 - a0));
    }
    for (int32_t a = 1; a < pl.n_seq; ++a) x[a] = x[pl.seq_par[a]] * b[a];
}

void initial_strategy(int prec, const PlayerPlan &pl, std::vector<char> &b, std::vector<char> &x)
{
    if (prec == CFR_FP64) initial_strategy_t<double, double>(pl, b, x);
    else if (prec == CFR_FP32) initial_strategy_t<float, float>(pl, b, x);
    else initial_strategy_t<float, double>(pl, b, x);
}

template <typename T>
hipError_t h2d(void *dst, const T *src, size_t count, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, st);
}

}  // namespace

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

void prepare_game(const cfr_game_desc *g, bool lone, bool with_matrix, HostGame &hg)
{
    for (int p = 0; p < 2; ++p) plan_player(g->player[p], lone, hg.pl[p]);
    const PlayerPlan &a = hg.pl[0], &b = hg.pl[1];
    hg.nnz = g->nnz;
    const bool same = a.identity && b.identity;
    if (!with_matrix) {
        // row pointers in level order from the row and column lengths
        hg.ptr[0].assign((size_t)a.n_seq + 1, 0);
        for (int32_t r = 0; r < a.n_seq; ++r) {
            const int32_t o = a.old_of_new[r];
            hg.ptr[0][r + 1] = hg.ptr[0][r] + (int32_t)(g->row_ptr[o + 1] - g->row_ptr[o]);
        }
        std::vector<int32_t> cc((size_t)b.n_seq, 0);
        for (int64_t e = 0; e < g->nnz; ++e) cc[g->col_idx[e]]++;
        hg.ptr[1].assign((size_t)b.n_seq + 1, 0);
        for (int32_t r = 0; r < b.n_seq; ++r) hg.ptr[1][r + 1] = hg.ptr[1][r] + cc[b.old_of_new[r]];
        return;
    }
    const int64_t *rptr = g->row_ptr;
    std::vector<int64_t> ptr_buf;
    hg.idx[0] = g->col_idx;
    hg.val[0] = g->val;
    if (!same) {
        permute_rows(a.n_seq, a.old_of_new, b.new_of_old, g->row_ptr, g->col_idx, g->val, ptr_buf,
                     hg.own_idx[0], hg.own_val[0]);
        rptr = ptr_buf.data();
        hg.idx[0] = hg.own_idx[0].data();
        hg.val[0] = hg.own_val[0].data();
    }
    hg.ptr[0] = narrow_ptr(rptr, (size_t)a.n_seq + 1);
    if (same && g->col_ptr) {
        // validated to be the exact transpose
        hg.ptr[1] = narrow_ptr(g->col_ptr, (size_t)b.n_seq + 1);
        hg.idx[1] = g->row_idx;
        hg.val[1] = g->val_csc;
    } else {
        std::vector<int64_t> tptr;
        transpose(a.n_seq, b.n_seq, rptr, hg.idx[0], hg.val[0], tptr, hg.own_idx[1],
                  hg.own_val[1]);
        hg.ptr[1] = narrow_ptr(tptr.data(), (size_t)b.n_seq + 1);
        hg.idx[1] = hg.own_idx[1].data();
        hg.val[1] = hg.own_val[1].data();
    }
}

// Page-locked host buffer freed with hipHostFree, or null.
static std::shared_ptr<void> pinned_buffer(size_t bytes)
{
    void *p = nullptr;
    if (bytes == 0 || hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess || !p) {
        (void)hipGetLastError();
        return nullptr;
    }
    return std::shared_ptr<void>(p, [](void *q) { (void)hipHostFree(q); });
}

void build_image(const HostGame &hg, int prec, bool pinned, bool borrow, GameImage &img)
{
    const size_t V = value_bytes(prec);
    const size_t nnz = (size_t)hg.nnz;
    img.prec = prec;
    img.nnz = hg.nnz;
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        cur = (cur + 255) & ~(size_t)255;
        const size_t at = cur;
        cur += bytes;
        return at;
    };
    for (int p = 0; p < 2; ++p) {
        const size_t n = (size_t)hg.pl[p].n_seq, ni = (size_t)hg.pl[p].n_inf;
        img.n_seq[p] = hg.pl[p].n_seq;
        img.n_inf[p] = hg.pl[p].n_inf;
        GameImage::Player &q = img.pl[p];
        q.inf_first = take(4 * (ni + 1));
        q.seq_par = take(4 * (n + 1));
        q.child_ptr = take(4 * (n + 1));
        q.child_idx = take(4 * ni);
        q.cslot = take(4 * ni);
        q.ccount = take(n + 1);
        q.b0 = take(V * (n + 1));
        q.x0 = take(V * (n + 1));
        q.perm = take(4 * (n + 1));
        q.pos = take(4 * (n + 1));
    }
    const bool copy_idx = !borrow, copy_val = !borrow || V == 4;
    for (int w = 0; w < 2; ++w) {
        img.ptr[w] = take(4 * hg.ptr[w].size());
        img.idx[w] = copy_idx ? take(4 * nnz) : 0;
        img.val[w] = copy_val ? take(V * nnz) : 0;
    }
    img.bytes = (cur + 255) & ~(size_t)255;
    img.pinned = pinned ? pinned_buffer(img.bytes) : nullptr;
    img.locked = img.pinned != nullptr;
    if (img.locked) {
        img.base = (char *)img.pinned.get();
    } else {
        img.plain.assign(img.bytes, 0);
        img.base = img.plain.data();
    }
    char *B = img.base;
    for (int p = 0; p < 2; ++p) {
        const PlayerPlan &pl = hg.pl[p];
        const GameImage::Player &q = img.pl[p];
        const size_t n = (size_t)pl.n_seq, ni = (size_t)pl.n_inf;
        std::memcpy(B + q.inf_first, pl.inf_first.data(), 4 * (ni + 1));
        int32_t *sp = (int32_t *)(B + q.seq_par);
        std::memcpy(sp, pl.seq_par.data(), 4 * n);
        sp[n] = 0;  // the sentinel's parent: the empty sequence
        std::memcpy(B + q.child_ptr, pl.child_ptr.data(), 4 * (n + 1));
        if (ni) std::memcpy(B + q.child_idx, pl.child_idx.data(), 4 * ni);
        // value slots: the decision points below a sequence with at most
        // kFastKids of them, in ascending order (local 4 * sequence + rank)
        int32_t *cs = (int32_t *)(B + q.cslot);
        uint8_t *cc = (uint8_t *)(B + q.ccount);
        for (size_t j = 0; j < ni; ++j) cs[j] = -1;
        for (size_t a = 0; a < n; ++a) {
            const int32_t c0 = pl.child_ptr[a], cnt = pl.child_ptr[a + 1] - c0;
            cc[a] = (uint8_t)std::min(cnt, 255);
            if (cnt > kFastKids) continue;
            for (int32_t k = 0; k < cnt; ++k)
                cs[(size_t)pl.child_idx[(size_t)(c0 + k)]] = 4 * (int32_t)a + k;
        }
        cc[n] = 0;
        std::vector<char> hb, hx;
        initial_strategy(prec, pl, hb, hx);
        std::memcpy(B + q.b0, hb.data(), hb.size());
        std::memcpy(B + q.x0, hx.data(), hx.size());
    }
    // first-touch order of each player's sequences in the product that
    // gathers them (rows in order, columns ascending)
    for (int w = 0; w < 2; ++w) {
        const int q = 1 - w;
        const int32_t n = hg.pl[q].n_seq;
        int32_t *perm = (int32_t *)(B + img.pl[q].perm);
        int32_t *pos = (int32_t *)(B + img.pl[q].pos);
        std::vector<char> seen((size_t)n, 0);
        int32_t next = 0;
        for (size_t i = 0; i < nnz; ++i) {
            const int32_t c = hg.idx[w][i];
            if (!seen[(size_t)c]) {
                seen[(size_t)c] = 1;
                perm[next++] = c;
            }
        }
        for (int32_t c = 0; c < n; ++c)
            if (!seen[(size_t)c]) perm[next++] = c;
        perm[n] = n;  // the sentinel maps to itself
        for (int32_t j = 0; j <= n; ++j) pos[perm[j]] = j;
    }
    for (int w = 0; w < 2; ++w) {
        std::memcpy(B + img.ptr[w], hg.ptr[w].data(), 4 * hg.ptr[w].size());
        if (copy_idx) {
            if (nnz) std::memcpy(B + img.idx[w], hg.idx[w], 4 * nnz);
            img.idx_src[w] = (const int32_t *)(B + img.idx[w]);
        } else {
            img.idx_src[w] = hg.idx[w];
        }
        if (V == 4) {
            float *f = (float *)(B + img.val[w]);
            for (size_t i = 0; i < nnz; ++i) f[i] = (float)hg.val[w][i];
            img.val_src[w] = f;
        } else if (copy_val) {
            if (nnz) std::memcpy(B + img.val[w], hg.val[w], 8 * nnz);
            img.val_src[w] = B + img.val[w];
        } else {
            img.val_src[w] = hg.val[w];
        }
    }
}

// The quads of one product, host side: the same rule as the device build
// (a quad is a maximal run of consecutive nonzeros of a row, in row order,
// whose columns increase and share one aligned group of four).
void build_image_quads(const HostGame &hg, const int perm[2], bool pinned, GameImage &img)
{
    GameImage::Quads &Q = img.quads;
    const size_t V = value_bytes(img.prec);
    std::vector<int32_t> cols;
    // pass 1: quad counts (row pointers), with each product's column order
    for (int w = 0; w < 2; ++w) {
        const int q = 1 - w;
        const std::vector<int32_t> &rp = hg.ptr[w];
        const int32_t *ix = img.idx_src[w];
        const int32_t *pos = (const int32_t *)(img.base + img.pl[q].pos);
        Q.perm[w] = perm[w] ? 1 : 0;
        std::vector<int32_t> &qp = Q.qptr[w];
        qp.assign(rp.size(), 0);
        for (size_t r = 0; r + 1 < rp.size(); ++r) {
            int32_t c = 0, prev = -1;
            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
                const int32_t col = Q.perm[w] ? pos[ix[e]] : ix[e];
                if (e == rp[r] || (col >> 2) != (prev >> 2) || col <= prev) ++c;
                prev = col;
            }
            qp[r + 1] = qp[r] + c;
        }
        Q.nq[w] = qp.back();
    }
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        cur = (cur + 255) & ~(size_t)255;
        const size_t at = cur;
        cur += bytes;
        return at;
    };
    for (int w = 0; w < 2; ++w) {
        Q.ptr[w] = take(4 * Q.qptr[w].size());
        Q.idx[w] = take(4 * (size_t)Q.nq[w]);
        Q.val[w] = take(4 * V * (size_t)Q.nq[w]);
    }
    const size_t bytes = std::max<size_t>((cur + 255) & ~(size_t)255, 256);
    Q.pinned = pinned ? pinned_buffer(bytes) : nullptr;
    Q.locked = Q.pinned != nullptr;
    if (Q.locked) {
        Q.base = (char *)Q.pinned.get();
    } else {
        Q.plain.assign(bytes, 0);
        Q.base = Q.plain.data();
    }
    // pass 2: the quads
    for (int w = 0; w < 2; ++w) {
        const int q = 1 - w;
        const std::vector<int32_t> &rp = hg.ptr[w];
        const int32_t *ix = img.idx_src[w];
        const int32_t *pos = (const int32_t *)(img.base + img.pl[q].pos);
        std::memcpy(Q.base + Q.ptr[w], Q.qptr[w].data(), 4 * Q.qptr[w].size());
        uint32_t *qi = (uint32_t *)(Q.base + Q.idx[w]);
        char *qv = Q.base + Q.val[w];
        const char *vs = (const char *)img.val_src[w];
        int64_t k = 0;
        for (size_t r = 0; r + 1 < rp.size(); ++r) {
            uint32_t mask = 0;
            int32_t prev = -1;
            for (int32_t e = rp[r]; e <= rp[r + 1]; ++e) {
                const bool end = e == rp[r + 1];
                const int32_t col = end ? 0 : (Q.perm[w] ? pos[ix[e]] : ix[e]);
                if (mask != 0 && (end || (col >> 2) != (prev >> 2) || col <= prev)) {
                    qi[k] = (uint32_t)(prev >> 2) | (mask << kQuadMaskShift);
                    ++k;
                    mask = 0;
                }
                if (end) break;
                if (mask == 0) std::memset(qv + 4 * V * (size_t)k, 0, 4 * V);
                std::memcpy(qv + V * (4 * (size_t)k + (size_t)(col & 3)), vs + V * (size_t)e, V);
                mask |= 1u << (col & 3);
                prev = col;
            }
        }
        Q.built[w] = true;
    }
}

Capacity lone_capacity(const HostGame &hg, int items_csr, int rows_csr, int items_csc,
                       int rows_csc)
{
    Capacity c;
    c.slots = 1;
    for (int p = 0; p < 2; ++p) {
        const PlayerPlan &pl = hg.pl[p];
        c.seq[p] = seq_block(pl.n_seq);
        c.inf[p] = (int64_t)pl.n_inf + 1;
        c.t_up[p] = 0;
        c.t_down[p] = 0;
        for (int32_t lv = 0; lv < pl.n_levels; ++lv) {
            c.t_up[p] += chunks(pl.lvl_inf[lv + 1] - pl.lvl_inf[lv]);
            if (lv > 0) c.t_down[p] += chunks(pl.lvl_seq[lv + 1] - pl.lvl_seq[lv]);
        }
        c.t_seq[p] = chunks(pl.n_seq);
        c.t_dall[p] = pl.n_levels > 1 ? chunks(pl.n_seq - pl.lvl_seq[1]) : 0;
        c.top_off[p] = (int64_t)pl.top_off.size();
        c.top_list[p] = (int64_t)pl.top_list.size();
        c.fuse_off[p] = (int64_t)pl.fuse_off.size();
        c.fuse_list[p] = (int64_t)pl.fuse_list.size();
    }
    c.nnz = hg.nnz;
    // product tables large enough for every tiling the tuner may choose
    // (the most blocks come from the smallest caps)
    (void)items_csr;
    (void)rows_csr;
    (void)items_csc;
    (void)rows_csc;
    c.t_csr = (int64_t)partition_rows(hg.ptr[0], kMinBlockCap, 64).size() - 1;
    c.t_csc = (int64_t)partition_rows(hg.ptr[1], kMinBlockCap, 64).size() - 1;
    return c;
}

void bound_tables(Capacity &c)
{
    // A game's product blocks: two consecutive blocks together exceed the
    // nonzero cap unless the row cap closed the first, so a game with z
    // nonzeros and n rows has at most 2 z / cap + n / row_cap + 2 blocks
    // (smallest tiling: kMinBlockCap stream elements, each holding at least
    // one nonzero, and 64 rows).  Range blocks: one per
    // kRangeBlock indices plus one partial block per (game, level), and a
    // game has at most as many levels as decision points.
    for (int w = 0; w < 2; ++w) {
        const int64_t t = 2 * c.nnz / kMinBlockCap + c.seq[w] / 64 + 2 * c.slots + 1;
        if (w == 0) c.t_csr = t;
        else c.t_csc = t;
    }
    for (int p = 0; p < 2; ++p) {
        c.t_up[p] = c.inf[p] / kRangeBlock + c.inf[p] + 1;
        c.t_down[p] = c.seq[p] / kRangeBlock + c.inf[p] + 1;
        c.t_seq[p] = c.seq[p] / kRangeBlock + c.slots + 1;
        c.t_dall[p] = c.seq[p] / kRangeBlock + c.slots + 1;
        c.top_off[p] = 0;
        c.top_list[p] = 0;
        // the fused levels of the one game iterating alone: a game's list
        // holds at most its own decision points and at most kFuseLevels
        // levels of kFuseDeepMax, and a block holds one of them at least
        c.fuse_list[p] = std::min<int64_t>(kFuseListMax, c.inf[p]);
        c.fuse_off[p] = (int64_t)(kFuseLevels + 1) * c.fuse_list[p];
    }
}

size_t engine_bytes(const Capacity &c, int prec)
{
    Carver k;
    carve(k, c, prec);
    return k.cur + 256;
}

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

HostTimer::HostTimer(double *a, int64_t *c) : acc(a), cnt(c), t0(now_s()) {}
HostTimer::~HostTimer()
{
    *acc += now_s() - t0;
    ++*cnt;
}

// ---------------------------------------------------------------------------
// Range allocator
// ---------------------------------------------------------------------------

void RangeAlloc::init(int64_t c)
{
    cap = c;
    free_.clear();
    if (c > 0) free_[0] = c;
}

int64_t RangeAlloc::take(int64_t n)
{
    if (n <= 0) return 0;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < n) continue;
        const int64_t at = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[at + n] = len - n;
        return at;
    }
    return -1;
}

void RangeAlloc::give(int64_t at, int64_t n)
{
    if (n <= 0) return;
    auto it = free_.emplace(at, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        free_.erase(nx);
    }
    if (it != free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            free_.erase(it);
        }
    }
}

int64_t RangeAlloc::largest() const
{
    int64_t m = 0;
    for (const auto &kv : free_) m = std::max(m, kv.second);
    return m;
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------

int Engine::init(const Capacity &c, int precision, int dev, hipStream_t stream, void *workspace,
                 size_t workspace_bytes)
{
    // value slots are addressed as 4 * sequence in int32
    if (c.seq[0] > (int64_t)1 << 29 || c.seq[1] > (int64_t)1 << 29)
        return fail(CFR_EINVAL, "more than 2^29 sequences per player");
    cap = c;
    prec = precision;
    device = dev;
    st = stream;
    const size_t need = engine_bytes(c, prec);
    if (workspace) {
        if (workspace_bytes < need)
            return fail(CFR_ENOMEM, "workspace smaller than the required size");
        ws = workspace;
        ws_bytes = workspace_bytes;
        own_ws = false;
    } else {
        hipError_t e = hipMalloc(&ws, need);
        if (e != hipSuccess) {
            ws = nullptr;
            return fail(CFR_ENOMEM, hip_msg("hipMalloc of the workspace", e));
        }
        ws_bytes = need;
        own_ws = true;
    }
    Carver k;
    k.base = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    Layout L = carve(k, c, prec);
    sc = L.sc;
    partials = L.partials;
    for (int p = 0; p < 2; ++p) dp[p] = L.dp[p];
    for (int w = 0; w < 2; ++w) {
        ptr[w] = L.ptr[w];
        idx[w] = L.idx[w];
        val[w] = L.val[w];
    }
    tab_region[0] = L.tab[0];
    tab_region[1] = L.tab[1];
    tab_bytes = L.tab_bytes;
    const TableLayout T = table_layout(c);
    Tables *ts[2] = {&it, &ev};
    for (int r = 0; r < 2; ++r) {
        Tables &t = *ts[r];
        char *base = tab_region[r];
        t.csr = (SpmvBlock *)(base + T.csr);
        t.csc = (SpmvBlock *)(base + T.csc);
        for (int p = 0; p < 2; ++p) {
            t.up[p] = (RangeBlock *)(base + T.up[p]);
            t.down[p] = (RangeBlock *)(base + T.down[p]);
            t.seq[p] = (RangeBlock *)(base + T.seq[p]);
            t.dall[p] = (RangeBlock *)(base + T.dall[p]);
            t.root[p] = (SlotRef *)(base + T.root[p]);
        }
        t.fin = (SlotRef *)(base + T.fin);
        t.valid = false;
    }
    // Every index array starts at zero: the fast sweep path issues clamped
    // loads that may read child_idx[0] of an unused range.
    hipError_t e = hipMemsetAsync(sc, 0, sizeof(Scalars) * (size_t)c.slots, st);
    for (int p = 0; p < 2 && e == hipSuccess; ++p)
        e = hipMemsetAsync(dp[p].child_idx, 0, 4 * (size_t)std::max<int64_t>(c.inf[p], 1), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error("workspace initialisation", e);
    // an allocation-free engine admits its one game synchronously on the
    // caller's stream and stages from ordinary host memory
    if (no_alloc) return init_arenas(c);
    e = hipStreamCreateWithFlags(&up_st, hipStreamNonBlocking);
    if (e != hipSuccess) return device_error("upload stream", e);
    {
        void *p = nullptr;
        if (hipHostMalloc(&p, sizeof(Scalars) * (size_t)c.slots, hipHostMallocDefault) ==
                hipSuccess &&
            p)
            scal_stage = (Scalars *)p;
        else
            (void)hipGetLastError();
    }
    {
        // results of asynchronous checks (run_begin / run_end)
        void *p = nullptr;
        if (hipHostMalloc(&p, sizeof(Scalars) * (size_t)c.slots, hipHostMallocDefault) ==
                hipSuccess &&
            p)
            eval_stage = (Scalars *)p;
        else
            (void)hipGetLastError();
        if (hipEventCreateWithFlags(&eval_ev, hipEventDisableTiming) != hipSuccess) {
            eval_ev = nullptr;
            (void)hipGetLastError();
        }
    }
    return init_arenas(c);
}

int Engine::init_arenas(const Capacity &c)
{
    for (int p = 0; p < 2; ++p) {
        seq_alloc[p].init(c.seq[p]);
        inf_alloc[p].init(c.inf[p]);
    }
    nnz_alloc.init(c.nnz);
    slots.assign((size_t)c.slots, Slot());
    return CFR_OK;
}

void Engine::drop_graph()
{
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    direct_runs = 0;
}

void Engine::release()
{
    if (pending && eval_ev) (void)hipEventSynchronize(eval_ev);
    for (int k = 0; k < 2; ++k) {
        for (auto &pr : events[k]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        events[k].clear();
    }
    drop_graph();
    reap_uploads(true);
    if (cap_st) (void)hipStreamDestroy(cap_st);
    cap_st = nullptr;
    if (up_st) (void)hipStreamDestroy(up_st);
    up_st = nullptr;
    if (scal_stage) (void)hipHostFree(scal_stage);
    scal_stage = nullptr;
    if (eval_ev) (void)hipEventDestroy(eval_ev);
    eval_ev = nullptr;
    if (eval_stage) (void)hipHostFree(eval_stage);
    eval_stage = nullptr;
    pending = false;
    if (own_ws && ws) (void)hipFree(ws);
    ws = nullptr;
    for (QuadStore &Q : quad) {
        if (Q.ptr) (void)hipFree(Q.ptr);
        if (Q.idx) (void)hipFree(Q.idx);
        if (Q.val) (void)hipFree(Q.val);
        Q = QuadStore();
    }
}

int Engine::device_error(const char *what, hipError_t e)
{
    failed = true;
    return fail(CFR_EDEVICE, hip_msg(what, e));
}

int Engine::sync(const char *what)
{
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return device_error(what, e);
    return CFR_OK;
}

int Engine::sequential() const
{
    if (spmv_order == CFR_SPMV_SEQUENTIAL) return 1;
    if (spmv_order == CFR_SPMV_PARALLEL) return 0;
    return prec == CFR_FP64 ? 1 : 0;
}

void Engine::partition(Slot &s, int which)
{
    const int k = (int)(&s - slots.data());
    s.blocks[which].clear();
    const bool quads = vec[which] == 3;
    // stream form 3 partitions the game's quads, once they are built
    if (quads && s.qb[which] < 0) return;
    const std::vector<int32_t> &rp = quads ? s.qptr[which] : s.ptr[which];
    const int64_t base = quads ? s.qb[which] : s.nb;
    const std::vector<int32_t> blk =
        partition_rows(rp, spmv_block_cap_v(items[which], vec[which]), rows[which]);
    s.blocks[which].reserve(blk.size());
    for (size_t i = 0; i + 1 < blk.size(); ++i) {
        const int32_t r0 = blk[i], r1 = blk[i + 1];
        SpmvBlock b{};
        b.row0 = (int32_t)(s.sb[which] + r0);
        b.nr = r1 - r0;
        b.n = rp[r1] - rp[r0];
        b.p0 = rp[r0];
        b.e0 = base + rp[r0];
        b.slot = k;
        b.begin = i == 0 ? 1 : 0;
        s.blocks[which].push_back(b);
    }
}

void Engine::drop_quads(Slot &s, int which)
{
    if (s.qb[which] >= 0 && s.nq[which] > 0) quad[which].alloc.give(s.qb[which], s.nq[which]);
    s.qb[which] = -1;
    s.nq[which] = 0;
    s.qptr[which].clear();
    s.qptr[which].shrink_to_fit();
    if (vec[which] == 3) s.blocks[which].clear();
}

int Engine::grow_quads(int which, int64_t need)
{
    QuadStore &Q = quad[which];
    const size_t V = value_bytes(prec);
    int64_t ncap = std::max<int64_t>(need, Q.cap + Q.cap / 2);
    // a batch starts with room for many games (each growth waits for both
    // streams and copies the store): min(kQuadStoreMin, its nonzero capacity)
    if (!lone && quad_reserved == 0)
        ncap = std::max<int64_t>(ncap, std::min<int64_t>(kQuadStoreMin, cap.nnz));
    uint32_t *ni = nullptr;
    void *nv = nullptr;
    hipError_t e = hipMalloc((void **)&ni, 4 * (size_t)ncap);
    if (e == hipSuccess) e = hipMalloc(&nv, 4 * V * (size_t)ncap);
    if (e != hipSuccess) {
        if (ni) (void)hipFree(ni);
        if (nv) (void)hipFree(nv);
        (void)hipGetLastError();
        return fail(CFR_ENOMEM, "cannot allocate the quad stream of a product");
    }
    if (Q.cap > 0) {
        // admission copies may still be writing into the old buffers
        if (up_st) e = hipStreamSynchronize(up_st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ni, Q.idx, 4 * (size_t)Q.cap, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(nv, Q.val, 4 * V * (size_t)Q.cap, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipFree(ni);
            (void)hipFree(nv);
            return device_error("quad stream copy", e);
        }
        (void)hipFree(Q.idx);
        (void)hipFree(Q.val);
        Q.alloc.give(Q.cap, ncap - Q.cap);
    } else {
        Q.alloc.init(ncap);
    }
    Q.idx = ni;
    Q.val = nv;
    Q.cap = ncap;
    Q.alloc.cap = ncap;
    drop_graph();
    return CFR_OK;
}

int Engine::reserve_quads(int64_t n)
{
    quad_reserved = n;
    for (int w = 0; w < 2; ++w) {
        QuadStore &Q = quad[w];
        if (!Q.ptr) {
            if (hipMalloc((void **)&Q.ptr, 4 * (size_t)std::max<int64_t>(cap.seq[w], 1)) !=
                hipSuccess) {
                Q.ptr = nullptr;
                (void)hipGetLastError();
                return fail(CFR_ENOMEM, "cannot allocate the quad row pointers of a product");
            }
        }
        if (Q.cap < n) {
            int rc = grow_quads(w, n);
            if (rc) return rc;
        }
    }
    return CFR_OK;
}

int Engine::ensure_quads(const std::vector<int> &set)
{
    for (int w = 0; w < 2; ++w) {
        if (vec[w] != 3) continue;
        std::vector<int> todo;
        for (int k : set)
            if (slots[(size_t)k].qb[w] < 0) todo.push_back(k);
        if (todo.empty()) continue;
        HostTimer timer(&host_s[kHostQuads], &host_n[kHostQuads]);
        // the stream waits for these games' admission copies (and only
        // theirs: games admitted meanwhile keep copying)
        hipError_t e = wait_uploads(todo);
        if (e != hipSuccess) return device_error("admission copies", e);
        QuadStore &Q = quad[w];
        if (!Q.ptr) {
            e = hipMalloc((void **)&Q.ptr, 4 * (size_t)std::max<int64_t>(cap.seq[w], 1));
            if (e != hipSuccess) {
                Q.ptr = nullptr;
                (void)hipGetLastError();
                return fail(CFR_ENOMEM, "cannot allocate the quad row pointers of a product");
            }
        }
        // quads per row of every game, counted into the row-pointer slots
        // themselves, brought back with one synchronisation
        std::vector<std::vector<int32_t>> qp(todo.size());
        for (size_t t = 0; t < todo.size() && e == hipSuccess; ++t) {
            const Slot &s = slots[(size_t)todo[t]];
            const int32_t nr = (int32_t)s.ptr[w].size() - 1;
            const int32_t row0 = (int32_t)s.sb[w];
            qp[t].assign((size_t)nr + 1, 0);
            e = launch_quad_count(ptr[w], idx[w], s.nb, row0, nr, Q.ptr + row0, st);
            if (e == hipSuccess && nr > 0)
                e = hipMemcpyAsync(qp[t].data() + 1, Q.ptr + row0, 4 * (size_t)nr,
                                   hipMemcpyDeviceToHost, st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_error("quad count", e);
        int64_t need = 0;
        for (auto &v : qp) {
            for (size_t r = 1; r < v.size(); ++r) v[r] += v[r - 1];
            need += v.back();
        }
        // room for all of them at once (one reallocation at most)
        if (need > 0 && Q.alloc.largest() < need) {
            int rc = grow_quads(w, std::max<int64_t>(Q.cap + need, 2 * Q.cap));
            if (rc) return rc;
        }
        for (size_t t = 0; t < todo.size(); ++t) {
            Slot &s = slots[(size_t)todo[t]];
            const int32_t nr = (int32_t)qp[t].size() - 1;
            const int32_t row0 = (int32_t)s.sb[w];
            const int64_t nq = qp[t].back();
            int64_t qb = 0;
            if (nq > 0) {
                qb = Q.alloc.take(nq);
                if (qb < 0) {
                    int rc = grow_quads(w, std::max<int64_t>(Q.cap + nq, 2 * Q.cap));
                    if (rc) return rc;
                    qb = Q.alloc.take(nq);
                    if (qb < 0) return fail(CFR_ENOMEM, "quad stream exhausted");
                }
            }
            // the host row pointers live in the slot, so the copy may run on
            s.qptr[w] = std::move(qp[t]);
            e = hipMemcpyAsync(Q.ptr + row0, s.qptr[w].data(), 4 * ((size_t)nr + 1),
                               hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = launch_quad_fill(prec, ptr[w], idx[w], val[w], s.nb, row0, nr, Q.ptr, qb, Q.idx,
                                     Q.val, st);
            if (e != hipSuccess) return device_error("quad fill", e);
            s.qb[w] = qb;
            s.nq[w] = nq;
            partition(s, w);
        }
        drop_graph();
    }
    return CFR_OK;
}

int Engine::set_perm(int which, int on)
{
    on = on ? 1 : 0;
    if (perm_on[which] == on) return CFR_OK;
    reap_uploads(true);  // the index streams of games still being copied
    const int q = 1 - which;
    for (Slot &s : slots) {
        if (!s.live || s.nnz == 0) continue;
        hipError_t e = launch_remap(idx[which] + s.nb, s.nnz, on ? dp[q].pos : dp[q].perm, st);
        if (e != hipSuccess) return device_error("index remap", e);
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error("index remap", e);
    perm_on[which] = on;
    // quad copies follow the numbering of the index stream
    for (Slot &s : slots)
        if (s.live) drop_quads(s, which);
    it.valid = false;
    ev.valid = false;
    drop_graph();
    return CFR_OK;
}

void Engine::repartition(int which, int items_, int rows_, int vec_)
{
    items[which] = items_;
    rows[which] = rows_;
    vec[which] = vec_;
    for (Slot &s : slots)
        if (s.live) partition(s, which);
    it.valid = false;
    ev.valid = false;
    drop_graph();
}

int Engine::set_params(int k, const GameParams &gp)
{
    Slot &s = slots[(size_t)k];
    s.gp = gp;
    struct {
        double alpha, beta, gamma;
        int32_t variant, avg_kind;
    } h{gp.alpha, gp.beta, gp.gamma, gp.variant, gp.avg_kind};
    static_assert(sizeof(h) == offsetof(Scalars, pad) - offsetof(Scalars, alpha), "layout");
    hipError_t e = hipMemcpyAsync((char *)(sc + k) + offsetof(Scalars, alpha), &h, sizeof h,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error("game constants", e);
    it.valid = false;
    ev.valid = false;
    drop_graph();
    return CFR_OK;
}

int Engine::add(const HostGame &hg, const GameImage &img, const GameParams &gp, bool join_now,
                bool async, int *slot_out)
{
    HostTimer timer(&host_s[kHostAdd], &host_n[kHostAdd]);
    int k = -1;
    for (size_t i = 0; i < slots.size(); ++i)
        if (!slots[i].live) {
            k = (int)i;
            break;
        }
    if (k < 0) return fail(CFR_ENOMEM, "every game slot is in use");
    int64_t sb[2] = {-1, -1}, ib[2] = {-1, -1}, nb = -1;
    bool ok = true;
    for (int p = 0; p < 2 && ok; ++p) {
        sb[p] = seq_alloc[p].take(seq_block(hg.pl[p].n_seq));
        if (sb[p] < 0) ok = false;
        else {
            ib[p] = inf_alloc[p].take((int64_t)hg.pl[p].n_inf + 1);
            if (ib[p] < 0) ok = false;
        }
    }
    if (ok) {
        nb = hg.nnz > 0 ? nnz_alloc.take(hg.nnz) : 0;
        if (nb < 0) ok = false;
    }
    if (!ok) {
        for (int p = 0; p < 2; ++p) {
            if (sb[p] >= 0) seq_alloc[p].give(sb[p], seq_block(hg.pl[p].n_seq));
            if (ib[p] >= 0) inf_alloc[p].give(ib[p], (int64_t)hg.pl[p].n_inf + 1);
        }
        return fail(CFR_ENOMEM, "the game does not fit the free device capacity");
    }
    Slot &s = slots[(size_t)k];
    s = Slot();
    s.id = next_id++;
    s.gp = gp;
    s.nb = nb;
    s.nnz = hg.nnz;
    // Asynchronous admission copies the game's image on the upload stream
    // and returns; the image must outlive the copies (a prepared game owns
    // its own).  Indices are shifted to the game's global positions on the
    // device.
    const hipStream_t ups = async ? up_st : st;
    const char *B = img.base;
    hipError_t e = hipSuccess;
#define CHECK(x)                                                 \
    do {                                                         \
        e = (x);                                                 \
        if (e != hipSuccess) return device_error("add game", e); \
    } while (0)
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ups) : hipSuccess;
    };
    const size_t R = accum_bytes(prec), V = value_bytes(prec);
    for (int p = 0; p < 2; ++p) {
        const PlayerPlan &pl = hg.pl[p];
        const GameImage::Player &q = img.pl[p];
        s.sb[p] = sb[p];
        s.ib[p] = ib[p];
        s.n_seq[p] = pl.n_seq;
        s.n_inf[p] = pl.n_inf;
        s.n_levels[p] = pl.n_levels;
        s.lvl_inf[p] = pl.lvl_inf;
        s.lvl_seq[p] = pl.lvl_seq;
        s.lvl_kind[p] = pl.lvl_kind;
        s.lvl_pair[p] = pl.lvl_pair;
        // Small levels store their values in the parent's slots and the
        // level above reads them from there (one dependent load fewer);
        // big levels write their values contiguously, since slot writes
        // scatter.  Levels that the one-launch shallow sweep covers, and
        // the one right below them, keep to the plain layout it reads.
        // Slots need the player's whole index space below kSlotSeqLimit.
        s.lvl_slots[p].assign((size_t)pl.n_levels, 0);
        const int32_t top_low = lone ? pl.top_levels : 0;
        const bool slots_ok = slots_fit(cap.seq[p]);
        for (int32_t L = 1; L < pl.n_levels && slots_ok; ++L)
            if (pl.lvl_inf[L + 1] - pl.lvl_inf[L] <= kSlotLevelMax && L > top_low) {
                s.lvl_slots[p][L] |= kSlotsWrite;
                s.lvl_slots[p][L - 1] |= kSlotsRead;
            }
        s.old_of_new[p] = pl.old_of_new;
        const int32_t S = (int32_t)sb[p], I = (int32_t)ib[p];
        const size_t n = (size_t)pl.n_seq, ni = (size_t)pl.n_inf;
        DevPlayer &d = dp[p];
        CHECK(cp(d.inf_first + I, B + q.inf_first, 4 * (ni + 1)));
        CHECK(launch_add_offset(d.inf_first + I, (int64_t)ni + 1, S, ups));
        CHECK(cp(d.seq_par + S, B + q.seq_par, 4 * (n + 1)));
        CHECK(launch_add_offset(d.seq_par + S, (int64_t)n + 1, S, ups));
        CHECK(cp(d.child_ptr + S, B + q.child_ptr, 4 * (n + 1)));
        CHECK(launch_add_offset(d.child_ptr + S, (int64_t)n + 1, I, ups));
        CHECK(cp(d.child_idx + I, B + q.child_idx, 4 * ni));
        CHECK(launch_add_offset(d.child_idx + I, (int64_t)ni, I, ups));
        CHECK(cp(d.cslot + I, B + q.cslot, 4 * ni));
        // (read only on slot levels, which exist only when 4 * S fits)
        if (slots_fit(cap.seq[p]))
            CHECK(launch_add_offset_nonneg(d.cslot + I, (int64_t)ni, 4 * S, ups));
        CHECK(cp(d.ccount + S, B + q.ccount, n + 1));
        CHECK(cp((char *)d.b + V * (size_t)S, B + q.b0, V * (n + 1)));
        CHECK(cp((char *)d.x + V * (size_t)S, B + q.x0, V * (n + 1)));
        CHECK(cp(d.perm + S, B + q.perm, 4 * (n + 1)));
        CHECK(launch_add_offset(d.perm + S, (int64_t)n + 1, S, ups));
        CHECK(cp(d.pos + S, B + q.pos, 4 * (n + 1)));
        CHECK(launch_add_offset(d.pos + S, (int64_t)n + 1, S, ups));
        // state: zero regrets, predictions and averages
        CHECK(hipMemsetAsync((char *)d.r + R * (size_t)S, 0, R * (n + 1), ups));
        CHECK(hipMemsetAsync((char *)d.m + R * (size_t)S, 0, R * (n + 1), ups));
        CHECK(hipMemsetAsync((char *)d.s + R * (size_t)S, 0, R * (n + 1), ups));
        if (lone) {
            CHECK(h2d(d.top_off, pl.top_off.data(), pl.top_off.size(), ups));
            CHECK(h2d(d.top_list, pl.top_list.data(), pl.top_list.size(), ups));
            d.top_levels = pl.top_levels;
            d.n_roots = pl.n_roots;
            d.top_fast = 1;
            for (int32_t lv = 0; lv < pl.top_levels; ++lv) d.top_fast &= pl.lvl_kind[lv] != 0;
        }
        // the game's own structures for when it iterates alone
        s.top_levels[p] = lone ? pl.top_levels : 0;
        s.fuse_lo[p] = 0;
        s.fuse_hi[p] = -1;
        s.fuse_blocks[p] = 0;
        s.fuse_off[p].clear();
        s.fuse_list[p].clear();
        if (pl.fuse_hi > pl.fuse_lo && fuse_plan_ok(pl) &&
            (int64_t)pl.fuse_off.size() <= cap.fuse_off[p] &&
            (int64_t)pl.fuse_list.size() <= cap.fuse_list[p]) {
            s.fuse_lo[p] = pl.fuse_lo;
            s.fuse_hi[p] = pl.fuse_hi;
            s.fuse_blocks[p] = pl.fuse_blocks;
            s.fuse_off[p] = pl.fuse_off;
            s.fuse_list[p] = pl.fuse_list;
        }
    }
    // payoff matrix: row pointers at the row player's sequences, indices
    // shifted to the column player's global sequences (then renumbered to
    // first-touch order when the product gathers a permuted copy)
    for (int w = 0; w < 2; ++w) {
        s.ptr[w] = hg.ptr[w];
        CHECK(cp(ptr[w] + sb[w], B + img.ptr[w], 4 * hg.ptr[w].size()));
        CHECK(cp(idx[w] + nb, img.idx_src[w], 4 * (size_t)hg.nnz));
        const int32_t col_base = (int32_t)sb[1 - w];
        if (col_base != 0) CHECK(launch_add_offset(idx[w] + nb, hg.nnz, col_base, ups));
        if (perm_on[w]) CHECK(launch_remap(idx[w] + nb, hg.nnz, dp[1 - w].pos, ups));
        CHECK(cp((char *)val[w] + V * (size_t)nb, img.val_src[w], V * (size_t)hg.nnz));
    }
    // quad copies built with the image, when they match the product's
    // stream form and column order: copied like the rest (game starts are
    // multiples of four, so only the group index moves)
    for (int w = 0; w < 2; ++w) {
        const GameImage::Quads &IQ = img.quads;
        if (vec[w] != 3 || !IQ.built[w] || IQ.perm[w] != perm_on[w]) continue;
        HostTimer qtimer(&host_s[kHostQuads], &host_n[kHostQuads]);
        QuadStore &Q = quad[w];
        if (!Q.ptr) {
            if (hipMalloc((void **)&Q.ptr, 4 * (size_t)std::max<int64_t>(cap.seq[w], 1)) !=
                hipSuccess) {
                Q.ptr = nullptr;
                (void)hipGetLastError();
                continue;  // built on the device when the game joins
            }
        }
        const int64_t nq = IQ.nq[w];
        int64_t qb = 0;
        if (nq > 0) {
            qb = Q.alloc.take(nq);
            if (qb < 0) {
                if (grow_quads(w, std::max<int64_t>(Q.cap + nq, 2 * Q.cap))) continue;
                qb = Q.alloc.take(nq);
                if (qb < 0) continue;
            }
        }
        const int32_t nr = (int32_t)IQ.qptr[w].size() - 1;
        const char *QB = IQ.base;
        CHECK(cp(Q.ptr + sb[w], QB + IQ.ptr[w], 4 * ((size_t)nr + 1)));
        CHECK(cp(Q.idx + qb, QB + IQ.idx[w], 4 * (size_t)nq));
        CHECK(launch_add_offset((int32_t *)(Q.idx + qb), nq, (int32_t)(sb[1 - w] / 4), ups));
        CHECK(cp((char *)Q.val + 4 * V * (size_t)qb, QB + IQ.val[w], 4 * V * (size_t)nq));
        s.qb[w] = qb;
        s.nq[w] = nq;
        s.qptr[w] = IQ.qptr[w];
    }
    // the game's scalars: t = 0, its constants (from page-locked staging
    // when there is some)
    {
        Scalars h{};
        h.alpha = gp.alpha;
        h.beta = gp.beta;
        h.gamma = gp.gamma;
        h.variant = gp.variant;
        h.avg_kind = gp.avg_kind;
        const void *src = &h;
        if (scal_stage) {
            scal_stage[k] = h;
            src = &scal_stage[k];
        } else {
            std::vector<char> b(sizeof h);
            std::memcpy(b.data(), &h, sizeof h);
            s.staging.push_back(std::move(b));
            src = s.staging.back().data();
        }
        CHECK(cp(sc + k, src, sizeof h));
    }
    // a lone solver's game always iterates alone
    if (lone) CHECK(single_plans(k, ups));
    if (async) {
        CHECK(hipEventCreateWithFlags(&s.up_ev, hipEventDisableTiming));
        CHECK(hipEventRecord(s.up_ev, ups));
    } else {
        CHECK(hipStreamSynchronize(ups));
        s.staging.clear();
    }
#undef CHECK
    s.live = true;
    partition(s, 0);
    partition(s, 1);
    s.active = join_now;
    s.pending = !join_now;
    // a game admitted asynchronously while others iterate joins one check
    // later, so that its copies overlap that check period
    s.join_after = checks + (async && !join_now ? 1 : 0);
    if (join_now) {
        it.valid = false;
        drop_graph();
    }
    *slot_out = k;
    return CFR_OK;
}

hipError_t Engine::wait_uploads(const std::vector<int> &set)
{
    for (int k : set) {
        Slot &s = slots[(size_t)k];
        if (s.up_ev && !s.up_waited) {
            hipError_t e = hipStreamWaitEvent(st, s.up_ev, 0);
            if (e != hipSuccess) return e;
            s.up_waited = true;
        }
    }
    return hipSuccess;
}

void Engine::reap_uploads(bool wait)
{
    for (Slot &s : slots) {
        if (!s.up_ev) continue;
        if (!wait && hipEventQuery(s.up_ev) != hipSuccess) continue;
        if (wait) (void)hipEventSynchronize(s.up_ev);
        (void)hipEventDestroy(s.up_ev);
        s.up_ev = nullptr;
        s.staging.clear();
    }
}

void Engine::remove(int k)
{
    HostTimer timer(&host_s[kHostRemove], &host_n[kHostRemove]);
    Slot &s = slots[(size_t)k];
    if (!s.live) return;
    if (s.up_ev) {
        (void)hipEventSynchronize(s.up_ev);
        (void)hipEventDestroy(s.up_ev);
        s.up_ev = nullptr;
    }
    for (int p = 0; p < 2; ++p) {
        seq_alloc[p].give(s.sb[p], seq_block(s.n_seq[p]));
        inf_alloc[p].give(s.ib[p], (int64_t)s.n_inf[p] + 1);
    }
    if (s.nnz > 0) nnz_alloc.give(s.nb, s.nnz);
    for (int w = 0; w < 2; ++w) drop_quads(s, w);
    const bool was_active = s.active;
    s = Slot();
    if (was_active) {
        it.valid = false;
        drop_graph();
    }
    ev.valid = false;
}

std::vector<int> Engine::active_set() const
{
    std::vector<int> out;
    for (size_t i = 0; i < slots.size(); ++i)
        if (slots[i].live && slots[i].active) out.push_back((int)i);
    return out;
}

// Every entry stays inside its own game's ranges (what the kernels index).
bool Engine::tables_in_bounds(const Tables &T) const
{
    auto live = [&](int k) { return k >= 0 && k < (int)slots.size() && slots[(size_t)k].live; };
    for (int w = 0; w < 2; ++w) {
        const std::vector<SpmvBlock> &v = w == 0 ? T.h_csr : T.h_csc;
        const int cap_nnz = spmv_block_cap_v(items[w], vec[w]);
        const bool quads = vec[w] == 3;
        if (quads && !quad[w].idx) {
            for (const SpmvBlock &b : v)
                if (b.n > 0) return false;
        }
        for (const SpmvBlock &b : v) {
            if (!live(b.slot)) return false;
            const Slot &s = slots[(size_t)b.slot];
            if (b.nr < 1 || b.nr > kSpmvRowCap || b.n < 0 || (b.n > cap_nnz && b.nr != 1))
                return false;
            if (b.row0 < s.sb[w] || (int64_t)b.row0 + b.nr > s.sb[w] + s.n_seq[w]) return false;
            const int64_t base = quads ? s.qb[w] : s.nb, len = quads ? s.nq[w] : s.nnz;
            if (base < 0 || b.e0 < base || b.e0 + b.n > base + len) return false;
            if (b.e0 - base != b.p0) return false;
        }
    }
    for (int p = 0; p < 2; ++p) {
        for (const RangeBlock &r : T.h_up[p]) {
            if (!live(r.slot)) return false;
            const Slot &s = slots[(size_t)r.slot];
            if (r.hi - r.lo < 1 || r.hi - r.lo > kRangeBlock || r.lo < s.ib[p] ||
                r.hi > s.ib[p] + s.n_inf[p])
                return false;
        }
        for (const std::vector<RangeBlock> *v : {&T.h_down[p], &T.h_seq[p], &T.h_dall[p]})
            for (const RangeBlock &r : *v) {
                if (!live(r.slot)) return false;
                const Slot &s = slots[(size_t)r.slot];
                if (r.hi - r.lo < 1 || r.hi - r.lo > kRangeBlock || r.lo < s.sb[p] ||
                    r.hi > s.sb[p] + s.n_seq[p])
                    return false;
                if (v != &T.h_down[p] && r.aux != s.sb[p]) return false;
            }
        for (const SlotRef &r : T.h_root[p]) {
            if (!live(r.slot)) return false;
            const Slot &s = slots[(size_t)r.slot];
            if (r.root != s.sb[p] || r.a < s.ib[p] || r.b < r.a || r.b > s.ib[p] + s.n_inf[p])
                return false;
        }
    }
    for (const SlotRef &r : T.h_fin)
        if (!live(r.slot) || r.a < 0 || r.b < r.a || r.b > (int32_t)T.h_seq[0].size()) return false;
    return true;
}

int Engine::build_tables(Tables &T, char *region, const std::vector<int> &set)
{
    HostTimer timer(&host_s[kHostTables], &host_n[kHostTables]);
    (void)region;
    // the previous upload may still be in flight
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error("table upload", e);
    int qrc = ensure_quads(set);
    if (qrc) return qrc;
    const double V = (double)value_bytes(prec);
    T.h_csr.clear();
    T.h_csc.clear();
    T.h_fin.clear();
    T.bytes[0] = T.bytes[1] = 0;
    for (int k : set) {
        const Slot &s = slots[(size_t)k];
        T.h_csr.insert(T.h_csr.end(), s.blocks[0].begin(), s.blocks[0].end());
        T.h_csc.insert(T.h_csc.end(), s.blocks[1].begin(), s.blocks[1].end());
        // stream bytes: each nonzero's index and value, or each quad's
        // index and four values
        for (int w = 0; w < 2; ++w)
            T.bytes[w] += (vec[w] == 3 ? (double)s.nq[w] * (4.0 + 4.0 * V)
                                       : (double)s.nnz * (4.0 + V)) +
                          4.0 * (s.n_seq[w] + 1) + V * s.n_seq[1 - w] + V * s.n_seq[w];
    }
    std::vector<int> classes;
    for (int k : set) classes.push_back(slots[(size_t)k].gp.variant);
    std::sort(classes.begin(), classes.end());
    classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
    auto push_chunks = [](std::vector<RangeBlock> &v, int64_t lo, int64_t hi, int k, int32_t aux) {
        for (int64_t a = lo; a < hi; a += kRangeBlock)
            v.push_back(RangeBlock{(int32_t)a, (int32_t)std::min<int64_t>(hi, a + kRangeBlock), k,
                                   aux});
    };
    for (int p = 0; p < 2; ++p) {
        int maxL = 0;
        for (int k : set) maxL = std::max(maxL, (int)slots[(size_t)k].n_levels[p]);
        T.h_up[p].clear();
        T.h_down[p].clear();
        T.h_seq[p].clear();
        T.h_dall[p].clear();
        T.h_root[p].clear();
        T.dall_depth[p] = maxL;
        T.up_l[p].assign((size_t)maxL, {});
        T.up_level[p].assign((size_t)maxL, {0, 0});
        T.down_l[p].assign((size_t)maxL, {0, 0});
        for (int L = 0; L < maxL; ++L) {
            const int32_t lvl_start = (int32_t)T.h_up[p].size();
            for (int c : classes) {
                const int32_t off = (int32_t)T.h_up[p].size();
                int kind = 2;
                for (int k : set) {
                    const Slot &s = slots[(size_t)k];
                    if (s.gp.variant != c || L >= s.n_levels[p]) continue;
                    push_chunks(T.h_up[p], s.ib[p] + s.lvl_inf[p][L], s.ib[p] + s.lvl_inf[p][L + 1],
                                k, s.lvl_slots[p][L]);
                    kind = std::min(kind, (int)s.lvl_kind[p][L]);
                }
                const int32_t n = (int32_t)T.h_up[p].size() - off;
                // a launch over one game's level: its range goes by value
                RangeBlock dr{0, 0, 0, 0};
                if (set.size() == 1) {
                    const Slot &s = slots[(size_t)set[0]];
                    dr = RangeBlock{(int32_t)(s.ib[p] + s.lvl_inf[p][L]),
                                    (int32_t)(s.ib[p] + s.lvl_inf[p][L + 1]), set[0],
                                    (int32_t)s.lvl_slots[p][L]};
                }
                if (n > 0) T.up_l[p][L].push_back(Tables::Up{off, n, c, kind, dr});
            }
            T.up_level[p][L] = {lvl_start, (int32_t)T.h_up[p].size() - lvl_start};
            if (L > 0) {
                const int32_t off = (int32_t)T.h_down[p].size();
                for (int k : set) {
                    const Slot &s = slots[(size_t)k];
                    if (L >= s.n_levels[p]) continue;
                    push_chunks(T.h_down[p], s.sb[p] + s.lvl_seq[p][L], s.sb[p] + s.lvl_seq[p][L + 1],
                                k, 0);
                }
                T.down_l[p][L] = {off, (int32_t)T.h_down[p].size() - off};
            }
        }
        for (int k : set) {
            const Slot &s = slots[(size_t)k];
            const int32_t first = (int32_t)T.h_seq[p].size();
            push_chunks(T.h_seq[p], s.sb[p], s.sb[p] + s.n_seq[p], k, (int32_t)s.sb[p]);
            if (s.n_levels[p] > 1)
                push_chunks(T.h_dall[p], s.sb[p] + s.lvl_seq[p][1], s.sb[p] + s.n_seq[p], k,
                            (int32_t)s.sb[p]);
            if (p == 0) T.h_fin.push_back(SlotRef{k, 0, first, (int32_t)T.h_seq[p].size()});
            const int32_t j0 = s.n_levels[p] > 0 ? s.lvl_inf[p][0] : 0;
            const int32_t j1 = s.n_levels[p] > 0 ? s.lvl_inf[p][1] : 0;
            T.h_root[p].push_back(
                SlotRef{k, (int32_t)s.sb[p], (int32_t)(s.ib[p] + j0), (int32_t)(s.ib[p] + j1)});
        }
        if ((int64_t)T.h_up[p].size() > cap.t_up[p] || (int64_t)T.h_down[p].size() > cap.t_down[p] ||
            (int64_t)T.h_seq[p].size() > cap.t_seq[p] || (int64_t)T.h_dall[p].size() > cap.t_dall[p])
            return fail(CFR_EINVAL, "internal: sweep tables exceed their capacity");
        T.n_seq[p] = (int32_t)T.h_seq[p].size();
        T.n_dall[p] = (int32_t)T.h_dall[p].size();
        T.dall_direct[p] = RangeBlock{0, 0, 0, 0};
        if (set.size() == 1) {
            const Slot &s = slots[(size_t)set[0]];
            if (s.n_levels[p] > 1)
                T.dall_direct[p] = RangeBlock{(int32_t)(s.sb[p] + s.lvl_seq[p][1]),
                                              (int32_t)(s.sb[p] + s.n_seq[p]), set[0],
                                              (int32_t)s.sb[p]};
        }
        T.n_root[p] = (int32_t)T.h_root[p].size();
    }
    if ((int64_t)T.h_csr.size() > cap.t_csr || (int64_t)T.h_csc.size() > cap.t_csc)
        return fail(CFR_EINVAL, "internal: product tables exceed their capacity");
    T.n_csr = (int32_t)T.h_csr.size();
    T.n_csc = (int32_t)T.h_csc.size();
    T.n_fin = (int32_t)T.h_fin.size();
    if (!tables_in_bounds(T)) return fail(CFR_EINVAL, "internal: a table entry leaves its game");
    e = h2d(T.csr, T.h_csr.data(), T.h_csr.size(), st);
    if (e == hipSuccess) e = h2d(T.csc, T.h_csc.data(), T.h_csc.size(), st);
    for (int p = 0; p < 2 && e == hipSuccess; ++p) {
        e = h2d(T.up[p], T.h_up[p].data(), T.h_up[p].size(), st);
        if (e == hipSuccess) e = h2d(T.down[p], T.h_down[p].data(), T.h_down[p].size(), st);
        if (e == hipSuccess) e = h2d(T.seq[p], T.h_seq[p].data(), T.h_seq[p].size(), st);
        if (e == hipSuccess) e = h2d(T.dall[p], T.h_dall[p].data(), T.h_dall[p].size(), st);
        if (e == hipSuccess) e = h2d(T.root[p], T.h_root[p].data(), T.h_root[p].size(), st);
    }
    if (e == hipSuccess) e = h2d(T.fin, T.h_fin.data(), T.h_fin.size(), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_error("table upload", e);
    T.valid = true;
    return CFR_OK;
}

int Engine::rebuild()
{
    drop_graph();
    const std::vector<int> act = active_set();
    hipError_t e = wait_uploads(act);
    if (e != hipSuccess) return device_error("admission copies", e);
    int rc = build_tables(it, tab_region[0], act);
    if (rc) {
        it.valid = false;
        return rc;
    }
    // a batch whose only iterating game can use that game's own structures
    if (!lone) {
        e = single_plans(act.size() == 1 ? act[0] : -1, st);
        if (e != hipSuccess) {
            it.valid = false;
            return device_error("fused-level lists", e);
        }
    }
    return CFR_OK;
}

hipError_t Engine::single_plans(int k, hipStream_t s)
{
    single_slot = -1;
    for (int p = 0; p < 2; ++p) {
        dp[p].shallow = ShallowPlan();
        dp[p].fuse = FusePlan();
    }
    if (k < 0 || up_pass != CFR_UP_DEFAULT) return hipSuccess;
    const Slot &g = slots[(size_t)k];
    single_slot = k;
    for (int p = 0; p < 2; ++p) {
        DevPlayer &d = dp[p];
        if (g.top_levels[p] > 0) continue;  // k_top takes the shallow levels
        const int32_t I = (int32_t)g.ib[p], L = g.n_levels[p];
        const std::vector<int32_t> &li = g.lvl_inf[p];
        const std::vector<uint8_t> &kind = g.lvl_kind[p];
        // the shallow levels in one block: from the root down while they are
        // small and on the fast path (two levels at least, or nothing is
        // gained), the deepest of them reading value slots unless it is the
        // game's last level
        int32_t T = 0;
        while (T < L && T < kShallowLevels && kind[(size_t)T] != 0 && li[(size_t)T + 1] <= kShallowMax)
            ++T;
        if (T >= 2 && T < L && !(g.lvl_slots[p][(size_t)T - 1] & kSlotsRead)) T = 0;
        if (T >= 2) {
            d.shallow.levels = T;
            for (int32_t lv = 0; lv <= T; ++lv) d.shallow.lo[lv] = I + li[(size_t)lv];
            for (int32_t lv = 0; lv < T; ++lv) d.shallow.kind[lv] = kind[(size_t)lv];
        }
        // the fused levels below them; the shallowest stores its values as
        // the level above reads them, the deepest reads its children's
        // values as the level below stores them
        const int32_t T0 = g.fuse_lo[p], T1 = g.fuse_hi[p];
        if (T1 > T0 && d.shallow.levels <= T0) {
            hipError_t e = h2d(d.fuse_off, g.fuse_off[p].data(), g.fuse_off[p].size(), s);
            if (e == hipSuccess) e = h2d(d.fuse_list, g.fuse_list[p].data(), g.fuse_list[p].size(), s);
            if (e != hipSuccess) return e;
            d.fuse.levels = T1 - T0 + 1;
            d.fuse.lo = T0;
            d.fuse.base = I;
            d.fuse.blocks = g.fuse_blocks[p];
            d.fuse.top_slots = (g.lvl_slots[p][(size_t)T0] & kSlotsWrite) ? 1 : 0;
            d.fuse.deep_read = kind[(size_t)T1] == 2 ? 0
                               : (g.lvl_slots[p][(size_t)T1] & kSlotsRead) ? 1 : 2;
        }
    }
    return hipSuccess;
}

hipError_t Engine::spmv(const Tables &T, int which, const void *xin, void *yout, bool begin,
                        hipStream_t s, bool timed, bool gathered)
{
    const SpmvBlock *tab = which == 0 ? T.csr : T.csc;
    const int32_t n = which == 0 ? T.n_csr : T.n_csc;
    if (perm_on[which]) {
        // the product reads the gathered player's vector in first-touch order
        const int q = 1 - which;
        if (!gathered) {
            hipError_t e = launch_gather(prec, T.seq[q], T.n_seq[q], dp[q].perm, xin, dp[q].xp, s);
            if (e != hipSuccess) return e;
        }
        xin = dp[q].xp;
    }
    const bool quads = vec[which] == 3;
    const int remap = xcd_remap[which];
    const int32_t *rp = quads ? quad[which].ptr : ptr[which];
    const int32_t *ix = quads ? (const int32_t *)quad[which].idx : idx[which];
    const void *vl = quads ? quad[which].val : val[which];
    if (timed) {
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
        e = launch_spmv(prec, items[which], vec[which], tab, n, rp, ix, vl, xin, yout, remap,
                        sequential(), begin ? 1 : 0, sc, s, a, b);
        events[which].emplace_back(a, b);
        launches[which]++;
        return e;
    }
    return launch_spmv(prec, items[which], vec[which], tab, n, rp, ix, vl, xin, yout, remap,
                       sequential(), begin ? 1 : 0, sc, s);
}

hipError_t Engine::sweeps(const Tables &T, int p, double usign, hipStream_t s, bool *fold)
{
    const DevPlayer &d = dp[p];
    const int maxL = (int)T.up_l[p].size();
    hipError_t e;
    const bool top = lone && d.top_levels > 0;
    // the one-block shallow pass and the fused levels belong to the game
    // iterating alone (set by single_plans), with its own scalars
    const int one = single_slot;
    const int shallow = !top && one >= 0 ? d.shallow.levels : 0;
    const int low = top ? d.top_levels : shallow;
    // ObserveUtility, deepest level first (level 0's launch also does its
    // top-down step); with CFR_UP_PAIRS a lone game runs pairs of adjacent
    // levels that fit the two-level launch as one launch each
    const bool pairs = lone && up_pass == CFR_UP_PAIRS && !slots.empty() && slots[0].live;
    const bool fuse = !top && one >= 0 && up_pass == CFR_UP_DEFAULT && d.fuse.levels >= 2 &&
                      d.fuse.lo >= low;
    for (int L = maxL - 1; L >= low;) {
        if (fuse && L == d.fuse.lo + d.fuse.levels - 1) {
            // the fused levels, one launch
            if ((e = launch_fuse(prec, slots[(size_t)one].gp.variant, d, usign, sc + one, s)) !=
                hipSuccess)
                return e;
            L = d.fuse.lo - 1;
            continue;
        }
        const auto &lo = T.up_l[p][(size_t)L];
        if (pairs && L - 1 >= low && slots[0].lvl_pair[p][(size_t)L] && lo.size() == 1 &&
            T.up_l[p][(size_t)L - 1].size() == 1) {
            const Slot &g = slots[0];
            const Tables::Up &up = T.up_l[p][(size_t)L - 1][0];
            if ((e = launch_up_pair(prec, up.variant, g.lvl_kind[p][(size_t)L],
                                    g.lvl_slots[p][(size_t)L] & kSlotsRead,
                                    g.lvl_slots[p][(size_t)L - 1] & kSlotsWrite, L - 1 == 0 ? 1 : 0,
                                    up.direct, d, usign, sc, s)) != hipSuccess)
                return e;
            L -= 2;
            continue;
        }
        for (const Tables::Up &u : lo)
            if ((e = launch_up(prec, u.variant, u.kind, L == 0 ? 1 : 0, T.up[p] + u.off, u.n,
                               &u.direct, d,
                               usign, sc, s)) != hipSuccess)
                return e;
        --L;
    }
    if (top) {
        // the shallow levels of the lone game, both directions, one launch
        if ((e = launch_top(prec, slots[0].gp.variant, d, usign, 1, sc, s)) != hipSuccess) return e;
    } else if (shallow > 0) {
        // the shallow levels' bottom-up pass in one block (level 0 does its
        // top-down step there too)
        if ((e = launch_shallow(prec, slots[(size_t)one].gp.variant, d, usign, sc + one, s)) !=
            hipSuccess)
            return e;
    }
    if (!top && down_pass == CFR_DOWN_DEFAULT && T.dall_depth[p] <= kDownAllMaxDepth) {
        const RangeBlock &dr = T.dall_direct[p];
        if (fold && dr.hi > dr.lo) {
            // from the game's empty sequence on, writing the permuted copy too
            *fold = true;
            const RangeBlock all{dr.aux, dr.hi, dr.slot, dr.aux};
            return launch_down_all(prec, T.dall_depth[p], T.dall[p], T.n_dall[p], &all, d, 1, sc,
                                   s, 1, dr.lo);
        }
        return launch_down_all(prec, T.dall_depth[p], T.dall[p], T.n_dall[p], &dr, d, 1, sc, s);
    }
    // one launch per level below the levels whose top-down pass is done:
    // k_top's, else level 0 (its bottom-up launch, the one-block shallow
    // pass or a fused launch from level 0 does its step)
    for (int L = top ? std::max(d.top_levels, 1) : 1; L < maxL; ++L) {
        const auto &dl = T.down_l[p][(size_t)L];
        if ((e = launch_down(prec, T.down[p] + dl.first, dl.second, d, 1, sc, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t Engine::enqueue_iteration(hipStream_t s)
{
    hipError_t e;
    const bool timed = timing && s == st;
    if (mode == CFR_SIMULTANEOUS) {
        // both products read the strategies of iteration t before either
        // player moves on
        if ((e = spmv(it, 0, dp[1].x, dp[0].g, true, s, timed)) != hipSuccess) return e;
        if ((e = spmv(it, 1, dp[0].x, dp[1].g, false, s, timed)) != hipSuccess) return e;
        if ((e = sweeps(it, 0, 1.0, s)) != hipSuccess) return e;
        return sweeps(it, 1, -1.0, s);
    }
    // player 1's top-down pass, right before the product that reads its
    // strategy, may write the permuted copy that product gathers from
    bool folded = false;
    if ((e = spmv(it, 0, dp[1].x, dp[0].g, true, s, timed)) != hipSuccess) return e;
    if ((e = sweeps(it, 0, 1.0, s, perm_on[1] ? &folded : nullptr)) != hipSuccess) return e;
    if ((e = spmv(it, 1, dp[0].x, dp[1].g, false, s, timed, folded)) != hipSuccess) return e;
    return sweeps(it, 1, -1.0, s);
}

hipError_t Engine::build_graph()
{
    HostTimer timer(&host_s[kHostGraph], &host_n[kHostGraph]);
    hipError_t e = hipSuccess;
    if (!cap_st) {
        e = hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    e = hipStreamBeginCapture(cap_st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e2 = enqueue_iteration(cap_st);
    e = hipStreamEndCapture(cap_st, &graph);
    if (e2 != hipSuccess) return e2;
    if (e != hipSuccess) return e;
    return hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
}

int Engine::iterate(int64_t n)
{
    if (n <= 0) return CFR_OK;
    if (mode != CFR_SIMULTANEOUS && mode != CFR_ALTERNATING)
        return fail(CFR_ESTATE, "update mode not set");
    if (!it.valid) {
        int rc = rebuild();
        if (rc) return rc;
    }
    const std::vector<int> act = active_set();
    if (act.empty()) return CFR_OK;
    for (int k : act)
        if (slots[(size_t)k].gp.variant < CFR_VANILLA)
            return fail(CFR_ESTATE, "a game has no regret minimiser set");
    hipError_t e = hipSuccess;
    // Capturing and instantiating the iteration's graph costs about as much
    // host time as launching twenty iterations directly.  A batch's set of
    // games often changes at every check, so the first short run after a
    // change launches directly and the graph is built only when the same
    // set runs again (or for a long run).  A lone solver's set never
    // changes: it captures at once.
    constexpr int64_t kGraphNow = 32;
    if (use_graph && !timing && !gexec && !lone && n < kGraphNow && direct_runs == 0) {
        ++direct_runs;
        HostTimer timer(&host_s[kHostEnqueue], &host_n[kHostEnqueue]);
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) e = enqueue_iteration(st);
    } else if (use_graph && !timing) {
        if (!gexec) {
            e = build_graph();
            if (e != hipSuccess) {
                drop_graph();
                return device_error("graph capture of one iteration", e);
            }
        }
        HostTimer timer(&host_s[kHostEnqueue], &host_n[kHostEnqueue]);
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) e = hipGraphLaunch(gexec, st);
    } else {
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) e = enqueue_iteration(st);
    }
    if (e != hipSuccess) return device_error("iteration launch", e);
    for (int k : act) slots[(size_t)k].t += n;
    return CFR_OK;
}

int Engine::evaluate_launch(const std::vector<int> &set, int kind, Scalars *out)
{
    const Tables *T = nullptr;
    if (it.valid && set == active_set()) {
        T = &it;
    } else {
        if (!(ev.valid && ev_set == set)) {
            ev.valid = false;
            int rc = build_tables(ev, tab_region[1], set);
            if (rc) return rc;
            ev_set = set;
        }
        T = &ev;
    }
    hipError_t e = hipSuccess;
#define CHECK(x)                                                     \
    do {                                                             \
        e = (x);                                                     \
        if (e != hipSuccess) return device_error("evaluation", e);   \
    } while (0)
    e = wait_uploads(set);
    if (e != hipSuccess) return device_error("admission copies", e);
    const void *src[2] = {dp[0].x, dp[1].x};
    if (kind == CFR_AVERAGE) {
        for (int p = 0; p < 2; ++p) {
            CHECK(launch_normalize(prec, T->seq[p], T->n_seq[p], dp[p], sc, st));
            src[p] = dp[p].xbar;
        }
    }
    CHECK(spmv(*T, 0, src[1], dp[0].g, false, st, false));
    CHECK(spmv(*T, 1, src[0], dp[1].g, false, st, false));
    for (int p = 0; p < 2; ++p) {
        const double usign = p == 0 ? 1.0 : -1.0;
        for (int L = (int)T->up_level[p].size() - 1; L >= 0; --L) {
            const auto &ul = T->up_level[p][(size_t)L];
            CHECK(launch_br(prec, T->up[p] + ul.first, ul.second, dp[p], usign, st));
        }
        CHECK(launch_root_value(prec, T->root[p], T->n_root[p], dp[p], usign, sc, p, st));
    }
    CHECK(launch_dot(prec, T->seq[0], T->n_seq[0], src[0], dp[0].g, partials, T->fin, T->n_fin,
                     sc, 2, st));
    CHECK(hipMemcpyAsync(out, sc, sizeof(Scalars) * slots.size(), hipMemcpyDeviceToHost, st));
#undef CHECK
    return CFR_OK;
}

void Engine::evaluate_collect(const std::vector<int> &set, const Scalars *out)
{
    reap_uploads(false);
    for (int k : set) {
        Slot &s = slots[(size_t)k];
        const double br1 = out[(size_t)k].out[0], br2 = out[(size_t)k].out[1];
        s.last[0] = (br1 + br2) / 2.0;
        s.last[1] = br1 + br2;
        s.last[2] = br1;
        s.last[3] = br2;
        s.last[4] = out[(size_t)k].out[2];
        s.last_t = s.t;
    }
}

int Engine::evaluate(const std::vector<int> &set, int kind)
{
    if (set.empty()) return CFR_OK;
    HostTimer timer(&host_s[kHostEval], &host_n[kHostEval]);
    std::vector<Scalars> h(slots.size());
    int rc = evaluate_launch(set, kind, h.data());
    if (rc) return rc;
    rc = sync("evaluation");
    if (rc) return rc;
    evaluate_collect(set, h.data());
    return CFR_OK;
}

void Engine::apply_check(const std::vector<int> &set)
{
    bool changed = false;
    for (int k : set) {
        Slot &s = slots[(size_t)k];
        const bool hit = s.gp.target > 0 && s.last[0] <= s.gp.target;
        if (hit) s.reached = true;
        if (hit || (s.gp.max_it > 0 && s.t >= s.gp.max_it)) {
            s.active = false;
            changed = true;
        }
    }
    if (changed) {
        it.valid = false;
        drop_graph();
    }
}

// At a check boundary: games admitted since the last check join now (or,
// admitted asynchronously, once their copies had a check period).
static void join_pending(Engine &eng)
{
    bool joined = false;
    const bool idle = eng.active_set().empty();
    for (Slot &s : eng.slots)
        if (s.live && s.pending && (idle || s.join_after <= eng.checks)) {
            s.pending = false;
            s.active = true;
            joined = true;
        }
    if (joined) {
        eng.it.valid = false;
        eng.drop_graph();
    }
}

int Engine::run(int64_t n)
{
    if (pending) return fail(CFR_ESTATE, "a check period begun asynchronously has not ended");
    int64_t done = 0;
    while (done < n) {
        if (phase == 0) join_pending(*this);
        const std::vector<int> act = active_set();
        if (act.empty()) break;
        const int64_t chunk =
            check_every > 0 ? std::min(check_every - phase, n - done) : n - done;
        int rc = iterate(chunk);
        if (rc) return rc;
        done += chunk;
        if (check_every <= 0) continue;
        phase += chunk;
        if (phase < check_every) continue;
        phase = 0;
        ++checks;
        rc = evaluate(act, CFR_AVERAGE);
        if (rc) return rc;
        apply_check(act);
    }
    return CFR_OK;
}

int Engine::run_begin()
{
    if (pending) return fail(CFR_ESTATE, "a check period is already running");
    if (check_every <= 0) return fail(CFR_ESTATE, "no check period");
    if (!eval_stage || !eval_ev)
        return fail(CFR_EUNSUPPORTED, "no page-locked staging for asynchronous checks");
    if (phase == 0) join_pending(*this);
    const std::vector<int> act = active_set();
    if (act.empty()) return CFR_OK;
    const int64_t chunk = check_every - phase;
    int rc = iterate(chunk);
    if (rc) return rc;
    phase = 0;
    ++checks;
    HostTimer timer(&host_s[kHostEval], &host_n[kHostEval]);
    rc = evaluate_launch(act, CFR_AVERAGE, eval_stage);
    if (rc) return rc;
    hipError_t e = hipEventRecord(eval_ev, st);
    if (e != hipSuccess) return device_error("check event", e);
    pending = true;
    pending_set = act;
    return CFR_OK;
}

int Engine::run_ready()
{
    if (!pending) return 1;
    const hipError_t e = hipEventQuery(eval_ev);
    if (e == hipErrorNotReady) return 0;
    // completed, or failed: run_end reports a failure
    (void)hipGetLastError();
    return 1;
}

int Engine::run_end()
{
    if (!pending) return CFR_OK;
    pending = false;
    hipError_t e = hipEventSynchronize(eval_ev);
    if (e != hipSuccess) return device_error("check period", e);
    evaluate_collect(pending_set, eval_stage);
    apply_check(pending_set);
    pending_set.clear();
    return CFR_OK;
}

int Engine::time_spmv(int which, int reps, double *ms)
{
    if (!it.valid) {
        int rc = rebuild();
        if (rc) return rc;
    }
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return device_error("event", e);
    const void *xin = which == 0 ? dp[1].x : dp[0].x;
    void *yout = which == 0 ? dp[0].g : dp[1].g;
    // one untimed launch, then `reps` timed ones
    e = spmv(it, which, xin, yout, false, st, false);
    if (e == hipSuccess) e = hipEventRecord(a, st);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = spmv(it, which, xin, yout, false, st, false);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return device_error("product timing", e);
    *ms = (double)t / std::max(reps, 1);
    return CFR_OK;
}

int Engine::fetch_vector(int k, int player, int what, std::vector<double> &out)
{
    const Slot &s = slots[(size_t)k];
    const size_t n = (size_t)s.n_seq[player];
    const int64_t S = s.sb[player];
    out.assign(n, 0.0);
    const bool acc = what != 0;  // regrets and averages live in the accumulator type
    const size_t el = acc ? accum_bytes(prec) : value_bytes(prec);
    const void *src = what == 0 ? dp[player].x : what == 1 ? dp[player].s : dp[player].r;
    std::vector<char> h(n * el);
    Scalars hs{};
    hipError_t e = wait_uploads({k});
    if (e != hipSuccess) return device_error("admission copies", e);
    e = hipMemcpyAsync(h.data(), (const char *)src + el * (size_t)S, n * el,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && what == 1)
        e = hipMemcpyAsync(&hs, sc + k, sizeof hs, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return device_error("device-to-host copy", e);
    int rc = sync("device-to-host copy");
    if (rc) return rc;
    auto load = [&](size_t i) -> double {
        if (el == 8) {
            double v;
            std::memcpy(&v, h.data() + i * 8, 8);
            return v;
        }
        float v;
        std::memcpy(&v, h.data() + i * 4, 4);
        return (double)v;
    };
    if (what == 1 && hs.W <= 0) return fetch_vector(k, player, 0, out);  // no iteration yet
    for (size_t i = 0; i < n; ++i) {
        double v = load(i);
        if (what == 1) v = i == 0 ? 1.0 : v / hs.W;
        if (what == 2 && i == 0) v = 0.0;
        out[(size_t)s.old_of_new[player][i]] = v;
    }
    return CFR_OK;
}

}  // namespace cfr
