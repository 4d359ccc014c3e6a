// C ABI of libcfr (declared in include/cfr.h): host validation, the
// single-game solver and the batch of games, both on top of the engine in
// cfr_engine.hip.
//
// cfr_create validates the game on the host, renumbers each treeplex into
// level order, lays out one device workspace of exactly the game's size,
// copies the game once and puts both players at the uniform strategy.
// cfr_step then only enqueues kernels (or replays a captured graph of one
// iteration) on the caller's stream; the only host/device crossings are the
// copies in cfr_strategy, cfr_regrets and cfr_exploitability, which wait
// for the stream.  When the caller's numbering already is level order (the
// generator emits it), nothing is permuted and the payoff arrays are used
// as given.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "cfr.h"
#include "cfr_engine.h"

using cfr::fail;
using cfr::hip_msg;

namespace {

// ---------------------------------------------------------------------------
// Host validation
// ---------------------------------------------------------------------------

int validate_player(const cfr_player_desc &p, int who)
{
    char buf[256];
    const int64_t kMax = std::numeric_limits<int32_t>::max();
    if (p.n_seq < 1 || p.n_seq > kMax - 1) {
        snprintf(buf, sizeof buf, "player %d: n_seq=%lld out of range [1, INT32_MAX)", who + 1,
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
        cfr::transpose(g->player[0].n_seq, g->player[1].n_seq, g->row_ptr, g->col_idx, g->val, tp,
                       ti, tv);
        int64_t n2 = g->player[1].n_seq;
        if (std::memcmp(tp.data(), g->col_ptr, sizeof(int64_t) * (size_t)(n2 + 1)) != 0 ||
            (g->nnz > 0 &&
             (std::memcmp(ti.data(), g->row_idx, sizeof(int32_t) * (size_t)g->nnz) != 0 ||
              std::memcmp(tv.data(), g->val_csc, sizeof(double) * (size_t)g->nnz) != 0)))
            return fail(CFR_EINVAL, "csc is not the exact transpose of the csr");
    }
    return CFR_OK;
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
    if (o->down_pass != CFR_DOWN_DEFAULT && o->down_pass != CFR_DOWN_LEVELS)
        return fail(CFR_EINVAL, "unknown top-down pass");
    if (o->up_pass != CFR_UP_DEFAULT && o->up_pass != CFR_UP_LEVELS && o->up_pass != CFR_UP_PAIRS)
        return fail(CFR_EINVAL, "unknown bottom-up pass");
    if (!std::isfinite(o->dcfr_alpha) || !std::isfinite(o->dcfr_beta) ||
        !std::isfinite(o->dcfr_gamma))
        return fail(CFR_EINVAL, "DCFR exponents must be finite");
    return CFR_OK;
}

int check_game_params(const cfr_game_params *gp)
{
    if (!gp) return fail(CFR_EINVAL, "null game parameters");
    if (gp->variant < CFR_VANILLA || gp->variant > CFR_PCFR) return fail(CFR_EINVAL, "unknown variant");
    if (gp->avg_weight < CFR_AVG_DEFAULT || gp->avg_weight > CFR_AVG_POW_GAMMA)
        return fail(CFR_EINVAL, "unknown averaging weight");
    if (!std::isfinite(gp->dcfr_alpha) || !std::isfinite(gp->dcfr_beta) ||
        !std::isfinite(gp->dcfr_gamma))
        return fail(CFR_EINVAL, "DCFR exponents must be finite");
    if (!(gp->target_exploitability >= 0) || gp->max_iterations < 0)
        return fail(CFR_EINVAL, "target and iteration limit must be non-negative");
    return CFR_OK;
}

int check_tiling(const cfr_spmv_tiling *t)
{
    if (!t) return fail(CFR_EINVAL, "null tiling");
    for (int w = 0; w < 2; ++w) {
        if (!cfr::spmv_items_supported(t->items[w]))
            return fail(CFR_EINVAL, "nonzeros per thread must be 4, 8 or 16");
        if (t->rows[w] < 64 || t->rows[w] > cfr::kSpmvRowCap)
            return fail(CFR_EINVAL, "rows per block must be in [64, 256]");
        if (t->vec[w] < 0 || t->vec[w] > 3) return fail(CFR_EINVAL, "vec must be 0, 1, 2 or 3");
        if (t->vec[w] == 3 && t->items[w] < cfr::kQuadItemsMin)
            return fail(CFR_EINVAL, "stream form 3 takes 8 or 16 nonzeros per thread");
        if (t->perm[w] != 0 && t->perm[w] != 1) return fail(CFR_EINVAL, "perm must be 0 or 1");
        if (t->xcd[w] != 0 && t->xcd[w] != 1) return fail(CFR_EINVAL, "xcd must be 0 or 1");
    }
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

int check_device(int device)
{
    int n_dev = 0;
    hipError_t e = hipGetDeviceCount(&n_dev);
    if (e != hipSuccess || n_dev <= 0) return fail(CFR_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n_dev) return fail(CFR_EINVAL, "device out of range");
    return CFR_OK;
}

// Stream form 3 only where the column player's index space fits a quad word.
int check_tiling_fits(const cfr::Engine &e, const cfr_spmv_tiling *t)
{
    if (e.no_alloc && (t->vec[0] == 3 || t->vec[1] == 3))
        return fail(CFR_EUNSUPPORTED, "stream form 3 allocates its quad copies; a solver made by "
                                      "cfr_create_static cannot use it");
    for (int w = 0; w < 2; ++w)
        if (t->vec[w] == 3 && !cfr::quads_fit(e.cap.seq[1 - w]))
            return fail(CFR_EINVAL, "stream form 3 needs every column index below 2^30 (the "
                                    "column player's sequence capacity is larger)");
    return CFR_OK;
}

// Tiling choice shared by the solver and the batch.
void get_tiling(const cfr::Engine &e, cfr_spmv_tiling *t)
{
    for (int w = 0; w < 2; ++w) {
        t->items[w] = e.items[w];
        t->rows[w] = e.rows[w];
        t->vec[w] = e.vec[w];
        t->perm[w] = e.perm_on[w];
        t->xcd[w] = e.xcd_remap[w];
    }
}

int set_tiling(cfr::Engine &e, const cfr_spmv_tiling *t)
{
    for (int w = 0; w < 2; ++w) {
        int rc = e.set_perm(w, t->perm[w]);
        if (rc) return rc;
        if (e.xcd_remap[w] != t->xcd[w]) {
            e.xcd_remap[w] = t->xcd[w];
            e.drop_graph();
        }
        e.repartition(w, t->items[w], t->rows[w], t->vec[w]);
    }
    return CFR_OK;
}

// The autotuner: every candidate tiling of each product, timed on the
// engine's iterating games, the fastest kept.
int tune(cfr::Engine &e, int reps, cfr_spmv_tiling *chosen)
{
    if (reps < 1) return fail(CFR_EINVAL, "reps must be >= 1");
    static const int kItems[] = {4, 8, 16};
    static const int kRows[] = {64, 128, 256};
    // The current tiling is the incumbent; another replaces it only when
    // more than 2% faster, so that timing noise between near-equal tilings
    // does not flip the choice from run to run.
    for (int w = 0; w < 2; ++w) {
        int bi = e.items[w], br = e.rows[w], bv = e.vec[w], bp = e.perm_on[w];
        double best = -1;
        {
            int rc = e.time_spmv(w, reps, &best);
            if (rc) return rc;
            best *= 0.98;
        }
        for (int perm = 0; perm < 2; ++perm) {
            int rc = e.set_perm(w, perm);
            if (rc) return rc;
            for (int vec = 0; vec < 4; ++vec)
                for (int items : kItems)
                    for (int rows : kRows) {
                        if (vec == 3 && (items < cfr::kQuadItemsMin ||
                                         !cfr::quads_fit(e.cap.seq[1 - w])))
                            continue;
                        e.repartition(w, items, rows, vec);
                        double ms = 0;
                        rc = e.time_spmv(w, reps, &ms);
                        if (rc) return rc;
                        if (ms < best) {
                            best = ms;
                            bi = items;
                            br = rows;
                            bv = vec;
                            bp = perm;
                        }
                    }
        }
        int rc = e.set_perm(w, bp);
        if (rc) return rc;
        e.repartition(w, bi, br, bv);
        // the block order of the winner, with the same hysteresis
        {
            double cur = 0, alt = 0;
            rc = e.time_spmv(w, reps, &cur);
            if (rc) return rc;
            e.xcd_remap[w] ^= 1;
            e.drop_graph();
            rc = e.time_spmv(w, reps, &alt);
            if (rc) return rc;
            if (!(alt < 0.98 * cur)) {
                e.xcd_remap[w] ^= 1;
                e.drop_graph();
            }
        }
    }
    if (chosen) get_tiling(e, chosen);
    return CFR_OK;
}

int kernel_timing(cfr::Engine &e, int enable)
{
    int rc = e.sync("kernel timing");
    if (rc) return rc;
    for (int k = 0; k < 2; ++k) {
        for (auto &pr : e.events[k]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        e.events[k].clear();
        e.launches[k] = 0;
        e.total_ms[k] = 0;
    }
    e.timing = enable != 0;
    return CFR_OK;
}

int kernel_stats(cfr::Engine &e, int kernel, int64_t *launches, double *total_ms,
                 double *bytes_per_launch)
{
    int rc = e.sync("kernel stats");
    if (rc) return rc;
    for (auto &pr : e.events[kernel]) {
        float ms = 0;
        hipError_t err = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (err != hipSuccess) return e.device_error("event timing", err);
        e.total_ms[kernel] += ms;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    e.events[kernel].clear();
    if (launches) *launches = e.launches[kernel];
    if (total_ms) *total_ms = e.total_ms[kernel];
    if (bytes_per_launch) *bytes_per_launch = e.it.valid ? e.it.bytes[kernel] : 0.0;
    return CFR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Single-game solver
// ---------------------------------------------------------------------------

struct cfr_solver {
    cfr::Engine eng;
    int variant = -1, mode = -1;
};

namespace {

// Device bytes of a lone solver for this (validated) game.
size_t lone_bytes(const cfr_game_desc *game, int precision)
{
    cfr::HostGame hg;
    cfr::prepare_game(game, true, false, hg);
    const cfr::Capacity c = cfr::lone_capacity(hg, cfr::kSpmvItemsDefault, cfr::kSpmvRowCap,
                                               cfr::kSpmvItemsDefault, cfr::kSpmvRowCap);
    return cfr::engine_bytes(c, precision);
}

// cfr_create after validation, on the current device: the solver's state
// in `ws` (ws_bytes long), or in a workspace it allocates when ws is null.
// no_alloc: the solver allocates nothing on the device or in page-locked
// memory, now or later (no upload stream, no staging, no graph).
int create_lone(const cfr_game_desc *game, const cfr_options *opt, void *ws, size_t ws_bytes,
                bool no_alloc, cfr_solver **out)
{
    cfr_solver *s = new cfr_solver();
    cfr::Engine &e = s->eng;
    e.spmv_order = opt->spmv_order;
    e.use_graph = !no_alloc && opt->use_graph != 0;
    e.no_alloc = no_alloc;
    e.down_pass = opt->down_pass;
    e.up_pass = opt->up_pass;
    e.lone = true;
    int rc = CFR_OK;
    try {
        cfr::HostGame hg;
        cfr::prepare_game(game, true, true, hg);
        cfr::GameImage img;
        cfr::build_image(hg, opt->precision, false, true, img);
        const cfr::Capacity c = cfr::lone_capacity(hg, e.items[0], e.rows[0], e.items[1],
                                                   e.rows[1]);
        rc = e.init(c, opt->precision, opt->device, (hipStream_t)opt->stream, ws, ws_bytes);
        if (!rc) {
            cfr::GameParams gp;
            gp.variant = -1;
            gp.avg_kind = opt->avg_weight;
            gp.alpha = opt->dcfr_alpha;
            gp.beta = opt->dcfr_beta;
            gp.gamma = opt->dcfr_gamma;
            int slot = -1;
            rc = e.add(hg, img, gp, true, false, &slot);
        }
    } catch (...) {
        s->eng.release();
        delete s;
        throw;
    }
    if (rc) {
        s->eng.release();
        delete s;
        return rc;
    }
    *out = s;
    return CFR_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free solvers (cfr_create_static)
// ---------------------------------------------------------------------------
// Their device state lives in this array instead of in memory the library
// allocates.  Each GPU holds its own copy from the library's first use on
// that GPU until the process ends.  In host code the name stands for a
// host-side shadow, not a device address: the device address is taken once
// per device with hipGetSymbolAddress (static_slot) and only that address
// is handed to the engine, and from there to kernels and copies.
__device__ __align__(256) unsigned char scratch[CFR_STATIC_WORKSPACE_BYTES];

struct StaticSlot {
    void *ptr = nullptr;  // device address of `scratch` on this device
    bool busy = false;    // a solver made by cfr_create_static lives here
};
std::mutex g_static_mu;
std::vector<StaticSlot> g_static;  // by device ordinal

// Takes the current device's array for one solver: its device address, or
// an error (the array is already in use, or its address is unavailable).
int static_take(int dev, void **ptr)
{
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static.size() <= (size_t)dev) g_static.resize((size_t)dev + 1);
    StaticSlot &ss = g_static[(size_t)dev];
    if (!ss.ptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(CFR_EDEVICE, hip_msg("address of the static workspace", e));
        }
        ss.ptr = p;
    }
    if (ss.busy)
        return fail(CFR_ESTATE, "another solver made by cfr_create_static is alive on this "
                                "device (they share its static workspace)");
    ss.busy = true;
    *ptr = ss.ptr;
    return CFR_OK;
}

void static_give_back(int dev)
{
    std::lock_guard<std::mutex> lk(g_static_mu);
    if ((size_t)dev < g_static.size()) g_static[(size_t)dev].busy = false;
}

}  // namespace

struct cfr_prepared {
    cfr::HostGame hg;  // plans and row pointers (the streams live in the image)
    cfr::GameImage img;
    int precision = CFR_FP64;
    int64_t units[5] = {0, 0, 0, 0, 0};
};

struct cfr_batch {
    cfr::Engine eng;
    int find(int64_t id) const
    {
        for (size_t i = 0; i < eng.slots.size(); ++i)
            if (eng.slots[i].live && eng.slots[i].id == id) return (int)i;
        return -1;
    }
};

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
        *bytes = lone_bytes(game, opt->precision);
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_create(const cfr_game_desc *game, const cfr_options *opt, cfr_solver **out)
{
    if (!out) return fail(CFR_EINVAL, "null output");
    *out = nullptr;
    try {
        int rc = check_options(opt);
        if (rc) return rc;
        rc = validate_game(game, true);
        if (rc) return rc;
        rc = check_device(opt->device);
        if (rc) return rc;
        DeviceGuard guard(opt->device);
        return create_lone(game, opt, opt->workspace, opt->workspace_bytes, false, out);
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_create_static(const cfr_game_desc *game, const cfr_options *opt, cfr_solver **out)
{
    if (!out) return fail(CFR_EINVAL, "null output");
    *out = nullptr;
    bool taken = false;
    try {
        int rc = check_options(opt);
        if (rc) return rc;
        if (opt->workspace)
            return fail(CFR_EINVAL, "cfr_create_static takes no workspace (it uses the "
                                    "library's static one)");
        rc = validate_game(game, true);
        if (rc) return rc;
        const size_t need = lone_bytes(game, opt->precision);
        if (need > (size_t)CFR_STATIC_WORKSPACE_BYTES) {
            char buf[160];
            snprintf(buf, sizeof buf,
                     "the game needs %zu bytes of device state; the static workspace holds %zu",
                     need, (size_t)CFR_STATIC_WORKSPACE_BYTES);
            return fail(CFR_ENOMEM, buf);
        }
        rc = check_device(opt->device);
        if (rc) return rc;
        DeviceGuard guard(opt->device);
        void *ws = nullptr;
        rc = static_take(opt->device, &ws);
        if (rc) return rc;
        taken = true;
        rc = create_lone(game, opt, ws, (size_t)CFR_STATIC_WORKSPACE_BYTES, true, out);
        if (rc) static_give_back(opt->device);
        return rc;
    } catch (const std::exception &ex) {
        if (taken) static_give_back(opt->device);
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_step(cfr_solver *s, int64_t n, int variant, int mode)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->eng.failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (n < 0) return fail(CFR_EINVAL, "negative iteration count");
    if (variant < CFR_VANILLA || variant > CFR_PCFR) return fail(CFR_EINVAL, "unknown variant");
    if (mode != CFR_SIMULTANEOUS && mode != CFR_ALTERNATING) return fail(CFR_EINVAL, "unknown mode");
    if (s->variant >= 0 && (variant != s->variant || mode != s->mode))
        return fail(CFR_ESTATE, "variant and mode are fixed by the first cfr_step");
    if (n == 0) return CFR_OK;
    try {
        DeviceGuard guard(s->eng.device);
        if (s->variant < 0) {
            cfr::GameParams gp = s->eng.slots[0].gp;
            gp.variant = variant;
            int rc = s->eng.set_params(0, gp);
            if (rc) return rc;
            s->variant = variant;
            s->mode = mode;
            s->eng.mode = mode;
        }
        return s->eng.iterate(n);
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_strategy(cfr_solver *s, int player, int kind, double *out, int64_t len)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->eng.failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (player < 0 || player > 1 || !out) return fail(CFR_EINVAL, "bad player or output");
    if (kind != CFR_CURRENT && kind != CFR_AVERAGE) return fail(CFR_EINVAL, "unknown kind");
    if (len != s->eng.slots[0].n_seq[player]) return fail(CFR_EINVAL, "output length must equal n_seq");
    try {
        DeviceGuard guard(s->eng.device);
        std::vector<double> v;
        int rc = s->eng.fetch_vector(0, player, kind == CFR_AVERAGE ? 1 : 0, v);
        if (rc) return rc;
        std::memcpy(out, v.data(), sizeof(double) * v.size());
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_regrets(cfr_solver *s, int player, double *out, int64_t len)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->eng.failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (player < 0 || player > 1 || !out) return fail(CFR_EINVAL, "bad player or output");
    if (len != s->eng.slots[0].n_seq[player]) return fail(CFR_EINVAL, "output length must equal n_seq");
    try {
        DeviceGuard guard(s->eng.device);
        std::vector<double> v;
        int rc = s->eng.fetch_vector(0, player, 2, v);
        if (rc) return rc;
        std::memcpy(out, v.data(), sizeof(double) * v.size());
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_exploitability(cfr_solver *s, int kind, double *out, int64_t len)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->eng.failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (!out) return fail(CFR_EINVAL, "null output");
    if (len < 4) return fail(CFR_EINVAL, "the output holds fewer than 4 values");
    if (kind != CFR_CURRENT && kind != CFR_AVERAGE) return fail(CFR_EINVAL, "unknown kind");
    try {
        DeviceGuard guard(s->eng.device);
        int rc = s->eng.evaluate({0}, kind);
        if (rc) return rc;
        for (int64_t i = 0; i < std::min<int64_t>(len, 5); ++i) out[i] = s->eng.slots[0].last[i];
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

namespace {

// Checkpoint image: header, then the slot's scalars, then per player the
// arrays r, m, s (accumulator type) and b, x (value type) over the game's
// sequences (internal numbering).
struct StateHeader {
    char magic[8];
    int32_t version, precision, variant, mode;
    int64_t n_seq[2], n_inf[2], nnz, t;
};

size_t state_bytes(const cfr_solver *s)
{
    const cfr::Slot &sl = s->eng.slots[0];
    const size_t R = cfr::accum_bytes(s->eng.prec), V = cfr::value_bytes(s->eng.prec);
    size_t b = sizeof(StateHeader) + sizeof(cfr::Scalars);
    for (int p = 0; p < 2; ++p) b += (3 * R + 2 * V) * (size_t)sl.n_seq[p];
    return b;
}

}  // namespace

int cfr_state_size(cfr_solver *s, size_t *bytes)
{
    if (!s || !bytes) return fail(CFR_EINVAL, "null argument");
    *bytes = state_bytes(s);
    return CFR_OK;
}

int cfr_get_state(cfr_solver *s, void *out, size_t len)
{
    if (!s || !out) return fail(CFR_EINVAL, "null argument");
    if (s->eng.failed) return fail(CFR_ESTATE, "solver is in an error state");
    if (len < state_bytes(s)) return fail(CFR_EINVAL, "buffer smaller than cfr_state_size");
    DeviceGuard guard(s->eng.device);
    cfr::Engine &e = s->eng;
    const cfr::Slot &sl = e.slots[0];
    StateHeader h{};
    std::memcpy(h.magic, "CFRSTATE", 8);
    h.version = 1;
    h.precision = e.prec;
    h.variant = s->variant;
    h.mode = s->mode;
    for (int p = 0; p < 2; ++p) {
        h.n_seq[p] = sl.n_seq[p];
        h.n_inf[p] = sl.n_inf[p];
    }
    h.nnz = sl.nnz;
    h.t = sl.t;
    char *o = (char *)out;
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    const size_t R = cfr::accum_bytes(e.prec), V = cfr::value_bytes(e.prec);
    hipError_t err = hipMemcpyAsync(o, e.sc, sizeof(cfr::Scalars), hipMemcpyDeviceToHost, e.st);
    o += sizeof(cfr::Scalars);
    for (int p = 0; p < 2 && err == hipSuccess; ++p) {
        const size_t n = (size_t)sl.n_seq[p], S = (size_t)sl.sb[p];
        const cfr::DevPlayer &d = e.dp[p];
        const void *src[5] = {(const char *)d.r + R * S, (const char *)d.m + R * S,
                              (const char *)d.s + R * S, (const char *)d.b + V * S,
                              (const char *)d.x + V * S};
        const size_t el[5] = {R, R, R, V, V};
        for (int k = 0; k < 5 && err == hipSuccess; ++k) {
            err = hipMemcpyAsync(o, src[k], el[k] * n, hipMemcpyDeviceToHost, e.st);
            o += el[k] * n;
        }
    }
    if (err != hipSuccess) return e.device_error("state copy", err);
    return e.sync("state copy");
}

int cfr_set_state(cfr_solver *s, const void *in, size_t len)
{
    if (!s || !in) return fail(CFR_EINVAL, "null argument");
    if (s->eng.failed) return fail(CFR_ESTATE, "solver is in an error state");
    cfr::Engine &e = s->eng;
    cfr::Slot &sl = e.slots[0];
    if (len < sizeof(StateHeader)) return fail(CFR_EINVAL, "state image too short");
    StateHeader h;
    std::memcpy(&h, in, sizeof h);
    if (std::memcmp(h.magic, "CFRSTATE", 8) != 0 || h.version != 1)
        return fail(CFR_EINVAL, "not a state image of this library");
    if (h.precision != e.prec || h.n_seq[0] != sl.n_seq[0] || h.n_seq[1] != sl.n_seq[1] ||
        h.n_inf[0] != sl.n_inf[0] || h.n_inf[1] != sl.n_inf[1] || h.nnz != sl.nnz)
        return fail(CFR_EINVAL, "state image of another game or precision");
    if (len < state_bytes(s)) return fail(CFR_EINVAL, "state image too short");
    if (s->variant >= 0 && h.variant >= 0 && (h.variant != s->variant || h.mode != s->mode))
        return fail(CFR_ESTATE, "the solver already runs another variant or mode");
    DeviceGuard guard(e.device);
    const char *o = (const char *)in + sizeof h;
    const size_t R = cfr::accum_bytes(e.prec), V = cfr::value_bytes(e.prec);
    // the scalars carry the variant and constants the image was taken with
    hipError_t err = hipMemcpyAsync(e.sc, o, sizeof(cfr::Scalars), hipMemcpyHostToDevice, e.st);
    o += sizeof(cfr::Scalars);
    for (int p = 0; p < 2 && err == hipSuccess; ++p) {
        const size_t n = (size_t)sl.n_seq[p], S = (size_t)sl.sb[p];
        cfr::DevPlayer &d = e.dp[p];
        void *dst[5] = {(char *)d.r + R * S, (char *)d.m + R * S, (char *)d.s + R * S,
                        (char *)d.b + V * S, (char *)d.x + V * S};
        const size_t el[5] = {R, R, R, V, V};
        for (int k = 0; k < 5 && err == hipSuccess; ++k) {
            err = hipMemcpyAsync(dst[k], o, el[k] * n, hipMemcpyHostToDevice, e.st);
            o += el[k] * n;
        }
    }
    if (err != hipSuccess) return e.device_error("state copy", err);
    int rc = e.sync("state copy");
    if (rc) return rc;
    sl.t = h.t;
    if (h.variant >= 0) {
        cfr::Scalars sc;
        std::memcpy(&sc, (const char *)in + sizeof h, sizeof sc);
        cfr::GameParams gp = sl.gp;
        gp.variant = h.variant;
        gp.avg_kind = sc.avg_kind;
        gp.alpha = sc.alpha;
        gp.beta = sc.beta;
        gp.gamma = sc.gamma;
        sl.gp = gp;
        s->variant = h.variant;
        s->mode = h.mode;
        e.mode = h.mode;
        e.it.valid = false;
        e.ev.valid = false;
        e.drop_graph();
    }
    return CFR_OK;
}

int cfr_iteration(cfr_solver *s, int64_t *t)
{
    if (!s || !t) return fail(CFR_EINVAL, "null argument");
    *t = s->eng.slots[0].t;
    return CFR_OK;
}

int cfr_kernel_timing(cfr_solver *s, int enable)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->eng.no_alloc && enable)
        return fail(CFR_EUNSUPPORTED, "kernel timing creates HIP events; a solver made by "
                                      "cfr_create_static does not");
    DeviceGuard guard(s->eng.device);
    return kernel_timing(s->eng, enable);
}

int cfr_kernel_stats(cfr_solver *s, int kernel, int64_t *launches, double *total_ms,
                     double *bytes_per_launch)
{
    if (!s || kernel < 0 || kernel > 1) return fail(CFR_EINVAL, "bad solver or kernel");
    DeviceGuard guard(s->eng.device);
    return kernel_stats(s->eng, kernel, launches, total_ms, bytes_per_launch);
}

int cfr_get_tiling(cfr_solver *s, cfr_spmv_tiling *t)
{
    if (!s || !t) return fail(CFR_EINVAL, "null argument");
    get_tiling(s->eng, t);
    return CFR_OK;
}

int cfr_set_tiling(cfr_solver *s, const cfr_spmv_tiling *t)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    int rc = check_tiling(t);
    if (rc) return rc;
    try {
        rc = check_tiling_fits(s->eng, t);
        if (rc) return rc;
        DeviceGuard guard(s->eng.device);
        rc = s->eng.sync("tiling");
        if (rc) return rc;
        return set_tiling(s->eng, t);
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_tune(cfr_solver *s, int reps, cfr_spmv_tiling *chosen)
{
    if (!s) return fail(CFR_EINVAL, "null solver");
    if (s->eng.no_alloc)
        return fail(CFR_EUNSUPPORTED, "the autotuner times with HIP events; a solver made by "
                                      "cfr_create_static does not create them");
    if (s->eng.failed) return fail(CFR_ESTATE, "solver is in an error state");
    try {
        DeviceGuard guard(s->eng.device);
        return tune(s->eng, reps, chosen);
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_destroy(cfr_solver *s)
{
    if (!s) return CFR_OK;
    const bool static_ws = s->eng.no_alloc;
    const int dev = s->eng.device;
    {
        DeviceGuard guard(dev);
        (void)hipStreamSynchronize(s->eng.st);
        s->eng.release();
    }
    delete s;
    if (static_ws) static_give_back(dev);
    return CFR_OK;
}

const char *cfr_last_error(void) { return cfr::last_error_message(); }

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

int cfr_batch_options_default(cfr_batch_options *opt)
{
    if (!opt) return fail(CFR_EINVAL, "null options");
    std::memset(opt, 0, sizeof *opt);
    opt->precision = CFR_FP32_ACC64;
    opt->mode = CFR_ALTERNATING;
    opt->spmv_order = CFR_SPMV_DEFAULT;
    opt->max_games = 256;
    opt->check_every = 10;
    opt->use_graph = 1;
    return CFR_OK;
}

int cfr_game_params_default(cfr_game_params *gp)
{
    if (!gp) return fail(CFR_EINVAL, "null game parameters");
    std::memset(gp, 0, sizeof *gp);
    gp->variant = CFR_PCFR_PLUS;
    gp->avg_weight = CFR_AVG_DEFAULT;
    gp->dcfr_alpha = 1.5;
    gp->dcfr_beta = 0.0;
    gp->dcfr_gamma = 2.0;
    return CFR_OK;
}

int cfr_batch_game_size(const cfr_game_desc *game, int64_t *out)
{
    if (!out) return fail(CFR_EINVAL, "null output");
    int rc = validate_game(game, false);
    if (rc) return rc;
    out[0] = cfr::seq_block(game->player[0].n_seq);
    out[1] = cfr::seq_block(game->player[1].n_seq);
    out[2] = game->player[0].n_inf + 1;
    out[3] = game->player[1].n_inf + 1;
    out[4] = game->nnz;
    return CFR_OK;
}

static int batch_capacity(const cfr_batch_options *opt, cfr::Capacity &c)
{
    if (!opt) return fail(CFR_EINVAL, "null options");
    if (opt->precision < CFR_FP64 || opt->precision > CFR_FP32_ACC64)
        return fail(CFR_EINVAL, "unknown precision");
    if (opt->mode != CFR_SIMULTANEOUS && opt->mode != CFR_ALTERNATING)
        return fail(CFR_EINVAL, "unknown mode");
    if (opt->spmv_order < CFR_SPMV_DEFAULT || opt->spmv_order > CFR_SPMV_PARALLEL)
        return fail(CFR_EINVAL, "unknown summation order");
    const int64_t kMax = std::numeric_limits<int32_t>::max();
    if (opt->max_games < 1 || opt->max_games > 1 << 20)
        return fail(CFR_EINVAL, "max_games out of range [1, 2^20]");
    for (int p = 0; p < 2; ++p)
        if (opt->seq_capacity[p] < 2 || opt->seq_capacity[p] > kMax || opt->inf_capacity[p] < 1 ||
            opt->inf_capacity[p] > kMax)
            return fail(CFR_EINVAL, "index capacities out of range");
    if (opt->nnz_capacity < 0) return fail(CFR_EINVAL, "negative nonzero capacity");
    if (opt->check_every < 1) return fail(CFR_EINVAL, "check_every must be >= 1");
    if (opt->down_pass != CFR_DOWN_DEFAULT && opt->down_pass != CFR_DOWN_LEVELS)
        return fail(CFR_EINVAL, "unknown top-down pass");
    if (opt->quad_capacity < 0 || opt->quad_capacity > ((int64_t)1 << 40))
        return fail(CFR_EINVAL, "quad capacity out of range");
    c.slots = opt->max_games;
    for (int p = 0; p < 2; ++p) {
        c.seq[p] = opt->seq_capacity[p];
        c.inf[p] = opt->inf_capacity[p];
    }
    c.nnz = opt->nnz_capacity;
    cfr::bound_tables(c);
    return CFR_OK;
}

int cfr_batch_workspace_size(const cfr_batch_options *opt, size_t *bytes)
{
    if (!bytes) return fail(CFR_EINVAL, "null output");
    cfr::Capacity c;
    int rc = batch_capacity(opt, c);
    if (rc) return rc;
    *bytes = cfr::engine_bytes(c, opt->precision);
    return CFR_OK;
}

int cfr_batch_index_limits(const cfr_batch_options *opt, int *out)
{
    if (!out) return fail(CFR_EINVAL, "null output");
    cfr::Capacity c;
    int rc = batch_capacity(opt, c);
    if (rc) return rc;
    out[0] = cfr::slots_fit(c.seq[0]) ? 1 : 0;
    out[1] = cfr::slots_fit(c.seq[1]) ? 1 : 0;
    out[2] = cfr::quads_fit(c.seq[1]) ? 1 : 0;
    out[3] = cfr::quads_fit(c.seq[0]) ? 1 : 0;
    return CFR_OK;
}

int cfr_batch_create(const cfr_batch_options *opt, cfr_batch **out)
{
    if (!out) return fail(CFR_EINVAL, "null output");
    *out = nullptr;
    cfr_batch *b = nullptr;
    try {
        cfr::Capacity c;
        int rc = batch_capacity(opt, c);
        if (rc) return rc;
        rc = check_device(opt->device);
        if (rc) return rc;
        DeviceGuard guard(opt->device);
        b = new cfr_batch();
        cfr::Engine &e = b->eng;
        e.spmv_order = opt->spmv_order;
        e.use_graph = opt->use_graph != 0;
        e.down_pass = opt->down_pass;
        e.async_admission = opt->async_admission != 0;
        e.lone = false;
        e.mode = opt->mode;
        e.check_every = opt->check_every;
        rc = e.init(c, opt->precision, opt->device, (hipStream_t)opt->stream, nullptr, 0);
        if (rc == CFR_OK && opt->quad_capacity > 0) rc = e.reserve_quads(opt->quad_capacity);
        if (rc) {
            e.release();
            delete b;
            return rc;
        }
        *out = b;
        return CFR_OK;
    } catch (const std::exception &ex) {
        if (b) {
            b->eng.release();
            delete b;
        }
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_batch_add(cfr_batch *b, const cfr_game_desc *game, const cfr_game_params *gp, int64_t *id)
{
    if (!b || !id) return fail(CFR_EINVAL, "null argument");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    if (b->eng.failed) return fail(CFR_ESTATE, "batch is in an error state");
    try {
        int rc = check_game_params(gp);
        if (rc) return rc;
        rc = validate_game(game, true);
        if (rc) return rc;
        DeviceGuard guard(b->eng.device);
        cfr::HostGame hg;
        cfr::prepare_game(game, false, true, hg);
        cfr::GameImage img;
        cfr::build_image(hg, b->eng.prec, false, true, img);
        cfr::GameParams p;
        p.variant = gp->variant;
        p.avg_kind = gp->avg_weight;
        p.alpha = gp->dcfr_alpha;
        p.beta = gp->dcfr_beta;
        p.gamma = gp->dcfr_gamma;
        p.target = gp->target_exploitability;
        p.max_it = gp->max_iterations;
        int slot = -1;
        rc = b->eng.add(hg, img, p, b->eng.phase == 0, false, &slot);
        if (rc) return rc;
        *id = b->eng.slots[(size_t)slot].id;
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_prepare(const cfr_game_desc *game, int precision, cfr_prepared **out)
{
    if (!out) return fail(CFR_EINVAL, "null output");
    *out = nullptr;
    if (precision < CFR_FP64 || precision > CFR_FP32_ACC64) return fail(CFR_EINVAL, "unknown precision");
    cfr_prepared *p = nullptr;
    try {
        int rc = validate_game(game, true);
        if (rc) return rc;
        p = new cfr_prepared();
        p->precision = precision;
        cfr::prepare_game(game, false, true, p->hg);
        cfr::build_image(p->hg, precision, true, false, p->img);
        for (int w = 0; w < 2; ++w) {
            std::vector<int32_t>().swap(p->hg.own_idx[w]);
            std::vector<double>().swap(p->hg.own_val[w]);
            p->hg.idx[w] = nullptr;
            p->hg.val[w] = nullptr;
        }
        for (int q = 0; q < 2; ++q) {
            p->units[q] = cfr::seq_block(game->player[q].n_seq);
            p->units[2 + q] = game->player[q].n_inf + 1;
        }
        p->units[4] = game->nnz;
        *out = p;
        return CFR_OK;
    } catch (const std::exception &ex) {
        delete p;
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_prepare_quads(cfr_prepared *p, const int *perm)
{
    if (!p || !perm) return fail(CFR_EINVAL, "null argument");
    for (int w = 0; w < 2; ++w)
        if (perm[w] != 0 && perm[w] != 1) return fail(CFR_EINVAL, "perm must be 0 or 1");
    for (int w = 0; w < 2; ++w)
        if (!cfr::quads_fit(cfr::seq_block(p->hg.pl[1 - w].n_seq)))
            return fail(CFR_EINVAL, "stream form 3 needs every column index below 2^30");
    try {
        cfr::build_image_quads(p->hg, perm, true, p->img);
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
    return CFR_OK;
}

int cfr_prepared_size(const cfr_prepared *p, int64_t *out)
{
    if (!p || !out) return fail(CFR_EINVAL, "null argument");
    for (int i = 0; i < 5; ++i) out[i] = p->units[i];
    return CFR_OK;
}

int cfr_batch_add_prepared(cfr_batch *b, const cfr_prepared *p, const cfr_game_params *gp,
                           int64_t *id)
{
    if (!b || !p || !id) return fail(CFR_EINVAL, "null argument");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    if (b->eng.failed) return fail(CFR_ESTATE, "batch is in an error state");
    if (p->precision != b->eng.prec)
        return fail(CFR_EINVAL, "the game was prepared for another precision");
    try {
        int rc = check_game_params(gp);
        if (rc) return rc;
        DeviceGuard guard(b->eng.device);
        cfr::GameParams q;
        q.variant = gp->variant;
        q.avg_kind = gp->avg_weight;
        q.alpha = gp->dcfr_alpha;
        q.beta = gp->dcfr_beta;
        q.gamma = gp->dcfr_gamma;
        q.target = gp->target_exploitability;
        q.max_it = gp->max_iterations;
        int slot = -1;
        cfr::Engine &e = b->eng;
        if (e.async_admission) {
            // copies overlap the iterations of the games already running
            const bool idle = e.active_set().empty();
            rc = e.add(p->hg, p->img, q, e.phase == 0 && idle, true, &slot);
        } else {
            rc = e.add(p->hg, p->img, q, e.phase == 0, false, &slot);
        }
        if (rc) return rc;
        *id = b->eng.slots[(size_t)slot].id;
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_prepared_destroy(cfr_prepared *p)
{
    delete p;
    return CFR_OK;
}

int cfr_batch_run(cfr_batch *b, int64_t n, int64_t *n_active)
{
    if (!b) return fail(CFR_EINVAL, "null batch");
    if (b->eng.failed) return fail(CFR_ESTATE, "batch is in an error state");
    if (n < 0) return fail(CFR_EINVAL, "negative iteration count");
    try {
        DeviceGuard guard(b->eng.device);
        int rc = b->eng.run(n);
        if (rc) return rc;
        if (n_active) {
            int64_t k = 0;
            for (const cfr::Slot &s : b->eng.slots) k += s.live && (s.active || s.pending);
            *n_active = k;
        }
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

static void count_active(const cfr_batch *b, int64_t *n_active)
{
    if (!n_active) return;
    int64_t k = 0;
    for (const cfr::Slot &s : b->eng.slots) k += s.live && (s.active || s.pending);
    *n_active = k;
}

int cfr_batch_run_begin(cfr_batch *b)
{
    if (!b) return fail(CFR_EINVAL, "null batch");
    if (b->eng.failed) return fail(CFR_ESTATE, "batch is in an error state");
    try {
        DeviceGuard guard(b->eng.device);
        return b->eng.run_begin();
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_batch_run_ready(cfr_batch *b, int *ready)
{
    if (!b || !ready) return fail(CFR_EINVAL, "null argument");
    DeviceGuard guard(b->eng.device);
    *ready = b->eng.run_ready();
    return CFR_OK;
}

int cfr_batch_run_end(cfr_batch *b, int64_t *n_active)
{
    if (!b) return fail(CFR_EINVAL, "null batch");
    if (b->eng.failed) return fail(CFR_ESTATE, "batch is in an error state");
    try {
        DeviceGuard guard(b->eng.device);
        int rc = b->eng.run_end();
        if (rc) return rc;
        count_active(b, n_active);
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_batch_status(cfr_batch *b, int64_t id, cfr_game_status *out)
{
    if (!b || !out) return fail(CFR_EINVAL, "null argument");
    const int k = b->find(id);
    if (k < 0) return fail(CFR_EINVAL, "unknown game");
    const cfr::Slot &s = b->eng.slots[(size_t)k];
    out->state = s.active ? CFR_GAME_ACTIVE : s.pending ? CFR_GAME_WAITING : CFR_GAME_DONE;
    out->reached_target = s.reached ? 1 : 0;
    out->iterations = s.t;
    out->evaluated_at = s.last_t;
    out->exploitability = s.last_t >= 0 ? s.last[0] : std::nan("");
    return CFR_OK;
}

int cfr_batch_strategy(cfr_batch *b, int64_t id, int player, int kind, double *out, int64_t len)
{
    if (!b || !out) return fail(CFR_EINVAL, "null argument");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    if (b->eng.failed) return fail(CFR_ESTATE, "batch is in an error state");
    const int k = b->find(id);
    if (k < 0) return fail(CFR_EINVAL, "unknown game");
    if (player < 0 || player > 1) return fail(CFR_EINVAL, "bad player");
    if (kind != CFR_CURRENT && kind != CFR_AVERAGE) return fail(CFR_EINVAL, "unknown kind");
    if (len != b->eng.slots[(size_t)k].n_seq[player])
        return fail(CFR_EINVAL, "output length must equal n_seq");
    try {
        DeviceGuard guard(b->eng.device);
        std::vector<double> v;
        int rc = b->eng.fetch_vector(k, player, kind == CFR_AVERAGE ? 1 : 0, v);
        if (rc) return rc;
        std::memcpy(out, v.data(), sizeof(double) * v.size());
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_batch_exploitability(cfr_batch *b, int64_t id, int kind, double *out, int64_t len)
{
    if (!b || !out) return fail(CFR_EINVAL, "null argument");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    if (len < 4) return fail(CFR_EINVAL, "the output holds fewer than 4 values");
    if (b->eng.failed) return fail(CFR_ESTATE, "batch is in an error state");
    if (kind != CFR_CURRENT && kind != CFR_AVERAGE) return fail(CFR_EINVAL, "unknown kind");
    const int k = b->find(id);
    if (k < 0) return fail(CFR_EINVAL, "unknown game");
    try {
        DeviceGuard guard(b->eng.device);
        int rc = b->eng.evaluate({k}, kind);
        if (rc) return rc;
        for (int64_t i = 0; i < std::min<int64_t>(len, 5); ++i)
            out[i] = b->eng.slots[(size_t)k].last[i];
        return CFR_OK;
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_batch_remove(cfr_batch *b, int64_t id)
{
    if (!b) return fail(CFR_EINVAL, "null batch");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    const int k = b->find(id);
    if (k < 0) return fail(CFR_EINVAL, "unknown game");
    DeviceGuard guard(b->eng.device);
    int rc = b->eng.sync("remove");  // kernels of this game may still be in flight
    if (rc) return rc;
    b->eng.remove(k);
    return CFR_OK;
}

int cfr_batch_get_tiling(cfr_batch *b, cfr_spmv_tiling *t)
{
    if (!b || !t) return fail(CFR_EINVAL, "null argument");
    get_tiling(b->eng, t);
    return CFR_OK;
}

int cfr_batch_set_tiling(cfr_batch *b, const cfr_spmv_tiling *t)
{
    if (!b) return fail(CFR_EINVAL, "null batch");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    int rc = check_tiling(t);
    if (rc) return rc;
    try {
        rc = check_tiling_fits(b->eng, t);
        if (rc) return rc;
        DeviceGuard guard(b->eng.device);
        rc = b->eng.sync("tiling");
        if (rc) return rc;
        return set_tiling(b->eng, t);
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_batch_tune(cfr_batch *b, int reps, cfr_spmv_tiling *chosen)
{
    if (!b) return fail(CFR_EINVAL, "null batch");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    if (b->eng.failed) return fail(CFR_ESTATE, "batch is in an error state");
    try {
        DeviceGuard guard(b->eng.device);
        return tune(b->eng, reps, chosen);
    } catch (const std::exception &ex) {
        return fail(CFR_ENOMEM, std::string("host allocation failed: ") + ex.what());
    }
}

int cfr_batch_kernel_timing(cfr_batch *b, int enable)
{
    if (!b) return fail(CFR_EINVAL, "null batch");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    DeviceGuard guard(b->eng.device);
    return kernel_timing(b->eng, enable);
}

int cfr_batch_kernel_stats(cfr_batch *b, int kernel, int64_t *launches, double *total_ms,
                           double *bytes_per_launch)
{
    if (!b || kernel < 0 || kernel > 1) return fail(CFR_EINVAL, "bad batch or kernel");
    if (b->eng.pending)
        return fail(CFR_ESTATE, "a check period begun by cfr_batch_run_begin has not ended");
    DeviceGuard guard(b->eng.device);
    return kernel_stats(b->eng, kernel, launches, total_ms, bytes_per_launch);
}

int cfr_batch_host_stats(cfr_batch *b, double *out)
{
    if (!b || !out) return fail(CFR_EINVAL, "null argument");
    for (int i = 0; i < cfr::Engine::kHostN; ++i) {
        out[i] = b->eng.host_s[i];
        out[cfr::Engine::kHostN + i] = (double)b->eng.host_n[i];
    }
    return CFR_OK;
}

int cfr_batch_destroy(cfr_batch *b)
{
    if (!b) return CFR_OK;
    {
        DeviceGuard guard(b->eng.device);
        (void)hipStreamSynchronize(b->eng.st);
        b->eng.release();
    }
    delete b;
    return CFR_OK;
}

}  // extern "C"
