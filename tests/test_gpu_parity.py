"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: FP64 mode within 1e-9 relative (||gpu - oracle||_inf <=
1e-9 * max(1, ||oracle||_inf)) on current and average strategies, regrets,
best-response values, NashConv and the game value.  FP32 modes: within 1e-4
absolute on exploitability at the stated horizon (1000 iterations on the
medium and the large game), and on average strategies where the trajectory
is well conditioned (the tiny game at 10,000 iterations, the first
iterations of the medium and large games).  Between those points the
CFR+ and DCFR trajectories of the medium and large games are chaotic: the
FP64 oracle itself moves by more than 1e-4 in exploitability when its
payoffs are scaled by (1 + 1e-12) (tests/test_conditioning.py), and the
paper's appendix of additional results reports iterates of different
implementations diverging for the same reason.  There the errors of
exploitability, NashConv, both best responses and the average strategies
are reported beside the distance the FP64 oracle moves under that
perturbation and under float32 payoffs, and the GPU's evaluation of its own
profile is checked against the oracle's evaluation of the same profile.
Every FP32 error is printed in the session summary.
"""
import sys

import numpy as np
import pytest

import gamegen as gg
from helpers import dfs_renumber, rel_inf, report

pytestmark = pytest.mark.gpu

VARIANTS = ["vanilla", "cfr+", "dcfr", "pcfr+", "pcfr"]
MODES = ["simultaneous", "alternating"]


@pytest.fixture(scope="module")
def cfr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2605_14277_amd as m
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_fp64(gpu, orc, tol=1e-9, what=""):
    errs = {}
    for p in range(2):
        for kind in ("current", "average"):
            errs[f"x{p}_{kind}"] = rel_inf(gpu.strategy(p, kind), orc.strategy(p, kind))
        errs[f"r{p}"] = rel_inf(gpu.regrets(p), orc.regrets(p))
    for kind in ("current", "average"):
        eg, eo = gpu.exploitability(kind), orc.exploitability(kind)
        for k in ("nash_conv", "br1", "br2", "value"):
            errs[f"{k}_{kind}"] = abs(eg[k] - eo[k]) / max(1.0, abs(eo[k]))
    worst = max(errs.values())
    say(f"[parity {what}] worst rel err {worst:.3e}")
    assert worst <= tol, (what, {k: v for k, v in errs.items() if v > tol})
    return errs


def run_pair(cfr, oracle_mod, game, variant, mode, iters, precision="fp64", **kw):
    gpu = cfr.Solver(game, precision=precision, **kw)
    orc = oracle_mod.Oracle(game, **{k: v for k, v in kw.items()
                                     if k in ("alpha", "beta", "gamma", "avg")})
    gpu.step(iters, variant, mode)
    orc.step(iters, variant, mode)
    return gpu, orc


# --------------------------------------------------------------------------
# FP64
# --------------------------------------------------------------------------

def test_cfg1_vanilla_simultaneous_10k(cfr, oracle_mod):
    """Tiny game, vanilla CFR, simultaneous, FP64, 10000 iterations."""
    g = gg.cfg1()
    say("case: cfg1 vanilla simultaneous fp64 10000")
    gpu, orc = run_pair(cfr, oracle_mod, g, "vanilla", "simultaneous", 10000)
    compare_fp64(gpu, orc, what="cfg1")
    from pins import lp_game_value
    v_star, _ = lp_game_value(g)
    e = gpu.exploitability("average")
    assert abs(e["value"] - v_star) <= e["nash_conv"] + 1e-9
    assert e["expl"] < 2e-3


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", ["stops", "cfg2_d8"])
def test_variants_fp64(cfr, oracle_mod, games, name, variant, mode):
    g = games[name] if name in games else gg.make_config(name)
    say(f"case: {name} {variant} {mode} fp64 300")
    gpu, orc = run_pair(cfr, oracle_mod, g, variant, mode, 300)
    compare_fp64(gpu, orc, what=f"{name}/{variant}/{mode}")


def test_cfg2_cfr_plus_alternating_fp64_1000(cfr, oracle_mod):
    """Medium game (3.4e6 nonzeros), CFR+, alternating, FP64, 1000 iterations."""
    g = gg.cfg2()
    say(f"case: cfg2 cfr+ alternating fp64 1000 nnz={g.nnz}")
    gpu, orc = run_pair(cfr, oracle_mod, g, "cfr+", "alternating", 1000)
    compare_fp64(gpu, orc, what="cfg2-fp64")


def _polytope_residual(g, p, x):
    par, first = g.inf_parent[p], g.inf_first_seq[p]
    sums = np.add.reduceat(x[1:], first[:-1] - 1) if g.n_inf[p] else np.zeros(0)
    res = np.abs(sums - x[par]) if g.n_inf[p] else np.zeros(1)
    return max(float(res.max()), abs(float(x[0]) - 1.0))


def _float_rounded(g):
    """The same game with its payoff values rounded to float32 (what an
    FP32 path stores), still held in double."""
    import copy
    h = copy.copy(g)
    h.val = g.val.astype(np.float32).astype(np.float64)
    h.val_csc = g.val_csc.astype(np.float32).astype(np.float64)
    return h


def _scaled(g, factor):
    """The same game with every payoff value multiplied by `factor`."""
    import copy
    h = copy.copy(g)
    h.val = g.val * factor
    h.val_csc = g.val_csc * factor
    return h


def _profile_nash_conv(orc, x, y):
    """NashConv of an arbitrary profile, evaluated by the FP64 oracle."""
    return orc.best_response_to(0, y) + orc.best_response_to(1, x)


EVAL_KEYS = ("expl", "nash_conv", "br1", "br2")


def fp32_horizon_run(cfr, oracle_mod, g, name, variant, precision, checkpoints, tune=False):
    """Runs the FP32-mode solver beside three all-core FP64 oracles (on the
    game's payoffs, on the payoffs scaled by 1 + 1e-12, and on the payoffs
    rounded to float32) and returns the errors at each checkpoint.

    Asserted: at the last checkpoint (the stated horizon), exploitability of
    the average profile within 1e-4 of the FP64 oracle's at the same
    iteration; at every checkpoint, the GPU's NashConv of its own average
    profile within 1e-4 of the FP64 oracle's evaluation of that same profile
    (the best-response path), non-negative strategies and the sequence-form
    constraints.  Reported at every checkpoint: the errors of
    exploitability, NashConv, both best responses, the game value and the
    average strategies, beside the distance the FP64 oracle itself moves
    under the two payoff perturbations (regret matching amplifies any
    rounding difference, so iterates of implementations that round
    differently drift apart; the paper reports the same effect between its
    implementations)."""
    gpu = cfr.Solver(g, precision=precision)
    if tune:
        say(f"  tiling {gpu.tune(reps=3)}")
    orc = oracle_mod.Oracle(g, parallel=True)
    per = oracle_mod.Oracle(_scaled(g, 1.0 + 1e-12), parallel=True)
    rnd = oracle_mod.Oracle(_float_rounded(g), parallel=True)
    rows = []
    t = 0
    for T in checkpoints:
        gpu.step(T - t, variant, "alternating")
        for o in (orc, per, rnd):
            o.step(T - t, variant, "alternating")
        t = T
        xs = [gpu.strategy(p, "average") for p in range(2)]
        ref = [orc.strategy(p, "average") for p in range(2)]
        err = {f"xbar{p}": float(np.max(np.abs(xs[p] - ref[p]))) for p in range(2)}
        eg, eo = gpu.exploitability("average"), orc.exploitability("average")
        for k in EVAL_KEYS + ("value",):
            err[k] = abs(eg[k] - eo[k])
        spread = {}
        for tag, o in (("1e-12", per), ("f32", rnd)):
            e = o.exploitability("average")
            spread[tag] = {"expl": abs(e["expl"] - eo["expl"]),
                           "xbar": max(float(np.max(np.abs(o.strategy(p, "average") - ref[p])))
                                       for p in range(2))}
        # the GPU's evaluation of its own profile against the FP64 oracle's
        # evaluation of the same profile (checks the best-response kernels)
        err["br_kernels"] = abs(eg["nash_conv"] - _profile_nash_conv(orc, xs[0], xs[1]))
        for p in range(2):
            assert np.all(xs[p] >= 0)
            assert _polytope_residual(g, p, xs[p]) < 1e-5
        report(f"[{name} {variant} {precision} t={T}] expl gpu {eg['expl']:.6e} oracle "
               f"{eo['expl']:.6e} | |d| expl {err['expl']:.1e} nash_conv {err['nash_conv']:.1e} "
               f"br1 {err['br1']:.1e} br2 {err['br2']:.1e} value {err['value']:.1e} "
               f"(own profile {err['br_kernels']:.1e}) | xbar err {err['xbar0']:.1e}/"
               f"{err['xbar1']:.1e} | FP64 oracle moved by payoffs x(1+1e-12): expl "
               f"{spread['1e-12']['expl']:.1e} xbar {spread['1e-12']['xbar']:.1e}; by f32 "
               f"payoffs: expl {spread['f32']['expl']:.1e} xbar {spread['f32']['xbar']:.1e}")
        rows.append((T, err, spread))
        assert err["br_kernels"] <= 1e-4, (T, err["br_kernels"])
    assert err["expl"] <= 1e-4, (t, err["expl"])
    gpu.close()
    for o in (orc, per, rnd):
        o.close()
    return rows


@pytest.mark.parametrize("precision", ["fp32", "fp32_acc64"])
def test_cfg2_cfr_plus_alternating_fp32_1000(cfr, oracle_mod, precision):
    """Medium game (3.4e6 nonzeros), CFR+, alternating, 1000 iterations in
    the FP32 modes: exploitability within 1e-4 of the FP64 oracle at
    t = 1000; at t = 10, 100 and 1000 the errors of exploitability, NashConv,
    both best responses and the average strategies are reported beside the
    FP64 oracle's own spread under perturbed payoffs."""
    g = gg.cfg2()
    say(f"case: cfg2 cfr+ alternating {precision} 1000")
    fp32_horizon_run(cfr, oracle_mod, g, "cfg2", "cfr+", precision, (10, 100, 1000))


@pytest.mark.parametrize("precision", ["fp32", "fp32_acc64"])
def test_cfg2_fp32_short_horizon(cfr, oracle_mod, precision):
    """Before regret matching has amplified rounding, the FP32 path tracks
    the FP64 oracle run on the same float32 payoffs within 1e-4."""
    g = gg.cfg2()
    gpu = cfr.Solver(g, precision=precision)
    orc = oracle_mod.Oracle(_float_rounded(g))
    for n in (1, 2, 2):
        gpu.step(n, "cfr+", "alternating")
        orc.step(n, "cfr+", "alternating")
        for p in range(2):
            for kind in ("current", "average"):
                d = float(np.max(np.abs(gpu.strategy(p, kind) - orc.strategy(p, kind))))
                assert d <= 1e-4, (gpu.iteration, p, kind, d)
        d = abs(gpu.exploitability()["expl"] - orc.exploitability()["expl"])
        say(f"[{precision}] t={gpu.iteration} expl err {d:.2e}")
        assert d <= 1e-4


@pytest.mark.parametrize("precision", ["fp32", "fp32_acc64"])
def test_cfg1_fp32_stable_trajectory(cfr, oracle_mod, precision):
    """On the tiny game CFR+ is insensitive to float rounding, and the FP32
    modes meet 1e-4 on average strategies and exploitability outright."""
    g = gg.cfg1()
    gpu, orc = run_pair(cfr, oracle_mod, g, "cfr+", "alternating", 10000, precision=precision)
    for p in range(2):
        d = float(np.max(np.abs(gpu.strategy(p, "average") - orc.strategy(p, "average"))))
        say(f"[{precision}] cfg1 xbar{p} err {d:.2e}")
        assert d <= 1e-4
    assert abs(gpu.exploitability()["expl"] - orc.exploitability()["expl"]) <= 1e-4


# --------------------------------------------------------------------------
# Full-size game in the benchmark's launch configuration
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def large_game():
    return gg.cfg3()


def test_cfg3_dcfr_alternating_fp64(cfr, oracle_mod, large_game):
    """1e8-nonzero game, DCFR(1.5, 0, 2), alternating, FP64: the same kernels
    and launch shapes the benchmark times, within 1e-9 of the oracle over the
    first iterations (the oracle takes ~0.5 s per iteration here)."""
    g = large_game
    say(f"case: cfg3 dcfr alternating fp64 nnz={g.nnz}")
    gpu = cfr.Solver(g, precision="fp64")
    say(f"  tiling {gpu.tune(reps=3)}")
    orc = oracle_mod.Oracle(g)
    for n in (1, 1, 2):
        gpu.step(n, "dcfr", "alternating")
        orc.step(n, "dcfr", "alternating")
        compare_fp64(gpu, orc, what=f"cfg3-fp64 t={gpu.iteration}")
    gpu.close()
    orc.close()


def test_cfg3_dcfr_alternating_acc64_first_iterations(cfr, oracle_mod, large_game):
    """The benchmark's workload (FP32 values, FP64 accumulators, tuned
    tiling) over its first iterations, before rounding has been amplified:
    average strategies within 1e-4 and regrets within 1e-4 relative of the
    FP64 oracle."""
    g = large_game
    say(f"case: cfg3 dcfr alternating fp32_acc64 t<=2 nnz={g.nnz}")
    gpu = cfr.Solver(g, precision="fp32_acc64")
    say(f"  tiling {gpu.tune(reps=3)}")
    orc = oracle_mod.Oracle(g, parallel=True)
    for n in (1, 1):
        gpu.step(n, "dcfr", "alternating")
        orc.step(n, "dcfr", "alternating")
        for p in range(2):
            d = float(np.max(np.abs(gpu.strategy(p, "average") - orc.strategy(p, "average"))))
            dr = rel_inf(gpu.regrets(p), orc.regrets(p))
            say(f"  t={gpu.iteration} p{p} xbar abs err {d:.2e} regret rel err {dr:.2e}")
            assert d <= 1e-4 and dr <= 1e-4
        eg, eo = gpu.exploitability("average"), orc.exploitability("average")
        assert abs(eg["expl"] - eo["expl"]) <= 1e-4
    gpu.close()
    orc.close()


def test_cfg3_dcfr_alternating_acc64_1000(cfr, oracle_mod, large_game):
    """The benchmark's workload at its stated horizon: the 1e8-nonzero game,
    DCFR(1.5, 0, 2) (Algorithm 4), alternating updates, FP32 values with FP64
    accumulators, the autotuned tiling the benchmark times, 1000 iterations
    beside the all-core FP64 oracle: exploitability within 1e-4 at t = 1000;
    at t = 10, 100 and 1000 the errors of exploitability, NashConv, both best
    responses and the average strategies are reported beside the FP64
    oracle's own spread under perturbed payoffs."""
    g = large_game
    say(f"case: cfg3 dcfr alternating fp32_acc64 1000 nnz={g.nnz}")
    fp32_horizon_run(cfr, oracle_mod, g, "cfg3", "dcfr", "fp32_acc64", (10, 100, 1000),
                     tune=True)


# --------------------------------------------------------------------------
# Layout, edge cases, determinism
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["stops", "cfg2_d8"])
def test_caller_numbering_is_permuted_internally(cfr, oracle_mod, games, name):
    g = games[name] if name in games else gg.make_config(name)
    h = dfs_renumber(g)
    say(f"case: dfs-renumbered {name}")
    gpu, orc = run_pair(cfr, oracle_mod, h, "pcfr+", "alternating", 200)
    compare_fp64(gpu, orc, tol=1e-12, what=f"{name}-dfs")
    ref = cfr.Solver(g)
    ref.step(200, "pcfr+", "alternating")
    for p in range(2):
        m = h.meta["new_of_old"][p]
        assert rel_inf(gpu.strategy(p, "average")[m], ref.strategy(p, "average")) < 1e-12


@pytest.mark.parametrize("cols", [2047, 2048, 2049, 5000])
def test_long_rows(cfr, oracle_mod, cols):
    """Rows longer than one product block (2048 nonzeros) take the long-row
    path; both sides of the boundary are exercised."""
    rng = np.random.default_rng(cols)
    M = rng.uniform(-1, 1, size=(3, cols))
    g = gg.matrix_game(M)
    say(f"case: matrix game 3x{cols}")
    gpu, orc = run_pair(cfr, oracle_mod, g, "cfr+", "alternating", 100)
    compare_fp64(gpu, orc, tol=1e-12, what=f"3x{cols}")


QUADS = {"items": [16, 16], "rows": [256, 128], "vec": [3, 3], "perm": [0, 1], "xcd": [1, 1]}


@pytest.mark.parametrize("cols", [1023, 4096, 4100, 9000])
def test_long_rows_quads(cfr, oracle_mod, cols):
    """Stream form 3 (quads): a block holds 1024 quads, so rows of 4096
    nonzeros still fit and longer ones take the long-row path."""
    rng = np.random.default_rng(cols)
    M = rng.uniform(-1, 1, size=(3, cols))
    g = gg.matrix_game(M)
    say(f"case: matrix game 3x{cols}, quads")
    gpu = cfr.Solver(g, precision="fp64")
    gpu.tiling = QUADS
    orc = oracle_mod.Oracle(g)
    gpu.step(100, "cfr+", "alternating")
    orc.step(100, "cfr+", "alternating")
    compare_fp64(gpu, orc, tol=1e-12, what=f"3x{cols}-quads")


@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
def test_quads_without_nonzeros(cfr, oracle_mod, precision):
    """A game with no payoff nonzeros has no quads: every block of both
    products is empty and writes zero utilities."""
    g = gg.matrix_game(np.zeros((3, 4)))
    assert g.nnz == 0
    gpu = cfr.Solver(g, precision=precision)
    gpu.tiling = QUADS
    orc = oracle_mod.Oracle(g)
    gpu.step(20, "dcfr", "alternating")
    orc.step(20, "dcfr", "alternating")
    for p in range(2):
        assert np.allclose(gpu.strategy(p, "average"), orc.strategy(p, "average"), atol=1e-6)
    assert gpu.exploitability("average")["expl"] == 0.0


@pytest.mark.parametrize("name", ["stops", "cfg2_d8", "showdown", "cfg2"])
def test_quads_fp64_equal_elementwise(cfr, oracle_mod, games, name):
    """Absent quad positions add -0.0, which leaves every FP64 row sum exactly
    as the element stream gives it: the two forms agree bit for bit, and
    both match the oracle."""
    if name == "showdown":
        g = gg.public_game(4, S=6, max_depth=6, branch_lo=2, branch_hi=4, p_stop=0.1,
                           payoff_kind="showdown")
    elif name == "cfg2":
        g = gg.cfg2()
    else:
        g = games[name] if name in games else gg.make_config(name)
    say(f"case: {name} quads vs elements, fp64, nnz={g.nnz}")
    out = []
    for tiling in (None, QUADS, dict(QUADS, perm=[1, 0], rows=[64, 256]),
                   dict(QUADS, items=[8, 8])):
        gpu = cfr.Solver(g, precision="fp64")
        if tiling is not None:
            gpu.tiling = tiling
            assert gpu.tiling == tiling
        gpu.step(60, "dcfr", "alternating")
        out.append([gpu.strategy(p, k) for p in range(2) for k in ("current", "average")] +
                   [gpu.regrets(p) for p in range(2)])
        last = gpu
    for other in out[1:]:
        for a, c in zip(out[0], other):
            assert np.array_equal(a, c)
    orc = oracle_mod.Oracle(g)
    orc.step(60, "dcfr", "alternating")
    compare_fp64(last, orc, tol=1e-9, what=f"{name}-quads")


def _no_shallow_p2():
    """A public game whose player 2 has no one-block shallow pass (its top
    two levels hold 192 + 1056 decision points), so its fused launch starts
    at level 0 and covers its whole treeplex (three levels, 29 decision
    points per subtree)."""
    return gg.public_game(11, S=96, max_depth=6, branch_lo=2, branch_hi=3, p_stop=0.1,
                          payoff_kind="showdown", name="no-shallow-p2")


@pytest.mark.parametrize("name", ["cfg2", "no-shallow-p2"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sweep_structures_equal(cfr, oracle_mod, name, precision):
    """A lone game's default sweep runs the shallow levels in one block and
    the small levels below them in fused launches (from level 0 when there
    is no shallow pass, with level 0's top-down step), then the one-launch
    top-down pass.  It equals the top-down pass one launch per level
    (down_pass "levels": every level below level 0, whichever launch did
    the bottom-up pass of the levels above) and the whole sweep one launch
    per level (up_pass "levels" too) bit for bit, with and without the
    first-touch order on A^T x; in FP64 it also equals the oracle."""
    g = gg.cfg2() if name == "cfg2" else _no_shallow_p2()
    perm = {"items": [16, 16], "rows": [256, 256], "vec": [2, 2], "perm": [0, 1], "xcd": [1, 1]}
    for variant, mode, tiling in (("dcfr", "alternating", perm), ("pcfr+", "simultaneous", None),
                                  ("cfr+", "alternating", None)):
        out = []
        for kw in ({}, {"down_pass": "levels"}, {"up_pass": "levels", "down_pass": "levels"}):
            say(f"case: {name} {precision} {variant} {mode} tiling={tiling is not None} {kw}")
            s = cfr.Solver(g, precision=precision, **kw)
            if tiling is not None:
                s.tiling = tiling
            s.step(25, variant, mode)
            out.append([s.strategy(p, k) for p in range(2) for k in ("current", "average")] +
                       [s.regrets(p) for p in range(2)])
            if not kw and precision == "fp64":
                orc = oracle_mod.Oracle(g)
                orc.step(25, variant, mode)
                compare_fp64(s, orc, tol=1e-9, what=f"{name}-{variant}-{mode}")
                orc.close()
            s.close()
        for other in out[1:]:
            for a, c in zip(out[0], other):
                assert np.array_equal(a, c), (name, variant, mode)


@pytest.mark.parametrize("mode", ["alternating", "simultaneous"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_top_down_pass_writes_the_permuted_copy(cfr, precision, mode):
    """With alternating updates, player 1's top-down pass of a lone game
    writes the first-touch copy of x that the product A^T x reads, instead of
    a gather launch.  Evaluations (which gather the average strategy into the
    same copy) and a restored checkpoint sit between the steps.  Every
    iterate equals that of the same solver without the first-touch order,
    bit for bit: the order only renumbers the columns, and each row keeps
    its nonzeros in the same order."""
    g = gg.cfg2()
    base = {"items": [16, 16], "rows": [256, 256], "vec": [2, 2], "xcd": [1, 1]}
    out = []
    for perm in ([0, 0], [0, 1], [1, 1]):
        say(f"case: cfg2 {precision} {mode} perm {perm}")
        s = cfr.Solver(g, precision=precision)
        s.tiling = dict(base, perm=perm)
        rec = []
        s.step(7, "dcfr", mode)
        rec.append(s.exploitability("average")["expl"])
        state = s.get_state()
        s.step(5, "dcfr", mode)
        rec += [s.strategy(p, "current") for p in range(2)]
        s.set_state(state)
        s.step(9, "dcfr", mode)
        rec.append(s.exploitability("average")["expl"])
        rec += [s.strategy(p, k) for p in range(2) for k in ("current", "average")]
        rec += [s.regrets(p) for p in range(2)]
        out.append(rec)
        s.close()
    for other in out[1:]:
        for a, c in zip(out[0], other):
            assert np.array_equal(a, c)


@pytest.mark.parametrize("precision", ["fp32", "fp32_acc64"])
def test_quads_fp32_short_horizon(cfr, oracle_mod, precision):
    """Stream form 3 in the FP32 modes tracks the FP64 oracle on the same
    float32 payoffs within 1e-4."""
    g = gg.cfg2()
    gpu = cfr.Solver(g, precision=precision)
    gpu.tiling = QUADS
    orc = oracle_mod.Oracle(_float_rounded(g))
    for n in (1, 2, 2):
        gpu.step(n, "cfr+", "alternating")
        orc.step(n, "cfr+", "alternating")
        for p in range(2):
            for kind in ("current", "average"):
                d = float(np.max(np.abs(gpu.strategy(p, kind) - orc.strategy(p, kind))))
                assert d <= 1e-4, (gpu.iteration, p, kind, d)
        d = abs(gpu.exploitability()["expl"] - orc.exploitability()["expl"])
        say(f"[{precision} quads] t={gpu.iteration} expl err {d:.2e}")
        assert d <= 1e-4


def test_player_without_decisions(cfr, oracle_mod):
    from test_oracle_pins import _decision_problem
    g = _decision_problem()
    say("case: decision problem (player 2 never acts)")
    gpu, orc = run_pair(cfr, oracle_mod, g, "dcfr", "alternating", 50)
    compare_fp64(gpu, orc, tol=1e-12, what="one-decision")


def test_many_empty_rows_and_signals(cfr, oracle_mod):
    """Showdown payoffs with ties not stored: many empty rows and columns."""
    g = gg.public_game(4, S=6, max_depth=6, branch_lo=2, branch_hi=4, p_stop=0.1,
                       payoff_kind="showdown")
    say(f"case: showdown S=6 nnz={g.nnz}")
    gpu, orc = run_pair(cfr, oracle_mod, g, "dcfr", "simultaneous", 150)
    compare_fp64(gpu, orc, what="showdown")


def test_zero_iterations_and_current_profile(cfr, oracle_mod, games):
    g = games["cfg1"]
    gpu = cfr.Solver(g)
    orc = oracle_mod.Oracle(g)
    assert gpu.iteration == 0
    compare_fp64(gpu, orc, tol=1e-14, what="t=0")
    gpu.step(0, "vanilla", "simultaneous")
    assert gpu.iteration == 0


def test_repeatable_and_graph_equals_direct(cfr, games):
    g = gg.cfg2_literal()
    runs = []
    for use_graph in (True, True, False):
        s = cfr.Solver(g, use_graph=use_graph)
        s.step(120, "pcfr+", "alternating")
        runs.append([s.strategy(p, "average") for p in range(2)] +
                    [s.regrets(p) for p in range(2)])
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)


def test_split_steps_equal_one_call(cfr, games):
    g = games["stops"]
    a, b = cfr.Solver(g), cfr.Solver(g)
    a.step(90, "dcfr", "alternating")
    for _ in range(9):
        b.step(10, "dcfr", "alternating")
    for p in range(2):
        assert np.array_equal(a.strategy(p, "average"), b.strategy(p, "average"))


def test_state_errors(cfr, games):
    g = games["cfg1"]
    s = cfr.Solver(g)
    s.step(3, "cfr+", "alternating")
    with pytest.raises(cfr.CfrError) as ei:
        s.step(1, "dcfr", "alternating")
    assert ei.value.code == cfr.CFR_ESTATE
    with pytest.raises(cfr.CfrError) as ei:
        cfr.cfr_strategy(s.h, 0, 0, g.n_seq[0] + 1)
    assert ei.value.code == cfr.CFR_EINVAL
    s.step(2, "cfr+", "alternating")
    assert s.iteration == 5


def test_exploitability_output_length(cfr, games):
    """cfr_exploitability writes the first min(len, 5) values and refuses
    len < 4: a caller with room for the four of the contract gets exactly
    those, and the value past them is untouched."""
    import ctypes as C
    s = cfr.Solver(games["cfg1"])
    s.step(7, "cfr+", "alternating")
    full = cfr.cfr_exploitability(s.h, 1)
    out = np.full(5, -7.0)
    ptr = out.ctypes.data_as(C.POINTER(C.c_double))
    assert cfr._lib.cfr_exploitability(s.h, 1, ptr, 4) == cfr.CFR_OK
    assert np.array_equal(out[:4], full[:4]) and out[4] == -7.0
    assert cfr._lib.cfr_exploitability(s.h, 1, ptr, 3) == cfr.CFR_EINVAL
    s.close()


def test_workspace_too_small(cfr, games):
    import ctypes as C

    import torch
    g = games["cfg1"]
    ga = cfr.GameArrays(g)
    o = cfr.cfr_options_default()
    need = cfr.cfr_workspace_size(ga, o)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    o.workspace = C.c_void_p(ws.data_ptr())
    o.workspace_bytes = need - 1024
    with pytest.raises(cfr.CfrError) as ei:
        cfr.cfr_create(ga, o)
    assert ei.value.code == cfr.CFR_ENOMEM


def test_kernel_timing_reports(cfr, games):
    g = gg.cfg2_literal()
    s = cfr.Solver(g)
    s.kernel_timing(True)
    s.step(20, "cfr+", "alternating")
    for k in range(2):
        n, ms, by = s.kernel_stats(k)
        assert n == 20 and ms > 0 and by > g.nnz * 12
    s.kernel_timing(False)
    s.step(5, "cfr+", "alternating")
    assert s.iteration == 25


@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
@pytest.mark.parametrize("variant", ["dcfr", "pcfr+"])
def test_checkpoint_resume_equals_uninterrupted(cfr, games, precision, variant):
    """A state image taken after 30 iterations and loaded into a fresh
    solver continues exactly as the original: after 20 more iterations
    both equal an uninterrupted 50-iteration run bit for bit."""
    g = games["stops"]
    a = cfr.Solver(g, precision=precision, alpha=2.0, gamma=3.0)
    a.step(30, variant, "alternating")
    state = a.get_state()
    b = cfr.Solver(g, precision=precision)  # other constants: the image carries them
    b.set_state(state)
    assert b.iteration == 30
    a.step(20, variant, "alternating")
    b.step(20, variant, "alternating")
    c = cfr.Solver(g, precision=precision, alpha=2.0, gamma=3.0)
    c.step(50, variant, "alternating")
    for x in (a, b):
        for p in range(2):
            for kind in ("current", "average"):
                assert np.array_equal(x.strategy(p, kind), c.strategy(p, kind))
            assert np.array_equal(x.regrets(p), c.regrets(p))
    other = cfr.Solver(games["cfg1"], precision=precision)
    with pytest.raises(cfr.CfrError) as ei:
        other.set_state(state)
    assert ei.value.code == cfr.CFR_EINVAL
    for x in (a, b, c, other):
        x.close()


@pytest.mark.parametrize("avg", ["uniform", "linear", "quadratic", "pow_gamma"])
@pytest.mark.parametrize("mode", MODES)
def test_linear_cfr_and_averaging_weights(cfr, oracle_mod, games, avg, mode):
    """Linear CFR as DCFR(1, 1, 1), under each averaging weight a caller can
    set: the FP64 GPU path against the oracle run with the same parameters."""
    g = games["cfg2_d8"] if "cfg2_d8" in games else gg.make_config("cfg2_d8")
    say(f"case: cfg2_d8 dcfr(1,1,1) avg={avg} {mode}")
    gpu = cfr.Solver(g, precision="fp64", alpha=1.0, beta=1.0, gamma=1.0, avg=avg)
    orc = oracle_mod.Oracle(g, alpha=1.0, beta=1.0, gamma=1.0, avg=avg)
    gpu.step(150, "dcfr", mode)
    orc.step(150, "dcfr", mode)
    compare_fp64(gpu, orc, tol=1e-9, what=f"lcfr-{avg}-{mode}")
    gpu.close()
    orc.close()


def _wide_game(name):
    """Public trees with wide nodes: up to 7 actions and 7 decision points
    below a sequence (wide7), or up to 12 of both (wide12)."""
    if name == "wide7":
        return gg.public_game(7, S=3, max_depth=4, branch_lo=5, branch_hi=7, p_stop=0.0,
                              payoff_kind="iid", name="wide7")
    return gg.public_game(8, S=2, max_depth=3, branch_lo=9, branch_hi=12, p_stop=0.0,
                          payoff_kind="iid", name="wide12")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["wide7", "wide12"])
def test_wide_decision_points_fp64(cfr, oracle_mod, name, variant):
    """Decision points with more than four actions and sequences with more
    than four decision points below them take the generic sweep instance
    (child values read in chunks; above eight actions, the values are
    recomputed instead of held): FP64 within 1e-9 of the oracle, both
    schedules, best responses included."""
    g = _wide_game(name)
    for mode in MODES:
        say(f"case: {name} {variant} {mode} fp64 nnz={g.nnz}")
        gpu, orc = run_pair(cfr, oracle_mod, g, variant, mode, 200)
        compare_fp64(gpu, orc, tol=1e-9, what=f"{name}-{variant}-{mode}")
        gpu.close()
        orc.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
def test_wide_games_batched_equal_alone(cfr, precision):
    """The wide games in one batch with a narrow one: each equals the same
    game solved alone bit for bit."""
    games = [_wide_game("wide7"), _wide_game("wide12"), gg.make_config("cfg2_d8")]
    sizes = np.sum([cfr.Batch.game_size(g) for g in games], axis=0)
    b = cfr.Batch([int(sizes[0]), int(sizes[1])], [int(sizes[2]), int(sizes[3])], int(sizes[4]),
                  max_games=4,
                  precision=precision, mode="alternating", check_every=10)
    ids = [b.add(g, "pcfr+") for g in games]
    b.run(60)
    for gid, g in zip(ids, games):
        solo = cfr.Solver(g, precision=precision)
        solo.step(60, "pcfr+", "alternating")
        for p in range(2):
            for kind in ("current", "average"):
                assert np.array_equal(b.strategy(gid, p, kind), solo.strategy(p, kind)), \
                    (g.name, p, kind)
        for kind in ("current", "average"):
            assert b.exploitability(gid, kind)["expl"] == solo.exploitability(kind)["expl"]
        solo.close()
    b.close()


# --------------------------------------------------------------------------
# Two adjacent bottom-up levels in one launch
# --------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("mode", MODES)
def test_two_level_launches_equal_level_by_level(cfr, oracle_mod, variant, mode):
    """With the two-level option the medium game's bottom-up pass runs
    adjacent levels as one launch (player 1: levels 6+5, 4+3, 2+1 and 0;
    player 2: 5+4, 3+2, 1+0, the lowest pair including the root level's
    top-down step and the deepest pairs a level with nothing below it).  In
    FP64 every iterate equals the default one-launch-per-level pass bit for
    bit, and both match the oracle."""
    g = gg.cfg2()
    fused = cfr.Solver(g, precision="fp64", up_pass="pairs")
    plain = cfr.Solver(g, precision="fp64")
    orc = oracle_mod.Oracle(g, parallel=True)
    for n in (1, 29):
        fused.step(n, variant, mode)
        plain.step(n, variant, mode)
        orc.step(n, variant, mode)
        for p in range(2):
            for kind in ("current", "average"):
                assert np.array_equal(fused.strategy(p, kind), plain.strategy(p, kind)), (p, kind)
            assert np.array_equal(fused.regrets(p), plain.regrets(p)), p
    compare_fp64(fused, orc, what=f"cfg2 two-level {variant}/{mode}")
    fused.close()
    plain.close()
    orc.close()


@pytest.mark.parametrize("precision", ["fp32", "fp32_acc64"])
def test_two_level_launches_fp32_modes(cfr, precision):
    """The same in the FP32 modes on the medium game: bit for bit equal to
    one launch per level."""
    g = gg.cfg2()
    a = cfr.Solver(g, precision=precision, up_pass="pairs")
    b = cfr.Solver(g, precision=precision)
    for s in (a, b):
        s.step(40, "dcfr", "alternating")
    for p in range(2):
        assert np.array_equal(a.strategy(p, "average"), b.strategy(p, "average"))
        assert np.array_equal(a.regrets(p), b.regrets(p))
    a.close()
    b.close()


# --------------------------------------------------------------------------
# Shallow levels in one block
# --------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("mode", MODES)
def test_shallow_block_equals_level_by_level(cfr, oracle_mod, variant, mode):
    """By default a lone game runs its shallow levels' bottom-up pass in one
    block, the values passed between levels in LDS (the medium game: the top
    three levels of each player, 260 and 559 decision points; the deepest of
    them reads value slots).  In FP64 every iterate equals the
    one-launch-per-level pass bit for bit, and both match the oracle."""
    g = gg.cfg2()
    fused = cfr.Solver(g, precision="fp64")
    plain = cfr.Solver(g, precision="fp64", up_pass="levels")
    orc = oracle_mod.Oracle(g, parallel=True)
    for n in (1, 19):
        fused.step(n, variant, mode)
        plain.step(n, variant, mode)
        orc.step(n, variant, mode)
        for p in range(2):
            for kind in ("current", "average"):
                assert np.array_equal(fused.strategy(p, kind), plain.strategy(p, kind)), (p, kind)
            assert np.array_equal(fused.regrets(p), plain.regrets(p)), p
    compare_fp64(fused, orc, what=f"cfg2 shallow block {variant}/{mode}")
    for s in (fused, plain, orc):
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_acc64"])
def test_shallow_block_large_game(cfr, large_game, precision):
    """The large game (player 1's two shallow levels, 448 decision points,
    the deeper one reading value slots) in every precision: bit for bit
    equal to one launch per level over a few DCFR iterations."""
    a = cfr.Solver(large_game, precision=precision)
    b = cfr.Solver(large_game, precision=precision, up_pass="levels")
    for s in (a, b):
        s.step(6, "dcfr", "alternating")
    for p in range(2):
        assert np.array_equal(a.strategy(p, "average"), b.strategy(p, "average"))
        assert np.array_equal(a.regrets(p), b.regrets(p))
    a.close()
    b.close()


@pytest.mark.parametrize("seed", range(8))
def test_sweep_structures_on_irregular_games(cfr, seed):
    """Random public games of irregular shape (early stops, uneven branching,
    decision points with one action, from tiny to 1e6 nonzeros): the default
    sweep of a lone game (one-block shallow levels, fused small levels, the
    top-down pass writing the first-touch copy) equals the sweep one launch
    per level bit for bit in FP64, and so does the same game left iterating
    alone in a batch after a smaller game has finished."""
    rng = np.random.default_rng(1000 + seed)
    S = int(rng.choice([4, 12, 33, 70, 96]))
    depth = int(rng.integers(3, 8))
    lo = int(rng.integers(1, 3))
    hi = int(rng.integers(lo, 5))
    g = gg.public_game(2000 + seed, S=S, max_depth=depth, branch_lo=lo, branch_hi=hi,
                       p_stop=float(rng.uniform(0.0, 0.4)), payoff_kind="showdown",
                       name=f"irregular-{seed}")
    say(f"case: irregular game {seed}: S={S} depth={depth} branching {lo}..{hi}, nnz={g.nnz}")
    perm = {"items": [16, 16], "rows": [256, 256], "vec": [2, 2], "perm": [0, 1], "xcd": [1, 1]}
    out = []
    for kw in ({}, {"up_pass": "levels", "down_pass": "levels"}):
        s = cfr.Solver(g, precision="fp64", **kw)
        s.tiling = perm
        s.step(15, "pcfr+", "alternating")
        out.append([s.strategy(p, k) for p in range(2) for k in ("current", "average")] +
                   [s.regrets(p) for p in range(2)])
        s.close()
    for a, c in zip(out[0], out[1]):
        assert np.array_equal(a, c), seed
    first = gg.public_game(3000 + seed, S=3, max_depth=3, branch_lo=2, branch_hi=2, p_stop=0.0,
                           payoff_kind="showdown", name="first")
    units = np.sum([cfr.Batch.game_size(x) for x in (first, g)], axis=0)
    b = cfr.Batch([int(units[0]), int(units[1])], [int(units[2]), int(units[3])], int(units[4]),
                  max_games=2, precision="fp64", check_every=5)
    b.tiling = perm
    b.add(first, "cfr+", max_iterations=5)
    k = b.add(g, "pcfr+", max_iterations=15)
    while b.run(5):
        pass
    assert b.status(k)["iterations"] == 15
    got = [b.strategy(k, p, kind) for p in range(2) for kind in ("current", "average")]
    for a, c in zip(got, out[1][:4]):
        assert np.array_equal(a, c), seed
    b.close()
