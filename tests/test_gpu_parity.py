"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars (stated for this method's outputs): FP64 mode within 1e-9 relative
(||gpu - oracle||_inf <= 1e-9 * max(1, ||oracle||_inf)) on current and
average strategies, regrets, best-response values, NashConv and the game
value; FP32 modes within 1e-4 absolute on average strategies and
exploitability, with the error reported.
"""
import sys

import numpy as np
import pytest

import gamegen as gg
from helpers import dfs_renumber, rel_inf

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


@pytest.mark.parametrize("precision", ["fp32", "fp32_acc64"])
def test_cfg2_cfr_plus_alternating_fp32_1000(cfr, oracle_mod, precision):
    """FP32 modes against the FP64 oracle: 1e-4 absolute on average
    strategies and exploitability; every error is printed."""
    g = gg.cfg2()
    say(f"case: cfg2 cfr+ alternating {precision} 1000")
    gpu, orc = run_pair(cfr, oracle_mod, g, "cfr+", "alternating", 1000, precision=precision)
    errs = {}
    for p in range(2):
        errs[f"xbar{p}"] = float(np.max(np.abs(gpu.strategy(p, "average") -
                                               orc.strategy(p, "average"))))
        errs[f"x{p}"] = float(np.max(np.abs(gpu.strategy(p, "current") -
                                            orc.strategy(p, "current"))))
    eg, eo = gpu.exploitability("average"), orc.exploitability("average")
    for k in ("expl", "nash_conv", "br1", "br2", "value"):
        errs[k] = abs(eg[k] - eo[k])
    say(f"[{precision}] errors vs fp64 oracle: " +
        ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert errs["xbar0"] <= 1e-4 and errs["xbar1"] <= 1e-4
    assert errs["expl"] <= 1e-4


# --------------------------------------------------------------------------
# Full-size game in the benchmark's launch configuration
# --------------------------------------------------------------------------

def _polytope_residual(g, p, x):
    par, first = g.inf_parent[p], g.inf_first_seq[p]
    sums = np.add.reduceat(x[1:], first[:-1] - 1) if g.n_inf[p] else np.zeros(0)
    res = np.abs(sums - x[par]) if g.n_inf[p] else np.zeros(1)
    return max(float(res.max()), abs(float(x[0]) - 1.0))


@pytest.fixture(scope="module")
def large_game():
    return gg.cfg3()


def test_cfg3_dcfr_alternating_acc64(cfr, oracle_mod, large_game):
    """1e8-nonzero game, DCFR(1.5, 0, 2), alternating, FP32 values with FP64
    accumulators: the first iterations against the oracle, then properties
    that hold at any size after a longer run."""
    g = large_game
    say(f"case: cfg3 dcfr alternating fp32_acc64 nnz={g.nnz}")
    gpu = cfr.Solver(g, precision="fp32_acc64")
    orc = oracle_mod.Oracle(g)
    for n in (1, 2):
        gpu.step(n, "dcfr", "alternating")
        orc.step(n, "dcfr", "alternating")
        for p in range(2):
            d = float(np.max(np.abs(gpu.strategy(p, "average") - orc.strategy(p, "average"))))
            dr = rel_inf(gpu.regrets(p), orc.regrets(p))
            say(f"  t={gpu.iteration} p{p} xbar abs err {d:.2e} regret rel err {dr:.2e}")
            assert d <= 1e-4 and dr <= 1e-4
        eg, eo = gpu.exploitability("average"), orc.exploitability("average")
        say(f"  expl gpu {eg['expl']:.6f} oracle {eo['expl']:.6f}")
        assert abs(eg["expl"] - eo["expl"]) <= 1e-4
    orc.close()
    e0 = gpu.exploitability("average")["expl"]
    gpu.step(197, "dcfr", "alternating")
    e1 = gpu.exploitability("average")
    say(f"  t={gpu.iteration} expl {e1['expl']:.6f} (t=3: {e0:.6f})")
    assert e1["nash_conv"] >= 0 and e1["expl"] < e0
    for p in range(2):
        x = gpu.strategy(p, "average")
        assert np.all(x >= 0)
        assert _polytope_residual(g, p, x) < 1e-5


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
