"""The CPU oracle pinned against what the paper and the mathematics fix.

Each test names the passage or the fact it relies on.  None of them compares
the oracle with a retyped copy of itself: classical tree-walk CFR, closed-form
equilibria, the sequence-form LP, brute-force best responses, backward
induction, textbook regret matching on a matrix game and closed-form regret
trajectories all reach the expected numbers by another route.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gamegen as gg
from pins import (TreeWalkCFR, brute_force_best_response, lp_best_response,
                  lp_game_value, minimax_value, public_best_response)

VARIANTS = ["vanilla", "cfr+", "dcfr", "pcfr+", "pcfr"]
MODES = ["simultaneous", "alternating"]


def _A(g):
    return sp.csr_matrix((g.val, g.col_idx, g.row_ptr), shape=tuple(g.n_seq))


# --------------------------------------------------------------------------
# Classical CFR and sequence-form CFR give identical iterates (Section 2.1,
# Section 5).  This pins the array construction, both sweeps, the payoff
# step, every variant's post-step, the alternation order and the averages.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", ["cfg1", "stops", "s2d3"])
def test_tree_walk_cfr_identical_iterates(oracle_mod, games, name, variant, mode):
    g = games[name]
    o = oracle_mod.Oracle(g)
    tw = TreeWalkCFR(g, variant, mode)
    for _ in range(25):
        o.step(1, variant, mode)
        tw.step(1)
        for p in range(2):
            np.testing.assert_allclose(o.strategy(p), tw.seq_strategy(p), rtol=0, atol=1e-12)
            np.testing.assert_allclose(o.regrets(p), tw.regrets_seq(p), rtol=0, atol=1e-12)
            np.testing.assert_allclose(o.strategy(p, "average"), tw.average_seq(p),
                                       rtol=0, atol=1e-12)


def test_tree_walk_medium_game_few_iterations(oracle_mod):
    g = gg.cfg2_literal()
    o = oracle_mod.Oracle(g)
    tw = TreeWalkCFR(g, "cfr+", "alternating")
    for _ in range(2):
        o.step(1, "cfr+", "alternating")
        tw.step(1)
    for p in range(2):
        np.testing.assert_allclose(o.strategy(p), tw.seq_strategy(p), rtol=0, atol=1e-12)
        np.testing.assert_allclose(o.regrets(p), tw.regrets_seq(p), rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# Closed-form mixed equilibrium of 2x2 zero-sum games with no saddle point.
# --------------------------------------------------------------------------

MATRICES = [[[3.0, -1.0], [-2.0, 1.0]], [[1.0, -1.0], [-1.0, 1.0]],
            [[0.5, -0.25], [-0.75, 0.125]]]


@pytest.mark.parametrize("M", MATRICES)
@pytest.mark.parametrize("variant,mode,iters,tol", [
    ("vanilla", "simultaneous", 20000, 2e-2), ("cfr+", "alternating", 2000, 2e-3),
    ("dcfr", "alternating", 2000, 2e-3), ("pcfr+", "alternating", 2000, 2e-3)])
def test_2x2_closed_form(oracle_mod, M, variant, mode, iters, tol):
    (a, b), (c, d) = M
    den = a - b - c + d
    p_star, q_star, v_star = (d - c) / den, (d - b) / den, (a * d - b * c) / den
    o = oracle_mod.Oracle(gg.matrix_game(M))
    o.step(iters, variant, mode)
    x = o.strategy(0, "average")
    y = o.strategy(1, "average")
    e = o.exploitability("average")
    assert abs(x[1] - p_star) < tol and abs(y[1] - q_star) < tol
    assert abs(e["value"] - v_star) < tol
    assert 0.0 <= e["nash_conv"] < tol


def test_matrix_game_is_plain_regret_matching(oracle_mod):
    """One decision point per player: sequence-form CFR is textbook regret
    matching on the matrix game (simultaneous updates)."""
    rng = np.random.default_rng(5)
    M = rng.uniform(-1, 1, size=(4, 3))
    o = oracle_mod.Oracle(gg.matrix_game(M))
    R1, R2 = np.zeros(4), np.zeros(3)

    def rm(R):
        z = np.maximum(R, 0)
        return z / z.sum() if z.sum() > 0 else np.full(R.size, 1.0 / R.size)

    for _ in range(50):
        x, y = rm(R1), rm(R2)
        u1, u2 = M @ y, -(M.T @ x)
        R1 += u1 - x @ u1
        R2 += u2 - y @ u2
        o.step(1, "vanilla", "simultaneous")
        np.testing.assert_allclose(o.strategy(0)[1:], rm(R1), atol=1e-13)
        np.testing.assert_allclose(o.strategy(1)[1:], rm(R2), atol=1e-13)
        np.testing.assert_allclose(o.regrets(0)[1:], R1, atol=1e-12)


# --------------------------------------------------------------------------
# Sequence-form LP: game value and the sandwich it must satisfy.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["cfg1", "stops", "s2d3"])
def test_lp_value_sandwich_every_checkpoint(oracle_mod, games, name):
    g = games[name]
    v_star, _ = lp_game_value(g)
    o = oracle_mod.Oracle(g)
    for n in (1, 9, 90, 900):
        o.step(n, "vanilla", "simultaneous")
        e = o.exploitability("average")
        # min_y xbar^T A y <= v* <= max_x x^T A ybar
        assert -e["br2"] <= v_star + 1e-9
        assert v_star <= e["br1"] + 1e-9
        assert abs(e["value"] - v_star) <= e["nash_conv"] + 1e-9


def test_cfg1_vanilla_converges_to_lp_value(oracle_mod):
    g = gg.cfg1()
    v_star, _ = lp_game_value(g)
    o = oracle_mod.Oracle(g)
    o.step(10000, "vanilla", "simultaneous")
    e = o.exploitability("average")
    assert e["expl"] < 2e-3
    assert abs(e["value"] - v_star) <= e["nash_conv"] + 1e-12


# --------------------------------------------------------------------------
# Best responses: brute force over pure strategies, an LP over the polytope
# and a public-tree recursion must all equal the oracle's max-sweep.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["s2d3", "stops"])
def test_best_response_brute_force(oracle_mod, games, name):
    g = games[name]
    o = oracle_mod.Oracle(g)
    o.step(7, "cfr+", "alternating")
    xbar, ybar = o.strategy(0, "average"), o.strategy(1, "average")
    e = o.exploitability("average")
    assert e["br1"] == pytest.approx(brute_force_best_response(g, 0, ybar), abs=1e-13)
    assert e["br2"] == pytest.approx(brute_force_best_response(g, 1, xbar), abs=1e-13)
    assert e["br1"] == pytest.approx(public_best_response(g, 0, ybar), abs=1e-13)
    assert e["br2"] == pytest.approx(public_best_response(g, 1, xbar), abs=1e-13)


def test_best_response_lp_cfg1(oracle_mod):
    g = gg.cfg1()
    o = oracle_mod.Oracle(g)
    o.step(13, "dcfr", "alternating")
    xbar, ybar = o.strategy(0, "average"), o.strategy(1, "average")
    e = o.exploitability("average")
    assert e["br1"] == pytest.approx(lp_best_response(g, 0, ybar), abs=1e-9)
    assert e["br2"] == pytest.approx(lp_best_response(g, 1, xbar), abs=1e-9)
    assert e["br1"] == pytest.approx(public_best_response(g, 0, ybar), abs=1e-13)
    assert e["br2"] == pytest.approx(public_best_response(g, 1, xbar), abs=1e-13)


def test_perfect_information_minimax(oracle_mod, games):
    """One signal each: the value is the backward-induction minimax."""
    g = games["perfect"]
    v_star = minimax_value(g)
    o = oracle_mod.Oracle(g)
    o.step(3000, "cfr+", "alternating")
    e = o.exploitability("average")
    assert abs(e["value"] - v_star) < 1e-3
    assert e["expl"] < 1e-3
    assert -e["br2"] <= v_star + 1e-12 <= e["br1"] + 2e-12


# --------------------------------------------------------------------------
# Invariants (Section 2.1 polytope; the sweep computes expected utility).
# --------------------------------------------------------------------------

def _polytope_residual(g, p, x):
    par, first = g.inf_parent[p], g.inf_first_seq[p]
    res = abs(x[0] - 1.0)
    for j in range(g.n_inf[p]):
        res = max(res, abs(x[first[j]:first[j + 1]].sum() - x[par[j]]))
    return res


@pytest.mark.parametrize("variant", VARIANTS)
def test_invariants_each_iteration(oracle_mod, games, variant):
    g = games["stops"]
    o = oracle_mod.Oracle(g)
    for _ in range(40):
        b_t = [o.behavioral(p) for p in range(2)]
        o.step(1, variant, "simultaneous")
        for p in range(2):
            for kind in ("current", "average"):
                x = o.strategy(p, kind)
                assert _polytope_residual(g, p, x) < 1e-14
                assert np.all(x >= 0)
            # the instantaneous regret is orthogonal to the strategy played:
            # sum_a b_a (q_a - v_j) = 0 at every decision point
            q, v = o.last_observation(p)
            first = g.inf_first_seq[p]
            for j in range(g.n_inf[p]):
                sl = slice(first[j], first[j + 1])
                assert abs(np.dot(b_t[p][sl], q[sl] - v[j])) < 1e-14
        assert o.exploitability("average")["nash_conv"] >= -1e-15


def test_sweep_value_equals_expected_utility(oracle_mod, games):
    g = games["cfg1"]
    A = _A(g)
    o = oracle_mod.Oracle(g)
    for _ in range(15):
        x_t, y_t = o.strategy(0), o.strategy(1)
        o.step(1, "vanilla", "simultaneous")
        q, v = o.last_observation(0)
        roots = np.nonzero(g.inf_parent[0] == 0)[0]
        u1 = A @ y_t
        assert u1[0] + v[roots].sum() == pytest.approx(x_t @ u1, abs=1e-14)
        q2, v2 = o.last_observation(1)
        roots2 = np.nonzero(g.inf_parent[1] == 0)[0]
        u2 = -(A.T @ x_t)
        assert u2[0] + v2[roots2].sum() == pytest.approx(y_t @ u2, abs=1e-14)


def test_cfr_regret_bound(oracle_mod, games):
    """Vanilla CFR, simultaneous, uniform averaging: T * NashConv equals the
    sum of the players' overall regrets, which CFR bounds by the sum over
    decision points of the positive part of their largest action regret."""
    g = games["cfg1"]
    o = oracle_mod.Oracle(g)
    for T in (10, 100, 1000):
        o.step(T - o.iteration, "vanilla", "simultaneous")
        nash = o.exploitability("average")["nash_conv"]
        bound = 0.0
        for p in range(2):
            r, first = o.regrets(p), g.inf_first_seq[p]
            for j in range(g.n_inf[p]):
                bound += max(0.0, r[first[j]:first[j + 1]].max())
        assert T * nash <= bound + 1e-9


# --------------------------------------------------------------------------
# DCFR (Algorithm 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", MODES)
def test_dcfr_alpha_beta_one_is_linear_cfr(oracle_mod, games, mode):
    """With alpha = beta = 1 every regret is scaled by t/(t+1) after
    iteration t, so (t+1) r_t = sum_s s * inst_s: linear CFR.  Regret
    matching is scale-free, so the strategies coincide."""
    g = games["stops"]
    o = oracle_mod.Oracle(g, alpha=1.0, beta=1.0)
    tw = TreeWalkCFR(g, "vanilla", mode, inst_weight=lambda t: float(t))
    for t in range(1, 30):
        o.step(1, "dcfr", mode)
        tw.step(1)
        for p in range(2):
            np.testing.assert_allclose(o.strategy(p), tw.seq_strategy(p), atol=1e-12)
            np.testing.assert_allclose(o.regrets(p) * (t + 1), tw.regrets_seq(p),
                                       rtol=1e-12, atol=1e-12)


def _decision_problem():
    """Player 1 alone: one decision point with two actions worth 1 and 0.
    Player 2 has only the empty sequence."""
    return gg._from_triplets("one-decision", [3, 1], [1, 0],
                             [np.zeros(1, np.int32), np.zeros(0, np.int32)],
                             [np.array([1, 3], np.int32), np.array([1], np.int32)],
                             [1], [0], [1.0])


@pytest.mark.parametrize("alpha,beta", [(1.5, 0.0), (2.0, 0.5), (0.5, 3.0)])
def test_dcfr_sign_dependent_discount_closed_form(oracle_mod, alpha, beta):
    """After t=1 the first action is always played, so its regret only ever
    gets the positive-side factor and the second gets -1 per iteration plus
    the negative-side factor:
        r1(T) = 1/2 * prod_{t<=T} t^a/(t^a+1)
        r2(T) = -(1/2 * prod_{t<=T} f(t) + sum_{k=2..T} prod_{t=k..T} f(t)),
    f(t) = t^b/(t^b+1)."""
    o = oracle_mod.Oracle(_decision_problem(), alpha=alpha, beta=beta)
    for T in range(1, 40):
        o.step(1, "dcfr", "alternating")
        pos = [t ** alpha / (t ** alpha + 1) for t in range(1, T + 1)]
        neg = [t ** beta / (t ** beta + 1) for t in range(1, T + 1)]
        r1 = 0.5 * math.prod(pos)
        r2 = -(0.5 * math.prod(neg) + sum(math.prod(neg[k - 1:]) for k in range(2, T + 1)))
        r = o.regrets(0)
        assert r[1] == pytest.approx(r1, rel=1e-12)
        assert r[2] == pytest.approx(r2, rel=1e-12)


def test_cfr_plus_floor_decision_problem(oracle_mod):
    """CFR+ on the same problem: the second action's regret is floored at 0
    after every iteration, the first one's is +1/2 after t=1 and then fixed."""
    o = oracle_mod.Oracle(_decision_problem())
    o.step(10, "cfr+", "alternating")
    r = o.regrets(0)
    assert r[1] == 0.5 and r[2] == 0.0


# --------------------------------------------------------------------------
# Predictive variants (Algorithm 5)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("variant", ["pcfr+", "pcfr"])
@pytest.mark.parametrize("mode", MODES)
def test_literal_algorithm5_matches_stored_prediction(oracle_mod, games, variant, mode):
    g = games["cfg1"]
    a = oracle_mod.Oracle(g)
    b = oracle_mod.Oracle(g, literal_pcfr=True)
    for _ in range(30):
        a.step(1, variant, mode)
        b.step(1, variant, mode)
        for p in range(2):
            np.testing.assert_allclose(a.strategy(p), b.strategy(p), rtol=0, atol=1e-15)
            np.testing.assert_allclose(a.regrets(p), b.regrets(p), rtol=0, atol=1e-15)


def test_pcfr_plus_zero_prediction_is_cfr_plus(oracle_mod, games):
    """The prediction enters only through regret matching: at t=1 there is no
    previous utility, so the first two strategies of PCFR+ and CFR+ agree."""
    g = games["cfg1"]
    a = oracle_mod.Oracle(g, avg="linear")
    b = oracle_mod.Oracle(g, avg="linear")
    a.step(1, "pcfr+", "alternating")
    b.step(1, "cfr+", "alternating")
    for p in range(2):
        np.testing.assert_allclose(a.regrets(p), b.regrets(p), atol=0)
    # the next strategy differs only by the prediction term
    assert np.max(np.abs(a.prediction(0))) > 0


# --------------------------------------------------------------------------
# Convergence (exploitability of the average falls toward zero)
# --------------------------------------------------------------------------

def test_exploitability_falls(oracle_mod, games):
    g = games["cfg1"]
    o = oracle_mod.Oracle(g)
    vals = []
    for T in (10, 100, 1000, 10000):
        o.step(T - o.iteration, "vanilla", "simultaneous")
        vals.append(o.exploitability("average")["expl"])
    assert vals[-1] < vals[0] / 20
    assert all(b <= a * 1.5 for a, b in zip(vals, vals[1:]))
    finals = {}
    for variant in ("cfr+", "dcfr", "pcfr+"):
        o2 = oracle_mod.Oracle(g)
        o2.step(1000, variant, "alternating")
        finals[variant] = o2.exploitability("average")["expl"]
    # the modern variants beat vanilla at equal iterations on this game
    for variant, e in finals.items():
        assert e < vals[2], (variant, e, vals[2])


# --------------------------------------------------------------------------
# The all-core build runs the same per-element arithmetic on every host core
# (rows and columns of the payoff products, the sweeps one level at a time):
# its results equal the plain build's bit for bit, so every pin above holds
# for it too.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("mode", MODES)
def test_all_core_build_is_bit_identical(oracle_mod, games, variant, mode):
    cases = [games["stops"], games["perfect"], gg.make_config("cfg2_d8"),
             gg.public_game(5, S=4, max_depth=5, branch_lo=2, branch_hi=4, p_stop=0.2)]
    for g in cases:
        for literal in ((False, True) if variant in ("pcfr+", "pcfr") else (False,)):
            a = oracle_mod.Oracle(g, literal_pcfr=literal)
            b = oracle_mod.Oracle(g, literal_pcfr=literal, parallel=True)
            for n in (1, 29):
                a.step(n, variant, mode)
                b.step(n, variant, mode)
                for p in range(2):
                    for kind in ("current", "average"):
                        assert np.array_equal(a.strategy(p, kind), b.strategy(p, kind))
                    assert np.array_equal(a.regrets(p), b.regrets(p))
                    assert np.array_equal(a.prediction(p), b.prediction(p))
                for kind in ("current", "average"):
                    ea, eb = a.exploitability(kind), b.exploitability(kind)
                    assert all(ea[k] == eb[k] for k in ea), (ea, eb)
            y = np.random.default_rng(3).random(g.n_seq[1])
            assert a.best_response_to(0, y) == b.best_response_to(0, y)
    assert oracle_mod.threads(parallel=True) >= 1
