"""Serving with continuous batching, through the C ABI.

Requests arrive while others are iterating; they are prepared on worker
threads, admitted at check boundaries as slots and device ranges free up,
and freed when they meet their stopping rule.  Each result must be the same
as the game solved alone (bit for bit: same iterates, same checks) and match
the FP64 oracle (FP64: the oracle run for as many iterations; FP32 modes:
the oracle's evaluation of the served profile), and the requests must really
share the device (admitted while others are in flight).  Requests that
cannot be served are rejected without disturbing the others.
"""
import sys

import numpy as np
import pytest

import gamegen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2605_14277_amd as m
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests(pool, n, mean_gap, seed):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for k in range(n):
        t += rng.exponential(mean_gap)
        i = int(rng.integers(0, len(pool)))
        rel = [1e-2, 1e-3][int(rng.integers(0, 2))]
        out.append({"arrival": t, "game": pool[i], "variant": ["cfr+", "dcfr"][k % 2],
                    "target": rel * gg.payoff_range(pool[i]), "max_iterations": 150})
    return out


QUADS = {"items": [16, 16], "rows": [256, 256], "vec": [3, 3], "perm": [1, 1], "xcd": [0, 0]}


def _small_lane(cfr, pool, limit):
    """A small-game lane for the pool games of at most `limit` nonzeros,
    with room for about two of them at once."""
    units = sorted((cfr.Batch.game_size(g) for g in pool if g.nnz <= limit), key=lambda u: -u[4])
    cap = np.sum(units[:2], axis=0)
    return {"seq_capacity": [cap[0], cap[1]], "inf_capacity": [cap[2], cap[3]],
            "nnz_capacity": int(cap[4]), "max_games": 3, "nnz_limit": limit}


@pytest.mark.parametrize("lanes,solo", [(1, 0), (2, 0), (2, 1)],
                         ids=["one-lane", "two-lanes", "two-lanes-solo"])
@pytest.mark.parametrize("tiling", [None, QUADS], ids=["elements", "quads"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
def test_served_results_equal_alone(cfr, games, precision, tiling, lanes, solo):
    from paper_2605_14277_amd import serve
    pool = [games["cfg1"], games["stops"], games["s2d3"], games["perfect"], gg.cfg2_literal()]
    reqs = _requests(pool, 20, 0.004, seed=3)
    # room for about three games at once, so requests also wait for space
    units = sorted((cfr.Batch.game_size(g) for g in pool), key=lambda u: -u[4])
    cap = np.sum(units[:3], axis=0)
    # two lanes: the four small games (at most 1000 nonzeros) apart from the
    # medium game, each lane a batch on a stream of its own
    small = _small_lane(cfr, pool, 1000) if lanes == 2 else None
    # solo: the lane of the medium game holds one game and admits another
    # beside it only after a wait of 2 ms
    srv = serve.Server([cap[0], cap[1]], [cap[2], cap[3]], int(cap[4]), max_games=4,
                       precision=precision, check_every=10, workers=4, tiling=tiling, small=small,
                       solo=solo, admit_after=0.002)
    out = srv.serve(reqs, keep_strategies=True)
    srv.close()
    if lanes == 2:
        used = {o["lane"] for o in out}
        assert used == {0, 1}, used
        for r, o in zip(reqs, out):
            assert o["lane"] == (0 if r["game"].nnz <= 1000 else 1)
    overlaps = sum(1 for i in range(len(out)) for j in range(i + 1, len(out))
                   if out[i]["admitted"] < out[j]["finished"] and
                   out[j]["admitted"] < out[i]["finished"])
    say(f"  {precision}: {len(out)} requests, {overlaps} overlapping pairs, latency p50 "
        f"{np.percentile([o['latency'] for o in out], 50) * 1e3:.1f} ms")
    assert overlaps > 0
    for k, (r, o) in enumerate(zip(reqs, out)):
        assert o["iterations"] % 10 == 0 and o["latency"] >= 0
        assert o["admitted"] >= r["arrival"] and o["finished"] >= o["admitted"]
        if o["reached_target"]:
            assert o["expl"] <= r["target"]
        else:
            assert o["iterations"] == 150
        solo = cfr.Solver(r["game"], precision=precision)
        if tiling is not None:
            solo.tiling = tiling
        solo.step(o["iterations"], r["variant"], "alternating")
        for p in range(2):
            assert np.array_equal(o["strategy"][p], solo.strategy(p, "average")), (k, p)
        assert solo.exploitability("average")["expl"] == o["expl"], k
        solo.close()
        check_against_oracle(r, o, precision)


def check_against_oracle(r, o, precision):
    """A served result against the FP64 oracle.  FP64: the oracle run for
    the same number of iterations, within 1e-9 (relative) on both average
    strategies and NashConv.  FP32 modes: the served exploitability within
    1e-4 of the oracle's evaluation of the served profile (the trajectory
    itself is compared with the oracle's and the difference printed: at a
    few hundred iterations CFR+ and DCFR amplify any rounding difference,
    so trajectories of implementations that round differently need not
    agree to 1e-4 there)."""
    import oracle
    from helpers import rel_inf, report
    orc = oracle.Oracle(r["game"])
    orc.step(o["iterations"], r["variant"], "alternating")
    eo = orc.exploitability("average")
    if precision == "fp64":
        for p in range(2):
            d = rel_inf(o["strategy"][p], orc.strategy(p, "average"))
            assert d <= 1e-9, (p, d)
        assert abs(2 * o["expl"] - eo["nash_conv"]) <= 1e-9 * max(1.0, abs(eo["nash_conv"]))
    else:
        x, y = o["strategy"]
        own = 0.5 * (orc.best_response_to(0, y) + orc.best_response_to(1, x))
        xbar = max(float(np.max(np.abs(o["strategy"][p] - orc.strategy(p, "average"))))
                   for p in range(2))
        report(f"[serve {precision} {r['game'].name} {r['variant']} t={o['iterations']}] "
               f"expl served {o['expl']:.6e} oracle trajectory {eo['expl']:.6e} "
               f"(|d| {abs(o['expl'] - eo['expl']):.1e}, xbar {xbar:.1e}) | oracle on the "
               f"served profile {own:.6e} (|d| {abs(o['expl'] - own):.1e})")
        assert abs(o["expl"] - own) <= 1e-4
    orc.close()


def _malformed(game):
    """The game with one decision point given no action (cfr_prepare and
    cfr_validate refuse it with CFR_EINVAL)."""
    import copy
    g = copy.deepcopy(game)
    f = g.inf_first_seq[0].copy()
    f[1] = f[0]
    g.inf_first_seq[0] = f
    return g


@pytest.mark.parametrize("lanes", [1, 2], ids=["one-lane", "two-lanes"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
def test_served_stream_with_cap_malformed_and_oversized_requests(cfr, games, precision, lanes):
    """A stream in which one request stops on its iteration limit while
    others run (a target it cannot reach), one game is malformed and one is
    larger than the whole batch: the two are answered as rejected
    (CFR_EINVAL, CFR_ENOMEM) while the loop keeps serving, and every served
    result equals the game solved alone bit for bit and the FP64 oracle."""
    from paper_2605_14277_amd import serve
    pool = [games["cfg1"], games["stops"], games["s2d3"], games["perfect"]]
    reqs = _requests(pool, 14, 0.003, seed=11)
    # never reachable: stops on its 150-iteration limit
    reqs[3]["target"] = 1e-12
    big = gg.cfg2_literal()
    units = sorted((cfr.Batch.game_size(g) for g in pool), key=lambda u: -u[4])
    cap = np.sum(units[:3], axis=0)
    assert np.any(cfr.Batch.game_size(big) > cap)
    bad = dict(reqs[5], game=_malformed(reqs[5]["game"]))
    over = dict(reqs[8], game=big)
    reqs[5], reqs[8] = bad, over
    small = _small_lane(cfr, pool, 1000) if lanes == 2 else None
    srv = serve.Server([cap[0], cap[1]], [cap[2], cap[3]], int(cap[4]), max_games=4,
                       precision=precision, check_every=10, workers=4, small=small)
    out = srv.serve(reqs, keep_strategies=True)
    srv.close()
    assert out[5]["state"] == "rejected" and out[5]["code"] == cfr.CFR_EINVAL, out[5]
    assert out[8]["state"] == "rejected" and out[8]["code"] == cfr.CFR_ENOMEM, out[8]
    assert out[3]["state"] == "done" and out[3]["iterations"] == 150
    assert not out[3]["reached_target"]
    served = [k for k in range(len(reqs)) if k not in (5, 8)]
    overlaps = sum(1 for i in served for j in served if i < j and
                   out[i]["admitted"] < out[j]["finished"] and
                   out[j]["admitted"] < out[i]["finished"])
    assert overlaps > 0
    # the capped request shared the device with others while it ran
    assert any(out[3]["admitted"] < out[j]["finished"] and out[j]["admitted"] < out[3]["finished"]
               for j in served if j != 3)
    for k in served:
        r, o = reqs[k], out[k]
        assert o["state"] == "done"
        solo = cfr.Solver(r["game"], precision=precision)
        solo.step(o["iterations"], r["variant"], "alternating")
        for p in range(2):
            assert np.array_equal(o["strategy"][p], solo.strategy(p, "average")), (k, p)
        assert solo.exploitability("average")["expl"] == o["expl"], k
        solo.close()
        check_against_oracle(r, o, precision)
    say(f"  {precision}: {len(served)} served ({overlaps} overlapping pairs), 2 rejected")


def test_prepared_game_reuse_and_precision_check(cfr, games):
    from paper_2605_14277_amd import serve
    g = games["stops"]
    prep = serve.Prepared(g, "fp64")
    assert list(prep.units) == list(cfr.Batch.game_size(g))
    u = prep.units
    b = cfr.Batch([2 * u[0], 2 * u[1]], [2 * u[2], 2 * u[3]], int(2 * u[4]), max_games=2,
                  precision="fp64")
    a = serve.add_prepared(b, prep, "cfr+")
    c = serve.add_prepared(b, prep, "cfr+")  # the same prepared game twice
    b.run(30)
    assert np.array_equal(b.strategy(a, 0, "average"), b.strategy(c, 0, "average"))
    other = cfr.Batch([u[0], u[1]], [u[2], u[3]], int(u[4]), max_games=1, precision="fp32")
    with pytest.raises(cfr.CfrError) as ei:
        serve.add_prepared(other, prep, "cfr+")
    assert ei.value.code == cfr.CFR_EINVAL
    other.close()
    b.close()
    prep.close()
