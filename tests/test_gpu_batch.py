"""Batches of games on the GPU, through the C ABI.

No reduction in the library mixes two games, and a game's product blocks
are the same alone and in a batch, so every game's iterates in a batch must
equal the same game solved alone bit for bit, in every precision, whatever
else shares the launches.  FP64 results are also held to the oracle at
1e-9.  Games stop at checks on their own targets and limits, and games join
and leave between runs without disturbing the others.
"""
import sys

import numpy as np
import pytest

import gamegen as gg
from helpers import rel_inf

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


@pytest.fixture(scope="module")
def mix(games):
    from test_oracle_pins import _decision_problem
    return [
        ("cfg1", games["cfg1"], "cfr+"),
        ("stops", games["stops"], "dcfr"),
        ("s2d3", games["s2d3"], "pcfr+"),
        ("perfect", games["perfect"], "vanilla"),
        ("cfg2_d8", gg.cfg2_literal(), "pcfr"),
        ("showdown", gg.public_game(4, S=6, max_depth=6, branch_lo=2, branch_hi=4, p_stop=0.1,
                                    payoff_kind="showdown"), "dcfr"),
        ("one-decision", _decision_problem(), "cfr+"),
    ]


def capacity(cfr, games, slack=0):
    s = np.sum([cfr.Batch.game_size(g) for g in games], axis=0) + slack
    return [int(s[0]), int(s[1])], [int(s[2]), int(s[3])], int(s[4])


def make_batch(cfr, games, slack=0, **kw):
    seq, inf, nnz = capacity(cfr, games, slack)
    return cfr.Batch(seq, inf, nnz, **kw)


def lone(cfr, g, variant, mode, iters, precision):
    s = cfr.Solver(g, precision=precision)
    if iters:
        s.step(iters, variant, mode)
    return s


def assert_same(batch, gid, solo, what):
    for p in range(2):
        for kind in ("current", "average"):
            a, b = batch.strategy(gid, p, kind), solo.strategy(p, kind)
            assert np.array_equal(a, b), (what, p, kind, float(np.max(np.abs(a - b))))
    for kind in ("current", "average"):
        eb, es = batch.exploitability(gid, kind), solo.exploitability(kind)
        for k in ("expl", "br1", "br2", "value"):
            assert eb[k] == es[k], (what, kind, k, eb[k], es[k])


@pytest.mark.parametrize("precision,mode", [("fp64", "alternating"), ("fp64", "simultaneous"),
                                            ("fp32_acc64", "alternating"),
                                            ("fp32", "alternating")])
def test_batch_equals_lone_and_oracle(cfr, oracle_mod, mix, precision, mode):
    say(f"case: batch of {len(mix)} games, {precision}, {mode}")
    b = make_batch(cfr, [g for _, g, _ in mix], max_games=len(mix), precision=precision,
                   mode=mode, check_every=10)
    ids = [b.add(g, variant) for _, g, variant in mix]
    iters = 60
    assert b.run(iters) == len(mix)
    for (name, g, variant), gid in zip(mix, ids):
        st = b.status(gid)
        assert st["state"] == "active" and st["iterations"] == iters, st
        solo = lone(cfr, g, variant, mode, iters, precision)
        assert_same(b, gid, solo, name)
        solo.close()
        if precision == "fp64":
            orc = oracle_mod.Oracle(g)
            orc.step(iters, variant, mode)
            worst = 0.0
            for p in range(2):
                for kind in ("current", "average"):
                    worst = max(worst, rel_inf(b.strategy(gid, p, kind), orc.strategy(p, kind)))
            eb, eo = b.exploitability(gid), orc.exploitability("average")
            worst = max(worst, abs(eb["nash_conv"] - eo["nash_conv"]) / max(1, abs(eo["nash_conv"])))
            say(f"  {name} {variant}: oracle rel err {worst:.2e}")
            assert worst <= 1e-9, name
            orc.close()
    b.close()


def test_targets_stop_games_at_checks(cfr, mix):
    """Each game stops at the first check where its average exploitability
    is at most its target (or its limit is reached); its state is then that
    of the game solved alone for the same number of iterations."""
    K = 10
    chosen = [m for m in mix if m[0] in ("cfg1", "stops", "s2d3", "showdown")]
    b = make_batch(cfr, [g for _, g, _ in chosen], max_games=8, precision="fp64",
                   mode="alternating", check_every=K)
    ids, targets = [], {}
    for name, g, variant in chosen:
        target = 5e-3 if name != "showdown" else 0.0
        gid = b.add(g, variant, target=target, max_iterations=300)
        ids.append(gid)
        targets[gid] = target
    rounds = 0
    while b.run(50) > 0:
        rounds += 1
        assert rounds < 20
    for (name, g, variant), gid in zip(chosen, ids):
        st = b.status(gid)
        say(f"  {name}: {st}")
        assert st["state"] == "done" and st["iterations"] % K == 0
        assert st["evaluated_at"] == st["iterations"]
        if st["reached_target"]:
            assert st["expl"] <= targets[gid]
            if st["iterations"] > K:
                prev = lone(cfr, g, variant, "alternating", st["iterations"] - K, "fp64")
                assert prev.exploitability("average")["expl"] > targets[gid]
                prev.close()
        else:
            assert st["iterations"] == 300
        solo = lone(cfr, g, variant, "alternating", st["iterations"], "fp64")
        assert solo.exploitability("average")["expl"] == st["expl"]
        assert_same(b, gid, solo, name)
        solo.close()
    b.close()


QUADS = {"items": [16, 16], "rows": [256, 256], "vec": [3, 3], "perm": [0, 1], "xcd": [1, 0]}


@pytest.mark.parametrize("tiling", [None, QUADS], ids=["elements", "quads"])
def test_games_join_and_leave(cfr, mix, tiling):
    """Games join at checks and leave between them; their ranges (and, in
    stream form 3, their quad copies) are reused, and every game still
    equals the same game solved alone."""
    K = 10
    pool = {name: (g, v) for name, g, v in mix}
    b = make_batch(cfr, [pool[n][0] for n in ("cfg1", "stops", "s2d3", "cfg2_d8")],
                   max_games=4, precision="fp64", mode="alternating", check_every=K)
    if tiling is not None:
        b.tiling = tiling
    g1 = b.add(*pool["cfg1"])
    g2 = b.add(*pool["stops"])
    b.run(30)
    g3 = b.add(*pool["s2d3"])  # at a check: starts at once
    assert b.status(g3)["state"] == "active"
    b.run(20)
    b.remove(g1)  # its ranges are reused below
    g4 = b.add(*pool["cfg2_d8"])
    b.run(25)  # ends between two checks
    b.remove(g4)
    g5 = b.add(*pool["cfg1"])
    assert b.status(g5)["state"] == "waiting"
    b.run(5)  # reaches the check; g5 starts at the next run
    assert b.status(g5)["iterations"] == 0
    b.run(10)
    expect = {g2: ("stops", 90), g3: ("s2d3", 60), g5: ("cfg1", 10)}
    for gid, (name, iters) in expect.items():
        assert b.status(gid)["iterations"] == iters, (name, b.status(gid))
        g, variant = pool[name]
        solo = lone(cfr, g, variant, "alternating", iters, "fp64")
        assert_same(b, gid, solo, name)
        solo.close()
    b.close()


def test_capacity_and_errors(cfr, mix):
    g_small, g_big = mix[0][1], mix[4][1]
    b = make_batch(cfr, [g_big, g_small], max_games=2, precision="fp32_acc64")
    first = b.add(g_big, "cfr+")
    with pytest.raises(cfr.CfrError) as ei:
        b.add(g_big, "cfr+")
    assert ei.value.code == cfr.CFR_ENOMEM
    gid = b.add(g_small, "cfr+")  # the small game fits beside it
    with pytest.raises(cfr.CfrError):
        b.add(g_small, "cfr+")  # no slot left
    b.remove(first)
    again = b.add(g_big, "dcfr")
    b.run(10)
    assert b.status(again)["iterations"] == 10 and b.status(gid)["iterations"] == 10
    with pytest.raises(cfr.CfrError):
        b.status(first)
    b.close()


def test_tiling_and_tuner(cfr, mix):
    """Row sums in FP64 are sequential per row whatever the tiling, so a
    retiled or tuned batch reproduces the default one bit for bit (no row
    here exceeds the smallest block capacity)."""
    games = [g for _, g, _ in mix]
    out = []
    for tiling in (None,
                   {"items": [4, 8], "rows": [64, 128], "vec": [0, 1], "perm": [1, 0], "xcd": [1, 0]},
                   {"items": [16, 4], "rows": [256, 64], "vec": [1, 0], "perm": [0, 1], "xcd": [0, 1]},
                   {"items": [8, 8], "rows": [128, 128], "vec": [1, 1], "perm": [1, 1], "xcd": [1, 1]},
                   {"items": [16, 8], "rows": [256, 128], "vec": [2, 2], "perm": [0, 1], "xcd": [0, 0]},
                   {"items": [4, 16], "rows": [64, 256], "vec": [2, 0], "perm": [1, 0], "xcd": [1, 0]},
                   {"items": [16, 16], "rows": [256, 64], "vec": [3, 3], "perm": [0, 1], "xcd": [0, 1]},
                   {"items": [16, 8], "rows": [128, 256], "vec": [3, 2], "perm": [1, 1], "xcd": [1, 1]},
                   {"items": [8, 8], "rows": [64, 256], "vec": [3, 3], "perm": [1, 0], "xcd": [0, 0]},
                   "tune"):
        b = make_batch(cfr, games, max_games=len(mix), precision="fp64")
        ids = [b.add(g, v) for _, g, v in mix]
        if tiling == "tune":
            chosen = b.tune(reps=3)
            say(f"  tuner chose {chosen}")
            assert all(i in (4, 8, 16) for i in chosen["items"])
            assert all(64 <= r <= 256 for r in chosen["rows"])
            assert all(v in (0, 1, 2, 3) for v in chosen["vec"])
            assert all(v in (0, 1) for v in chosen["perm"])
            assert all(v in (0, 1) for v in chosen["xcd"])
        elif tiling is not None:
            b.tiling = tiling
            assert b.tiling == tiling
        b.run(40)
        out.append([b.strategy(gid, p, "average") for gid in ids for p in range(2)])
        b.close()
    for other in out[1:]:
        for a, c in zip(out[0], other):
            assert np.array_equal(a, c)


@pytest.mark.parametrize("precision", ["fp32_acc64", "fp32"])
def test_stream_load_forms_agree(cfr, mix, precision):
    """The three ways of reading the index and value streams stage every
    product at the same place, so with the same blocks the FP32 row sums
    (lane groups) come out bit for bit the same."""
    games = [g for _, g, _ in mix]
    out = []
    for vec in (0, 1, 2):
        b = make_batch(cfr, games, max_games=len(mix), precision=precision)
        ids = [b.add(g, v) for _, g, v in mix]
        b.tiling = {"items": [8, 16], "rows": [128, 256], "vec": [vec, vec], "perm": [0, 1]}
        b.run(30)
        out.append([b.strategy(gid, p, "average") for gid in ids for p in range(2)])
        b.close()
    for other in out[1:]:
        for a, c in zip(out[0], other):
            assert np.array_equal(a, c)


def test_tuning_cache(cfr, tmp_path):
    """A tiling tuned once for a size bucket is taken by the next solver or
    batch of that bucket."""
    g = gg.cfg2_literal()
    path = str(tmp_path / "tiling.json")
    s = cfr.Solver(g, precision="fp32_acc64")
    first = s.tune(reps=2, cache=path)
    s.close()
    s = cfr.Solver(g, precision="fp32_acc64")
    assert s.tune(reps=2, cache=path) == first and s.tiling == first
    s.close()
    games = [g, g]
    b = make_batch(cfr, games, max_games=2)
    for x in games:
        b.add(x, "cfr+")
    tb = b.tune(reps=2, cache=path)
    b.close()
    b = make_batch(cfr, games, max_games=2)
    for x in games:
        b.add(x, "cfr+")
    assert b.tune(reps=2, cache=path) == tb and b.tiling == tb
    b.close()


def test_single_solver_tune(cfr, oracle_mod):
    g = gg.cfg2_literal()
    s = cfr.Solver(g, precision="fp64")
    chosen = s.tune(reps=3)
    say(f"  tuner chose {chosen} for the depth-8 game")
    assert s.tiling == chosen
    s.step(100, "cfr+", "alternating")
    orc = oracle_mod.Oracle(g)
    orc.step(100, "cfr+", "alternating")
    for p in range(2):
        assert rel_inf(s.strategy(p, "average"), orc.strategy(p, "average")) <= 1e-9
    s.close()
    orc.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64", "fp32"])
def test_chain_top_down_pass_equals_level_by_level(cfr, mix, precision):
    """The one-launch top-down pass multiplies each sequence's parent chain
    from the root down, the same products in the same order as one launch
    per level: identical strategies, averages and regrets."""
    for name, g, variant in mix:
        out = []
        for down in ("default", "levels"):
            s = cfr.Solver(g, precision=precision, down_pass=down)
            s.step(40, variant, "alternating")
            out.append([s.strategy(p, k) for p in range(2) for k in ("current", "average")] +
                       [s.regrets(p) for p in range(2)])
            s.close()
        for a, b in zip(*out):
            assert np.array_equal(a, b), (name, precision)


@pytest.mark.parametrize("tiling", [None, QUADS, dict(QUADS, perm=[1, 1])],
                         ids=["elements", "quads", "quads-from-images"])
def test_asynchronous_admission(cfr, mix, tiling):
    """Admission copies run on their own stream: a game added while others
    iterate joins at the next check, one added to an idle batch at once, and
    every game still equals the same game solved alone.  With quads, the
    prepared games carry host-built quad copies in first-touch column order:
    a product in that order copies them, the other (A y in identity order
    under QUADS) builds its own on the device."""
    from paper_2605_14277_amd import serve
    pool = {name: (g, v) for name, g, v in mix}
    names = ("cfg1", "stops", "s2d3", "cfg2_d8")
    preps = {n: serve.Prepared(pool[n][0], "fp64", quads=(1, 1) if tiling else None)
             for n in names}
    units = np.sum([preps[n].units for n in names], axis=0)
    # with quads from images, a store reserved at creation (then grown)
    b = cfr.Batch([units[0], units[1]], [units[2], units[3]], int(units[4]), max_games=4,
                  precision="fp64", check_every=10, async_admission=True,
                  quad_capacity=1000 if tiling is not None and tiling["perm"] == [1, 1] else 0)
    if tiling is not None:
        b.tiling = tiling
    g1 = serve.add_prepared(b, preps["cfg1"], pool["cfg1"][1])
    assert b.status(g1)["state"] == "active"  # idle batch: joins at once
    b.run(20)
    g2 = serve.add_prepared(b, preps["stops"], pool["stops"][1])
    g3 = serve.add_prepared(b, preps["cfg2_d8"], pool["cfg2_d8"][1])
    assert b.status(g2)["state"] == "waiting"
    b.run(10)  # the copies overlap this period; g2 and g3 join at its check
    assert b.status(g2)["iterations"] == 0
    b.run(30)
    expect = {g1: ("cfg1", 60), g2: ("stops", 30), g3: ("cfg2_d8", 30)}
    for gid, (name, iters) in expect.items():
        assert b.status(gid)["iterations"] == iters, (name, b.status(gid))
        g, variant = pool[name]
        solo = lone(cfr, g, variant, "alternating", iters, "fp64")
        assert_same(b, gid, solo, name)
        solo.close()
    b.close()
    for p in preps.values():
        p.close()


def test_many_games_in_one_batch(cfr, mix):
    """Sixty games (copies of the mix under every variant) packed into one
    batch: the tables hold every game's blocks and levels, and each game
    still equals the same game solved alone."""
    variants = ["vanilla", "cfr+", "dcfr", "pcfr+", "pcfr"]
    entries = []
    for rep in range(2):
        for vi, v in enumerate(variants):
            for name, g, _ in mix[:6]:
                entries.append((name, g, v))
    b = make_batch(cfr, [g for _, g, _ in entries], max_games=len(entries), precision="fp32_acc64",
                   check_every=10)
    b.tiling = QUADS  # the same tiling for the lone solves below
    ids = [b.add(g, v) for _, g, v in entries]
    b.run(30)
    seen = set()
    for (name, g, v), gid in zip(entries, ids):
        if (name, v) in seen:
            continue
        seen.add((name, v))
        solo = cfr.Solver(g, precision="fp32_acc64")
        solo.tiling = QUADS
        solo.step(30, v, "alternating")
        assert_same(b, gid, solo, f"{name}/{v}")
        solo.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
def test_asynchronous_check_periods_equal_run(cfr, mix, precision):
    """Check periods begun and ended asynchronously (cfr_batch_run_begin /
    cfr_batch_run_end) give the same iterates, checks and stops as
    cfr_batch_run, bit for bit; between the two calls only status queries
    and cfr_batch_run_ready are allowed."""
    games = [g for _, g, _ in mix]
    targets = {name: 1e-3 * (float(np.ptp(g.val)) if g.nnz else 1.0) for name, g, _ in mix}
    out = []
    for asynchronous in (False, True):
        b = make_batch(cfr, games, max_games=len(mix), precision=precision, check_every=10)
        ids = [b.add(g, v, target=targets[name], max_iterations=300) for name, g, v in mix]
        if asynchronous:
            left = len(ids)
            rounds = 0
            while left:
                b.run_begin()
                if rounds == 0:
                    assert b.status(ids[0])["iterations"] >= 0  # allowed
                    for call in (lambda: b.run(10), lambda: b.strategy(ids[0], 0, "average"),
                                 lambda: b.add(games[0], "cfr+"), lambda: b.remove(ids[0])):
                        with pytest.raises(cfr.CfrError) as ei:
                            call()
                        assert ei.value.code == cfr.CFR_ESTATE
                if rounds % 2:
                    while not b.run_ready():  # polled, then ended without waiting
                        pass
                left = b.run_end()
                assert b.run_ready()
                rounds += 1
            assert b.run_end() == 0  # nothing begun: nothing to do
        else:
            b.run(100000)
        st = [b.status(gid) for gid in ids]
        out.append(([(x["iterations"], x["reached_target"], x["expl"]) for x in st],
                    [b.strategy(gid, p, "average") for gid in ids for p in range(2)]))
        b.close()
    assert out[0][0] == out[1][0]
    for a, c in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, c)


@pytest.mark.parametrize("name", ["cfg2", "no-shallow-p2"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
def test_game_left_alone_uses_its_own_sweep_structures(cfr, games, name, precision):
    """A batch whose other games have finished iterates the game left alone
    with that game's own one-block shallow levels and fused levels (from
    its prepared plan, at a nonzero index base: a finished game sits before
    it), after running a launch per level while both iterated; the result
    equals the lone solver's bit for bit.  The second game's player 2 has
    no shallow pass, so its fused launch starts at level 0."""
    if name == "cfg2":
        g = gg.cfg2()
    else:
        g = gg.public_game(11, S=96, max_depth=6, branch_lo=2, branch_hi=3, p_stop=0.1,
                           payoff_kind="showdown", name="no-shallow-p2")
    first = games["stops"]
    b = make_batch(cfr, [first, g], max_games=2, precision=precision, check_every=10)
    a = b.add(first, "cfr+", max_iterations=20)  # finishes after two checks
    k = b.add(g, "dcfr", max_iterations=70)
    while b.run(10):
        pass
    assert b.status(a)["iterations"] == 20 and b.status(k)["iterations"] == 70
    solo = lone(cfr, g, "dcfr", "alternating", 70, precision)
    assert_same(b, k, solo, f"{name} left alone ({precision})")
    solo.close()
    b.close()
