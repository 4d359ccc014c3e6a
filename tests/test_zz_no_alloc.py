"""The allocation-free solver (cfr_create_static) against the ordinary one
(cfr_create), through the C ABI.

Both run the same kernels in the same order, so every iterate, regret and
evaluation must be bit for bit the same.  Two solvers in a row share the
static workspace: the second, on a smaller game, must not see anything the
first left in it.
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


def _same_run(cfr, g, precision, variant, mode, iters):
    say(f"case: static vs allocating, {g.name} {precision} {variant} {mode} {iters}")
    ref = cfr.Solver(g, precision=precision)
    st = cfr.Solver(g, precision=precision, static_workspace=True)
    try:
        for n in (1, iters - 1):
            ref.step(n, variant, mode)
            st.step(n, variant, mode)
            assert st.iteration == ref.iteration
            for p in range(2):
                for kind in ("current", "average"):
                    assert np.array_equal(st.strategy(p, kind), ref.strategy(p, kind)), (p, kind)
                assert np.array_equal(st.regrets(p), ref.regrets(p)), p
            for kind in ("current", "average"):
                assert st.exploitability(kind) == ref.exploitability(kind), kind
    finally:
        st.close()
        ref.close()


def test_static_solver_equals_allocating_solver_twice(cfr):
    """Two static solvers in a row, the second on a smaller game, each equal
    to the allocating solver bit for bit."""
    big, small = gg.cfg2_literal(), gg.cfg1()
    assert small.nnz < big.nnz and small.n_seq[0] < big.n_seq[0]
    _same_run(cfr, big, "fp64", "pcfr+", "alternating", 60)
    _same_run(cfr, small, "fp64", "dcfr", "simultaneous", 40)


@pytest.mark.parametrize("precision", ["fp32", "fp32_acc64"])
def test_static_solver_fp32_modes(cfr, precision):
    _same_run(cfr, gg.cfg2_literal(), precision, "cfr+", "alternating", 30)
    _same_run(cfr, gg.cfg1(), precision, "vanilla", "alternating", 30)


def test_static_solver_one_per_device_and_refusals(cfr):
    """A second static solver while one lives is refused (they would share
    the array); after the first is released a new one is made.  Calls that
    would allocate are refused on a static solver."""
    g = gg.cfg1()
    a = cfr.Solver(g, precision="fp64", static_workspace=True)
    try:
        with pytest.raises(cfr.CfrError) as ei:
            cfr.Solver(g, precision="fp64", static_workspace=True)
        assert ei.value.code == cfr.CFR_ESTATE
        for call in (lambda: a.tune(reps=1), lambda: a.kernel_timing(True)):
            with pytest.raises(cfr.CfrError) as ei:
                call()
            assert ei.value.code == cfr.CFR_EUNSUPPORTED
        t = dict(a.tiling)
        t["vec"] = [3, 3]
        t["items"] = [16, 16]
        with pytest.raises(cfr.CfrError) as ei:
            a.tiling = t
        assert ei.value.code == cfr.CFR_EUNSUPPORTED
        a.step(5, "cfr+", "alternating")
    finally:
        a.close()
    b = cfr.Solver(g, precision="fp64", static_workspace=True)
    b.step(5, "cfr+", "alternating")
    assert b.iteration == 5
    b.close()
