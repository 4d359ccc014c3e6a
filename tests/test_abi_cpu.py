"""The C-ABI library on the CPU: it loads, exports every declared symbol,
and its host-only entry points (validation, workspace sizing) behave as the
header states.  No kernel runs here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import gamegen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfr.h")


@pytest.fixture(scope="module")
def cfr():
    import paper_2605_14277_amd as m
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfr_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(cfr):
    lib = C.CDLL(cfr.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_options_default(cfr):
    o = cfr.cfr_options_default()
    assert o.precision == 0 and o.dcfr_alpha == 1.5 and o.dcfr_beta == 0.0
    assert o.dcfr_gamma == 2.0 and o.use_graph == 1 and not o.workspace


@pytest.mark.parametrize("name", ["cfg1", "stops", "perfect"])
def test_valid_games_validate(cfr, games, name):
    ga = cfr.GameArrays(games[name])
    assert cfr.cfr_validate(ga) == cfr.CFR_OK
    ga2 = cfr.GameArrays(games[name], with_csc=False)
    assert cfr.cfr_validate(ga2) == cfr.CFR_OK


def _corrupt(game, what):
    import copy
    g = copy.deepcopy(game)
    if what == "no_action":
        f = g.inf_first_seq[0].copy()
        f[1] = f[0]
        g.inf_first_seq[0] = f
    elif what == "parent_after":
        p = g.inf_parent[0].copy()
        p[-1] = g.n_seq[0] - 1
        g.inf_parent[0] = p
    elif what == "parent_negative":
        p = g.inf_parent[1].copy()
        p[0] = -1
        g.inf_parent[1] = p
    elif what == "offsets_short":
        f = g.inf_first_seq[1].copy()
        f[-1] -= 1
        g.inf_first_seq[1] = f
    elif what == "row_ptr_end":
        r = g.row_ptr.copy()
        r[-1] += 1
        g.row_ptr = r
    elif what == "col_range":
        c = g.col_idx.copy()
        c[3] = g.n_seq[1]
        g.col_idx = c
    elif what == "col_unsorted":
        c = g.col_idx.copy()
        i = int(np.argmax(np.diff(g.row_ptr) >= 2))
        a = g.row_ptr[i]
        c[a], c[a + 1] = c[a + 1], c[a]
        g.col_idx = c
    elif what == "nan":
        v = g.val.copy()
        v[5] = np.nan
        g.val = v
    elif what == "csc_mismatch":
        v = g.val_csc.copy()
        v[0] += 1e-12
        g.val_csc = v
    elif what == "row_ptr_decreasing":
        r = g.row_ptr.copy()
        i = int(np.argmax(np.diff(r) >= 1)) + 1
        r[i] -= 1
        r[i + 1] = r[i] - 1 if i + 1 < r.size - 1 else r[i + 1]
        g.row_ptr = r
    return g


@pytest.mark.parametrize("what", ["no_action", "parent_after", "parent_negative", "offsets_short",
                                  "row_ptr_end", "col_range", "col_unsorted", "nan",
                                  "csc_mismatch", "row_ptr_decreasing"])
def test_malformed_games_rejected(cfr, games, what):
    g = _corrupt(games["cfg1"], what)
    rc = cfr.cfr_validate(cfr.GameArrays(g))
    assert rc == cfr.CFR_EINVAL, what
    assert cfr.cfr_last_error() != ""


def test_bad_options_rejected(cfr, games):
    ga = cfr.GameArrays(games["cfg1"])
    o = cfr.cfr_options_default()
    o.precision = 7
    with pytest.raises(cfr.CfrError) as ei:
        cfr.cfr_workspace_size(ga, o)
    assert ei.value.code == cfr.CFR_EINVAL
    o = cfr.cfr_options_default()
    o.dcfr_alpha = float("inf")
    with pytest.raises(cfr.CfrError):
        cfr.cfr_workspace_size(ga, o)


def test_workspace_linear_in_game_size(cfr):
    """Space is linear in the treeplex sizes plus nnz (Theorem 2): bytes per
    (sequence + nonzero) stay within a constant band across sizes."""
    ratios = {}
    for prec in ("fp64", "fp32", "fp32_acc64"):
        o = cfr.cfr_options_default()
        o.precision = cfr.PRECISIONS[prec]
        rs = []
        for g in (gg.cfg1(), gg.cfg2_literal(),
                  gg.public_game(9, S=8, max_depth=8, branch_lo=2, branch_hi=3, p_stop=0.1)):
            n = cfr.cfr_workspace_size(cfr.GameArrays(g), o)
            units = g.n_seq[0] + g.n_seq[1] + g.nnz
            rs.append(n / units)
        ratios[prec] = rs
        # 48 bytes per sequence of state at most, 2*(4+8) per nonzero, plus alignment
        assert max(rs[1:]) < 80
    assert ratios["fp32"][-1] < ratios["fp64"][-1]


def test_workspace_independent_of_numbering(cfr, games):
    from helpers import dfs_renumber
    g = games["stops"]
    h = dfs_renumber(g)
    o = cfr.cfr_options_default()
    assert cfr.cfr_validate(cfr.GameArrays(h)) == cfr.CFR_OK
    a = cfr.cfr_workspace_size(cfr.GameArrays(g), o)
    b = cfr.cfr_workspace_size(cfr.GameArrays(h), o)
    assert abs(a - b) <= 4096


def test_create_without_device_fails_cleanly(cfr, games):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ga = cfr.GameArrays(games["cfg1"])
    o = cfr.cfr_options_default()
    with pytest.raises(cfr.CfrError) as ei:
        cfr.cfr_create(ga, o)
    assert ei.value.code == cfr.CFR_EDEVICE


def test_null_solver_calls(cfr):
    lib = C.CDLL(cfr.LIB_PATH)
    lib.cfr_step.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int]
    assert lib.cfr_step(None, 1, 0, 0) == cfr.CFR_EINVAL
    lib.cfr_destroy.argtypes = [C.c_void_p]
    assert lib.cfr_destroy(None) == cfr.CFR_OK


# ---- batches (host side only) ------------------------------------------------

def test_batch_defaults_and_game_size(cfr, games):
    o = cfr.cfr_batch_options_default()
    assert o.precision == cfr.PRECISIONS["fp32_acc64"] and o.mode == cfr.MODES["alternating"]
    assert o.max_games == 256 and o.check_every == 10 and o.use_graph == 1
    gp = cfr.cfr_game_params_default()
    assert gp.variant == cfr.VARIANTS["pcfr+"] and gp.target_exploitability == 0
    g = games["stops"]
    u = cfr.cfr_batch_game_size(cfr.GameArrays(g))
    # sequence blocks are rounded up to a multiple of four
    r4 = lambda n: -(-n // 4) * 4
    assert list(u) == [r4(g.n_seq[0] + 1), r4(g.n_seq[1] + 1), g.n_inf[0] + 1, g.n_inf[1] + 1,
                       g.nnz]


def _batch_opts(cfr, seq, inf, nnz, **kw):
    o = cfr.cfr_batch_options_default()
    for p in range(2):
        o.seq_capacity[p] = seq[p]
        o.inf_capacity[p] = inf[p]
    o.nnz_capacity = nnz
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_batch_workspace_linear_in_capacity(cfr):
    """A batch's bytes grow linearly with its index and nonzero capacities:
    the per-unit cost of a capacity ten times larger stays within a few
    percent of the smaller one."""
    small = cfr.cfr_batch_workspace_size(_batch_opts(cfr, [10**5, 3 * 10**5], [4 * 10**4, 10**5],
                                                     10**7))
    large = cfr.cfr_batch_workspace_size(_batch_opts(cfr, [10**6, 3 * 10**6], [4 * 10**5, 10**6],
                                                     10**8))
    assert 9.5 < large / small < 10.5
    # nonzeros dominate: two index/value copies (CSR and CSC) of 8 bytes each
    per_nnz = (cfr.cfr_batch_workspace_size(_batch_opts(cfr, [10**5, 10**5], [10**4, 10**4], 2 * 10**7))
               - cfr.cfr_batch_workspace_size(_batch_opts(cfr, [10**5, 10**5], [10**4, 10**4], 10**7))) / 10**7
    assert 16 <= per_nnz < 17


def test_index_limits_at_the_boundaries(cfr):
    """Value slots hold 4 * sequence + rank in an int32: used up to a
    sequence capacity of 2^29, off above it.  Quad words keep the column's
    group of four in 28 bits: stream form 3 allowed up to a column capacity
    of 2^30, refused above it (per product: A y's columns are player 2's
    sequences, A^T x's player 1's)."""
    def lim(s1, s2):
        return cfr.cfr_batch_index_limits(_batch_opts(cfr, [s1, s2], [10, 10], 1000))
    assert lim(2**29 - 1, 2**29) == {"slots": [True, True], "quads": [True, True]}
    assert lim(2**29 + 1, 2**29)["slots"] == [False, True]
    assert lim(2**29, 2**29 + 4)["slots"] == [True, False]
    assert lim(2**30, 2**30)["quads"] == [True, True]
    assert lim(2**30, 2**30 + 1)["quads"] == [False, True]
    assert lim(2**30 + 4, 2**30)["quads"] == [True, False]
    assert lim(2**31 - 1, 2**31 - 1) == {"slots": [False, False], "quads": [False, False]}
    # a capacity the index type cannot hold at all is refused
    with pytest.raises(cfr.CfrError) as ei:
        lim(2**31, 10)
    assert ei.value.code == cfr.CFR_EINVAL


@pytest.mark.parametrize("field,value", [("quad_capacity", -1), ("precision", 9), ("mode", 3),
                                         ("max_games", 0),
                                         ("check_every", 0), ("nnz_capacity", -1),
                                         ("spmv_order", 5)])
def test_batch_bad_options_rejected(cfr, field, value):
    o = _batch_opts(cfr, [100, 100], [10, 10], 1000, **{field: value})
    with pytest.raises(cfr.CfrError) as ei:
        cfr.cfr_batch_workspace_size(o)
    assert ei.value.code == cfr.CFR_EINVAL


def test_batch_create_without_device_fails_cleanly(cfr):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(cfr.CfrError) as ei:
        cfr.cfr_batch_create(_batch_opts(cfr, [100, 100], [10, 10], 1000))
    assert ei.value.code == cfr.CFR_EDEVICE


def test_null_batch_calls(cfr):
    lib = C.CDLL(cfr.LIB_PATH)
    lib.cfr_batch_run.argtypes = [C.c_void_p, C.c_int64, C.c_void_p]
    assert lib.cfr_batch_run(None, 1, None) == cfr.CFR_EINVAL
    lib.cfr_batch_destroy.argtypes = [C.c_void_p]
    assert lib.cfr_batch_destroy(None) == cfr.CFR_OK
    lib.cfr_tune.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    assert lib.cfr_tune(None, 3, None) == cfr.CFR_EINVAL


def test_prepare_without_device(cfr, games):
    """cfr_prepare is host work only: it runs (and sizes the game) with no
    device, keeping its streams in ordinary memory when none can be locked."""
    from paper_2605_14277_amd import serve
    g = games["stops"]
    for prec in ("fp64", "fp32_acc64"):
        p = serve.Prepared(g, prec)
        assert list(p.units) == list(cfr.cfr_batch_game_size(cfr.GameArrays(g)))
        p.close()
    # host-built quad copies need no device either
    p = serve.Prepared(g, "fp32_acc64", quads=(1, 0))
    p.prepare_quads((0, 1))
    with pytest.raises(cfr.CfrError) as ei:
        p.prepare_quads((2, 0))
    assert ei.value.code == cfr.CFR_EINVAL
    p.close()
    import copy
    g2 = copy.copy(games["cfg1"])
    g2.col_idx = np.array(g2.col_idx, dtype=np.int32, copy=True)
    g2.col_idx[0] = 10**6
    bad = cfr.GameArrays(g2)
    with pytest.raises(cfr.CfrError) as ei:
        h = C.c_void_p()
        rc = cfr._lib.cfr_prepare(C.byref(bad.desc), 0, C.byref(h))
        cfr._check(rc, "cfr_prepare")
    assert ei.value.code == cfr.CFR_EINVAL


def test_tuning_cache_by_size_bucket(tmp_path):
    """The tuning cache stores one tiling per size bucket and hands it back
    without timing anything; another bucket, precision or kind tunes anew."""
    from paper_2605_14277_amd import LIB_PATH
    from paper_2605_14277_amd.tuning import size_key, tune_cached

    class Fake:
        def __init__(self, choice):
            self.tiling, self.choice, self.calls = None, choice, 0

        def tune(self, reps):
            self.calls += 1
            self.tiling = dict(self.choice)
            return self.tiling

    path = str(tmp_path / "tiling.json")
    t1 = {"items": [16, 16], "rows": [256, 256], "vec": [3, 3], "perm": [0, 1]}
    t2 = {"items": [8, 8], "rows": [128, 128], "vec": [2, 2], "perm": [1, 1]}
    k = size_key("solver", "fp32_acc64", 100_555_072, [1_218_369, 3_648_993], 1, LIB_PATH)
    # within the same powers of two: the same bucket
    assert k == size_key("solver", "fp32_acc64", 1.1e8, [1.3e6, 3.5e6], 1, LIB_PATH)
    assert k != size_key("solver", "fp64", 100_555_072, [1_218_369, 3_648_993], 1, LIB_PATH)
    assert k != size_key("batch", "fp32_acc64", 100_555_072, [1_218_369, 3_648_993], 1, LIB_PATH)
    assert k != size_key("solver", "fp32_acc64", 4e8, [1_218_369, 3_648_993], 1, LIB_PATH)
    a = Fake(t1)
    assert tune_cached(a, k, path, 3) == (t1, False) and a.calls == 1
    b = Fake(t2)
    assert tune_cached(b, k, path, 3) == (t1, True) and b.calls == 0 and b.tiling == t1
    k2 = size_key("solver", "fp64", 100_555_072, [1_218_369, 3_648_993], 1, LIB_PATH)
    c = Fake(t2)
    assert tune_cached(c, k2, path, 3) == (t2, False) and c.calls == 1
    import json
    assert json.load(open(path)) == {k: t1, k2: t2}


def test_static_solver_refusals_on_the_host(cfr, games):
    """cfr_create_static refuses, before any device call: a game whose
    device state exceeds the static workspace (CFR_ENOMEM), a caller
    workspace (CFR_EINVAL); a game that fits reaches the device check."""
    o = cfr.cfr_options_default()
    big = cfr.GameArrays(gg.cfg2())
    assert cfr.cfr_workspace_size(big, o) > cfr.STATIC_WORKSPACE_BYTES
    with pytest.raises(cfr.CfrError) as ei:
        cfr.cfr_create_static(big, o)
    assert ei.value.code == cfr.CFR_ENOMEM
    small = cfr.GameArrays(games["cfg1"])
    o.workspace = C.c_void_p(4096)
    o.workspace_bytes = 1 << 20
    with pytest.raises(cfr.CfrError) as ei:
        cfr.cfr_create_static(small, o)
    assert ei.value.code == cfr.CFR_EINVAL
    import torch
    if not torch.cuda.is_available():
        o = cfr.cfr_options_default()
        with pytest.raises(cfr.CfrError) as ei:
            cfr.cfr_create_static(small, o)
        assert ei.value.code == cfr.CFR_EDEVICE


def test_static_workspace_size_matches_header(cfr):
    text = open(HEADER).read()
    m = re.search(r"#define CFR_STATIC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == cfr.STATIC_WORKSPACE_BYTES
