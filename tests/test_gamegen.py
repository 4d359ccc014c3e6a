"""The seeded input generator: sizes, determinism, and the payoff matrix
checked against a direct path-by-path construction."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import gamegen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gamegen_sha256.json")


def test_cfg1_sizes():
    g = gg.cfg1()
    assert g.tree.n_terminals == 16
    assert g.n_seq == [31, 61]
    assert g.n_inf == [15, 30]
    assert g.nnz == 144


def test_determinism_against_stored_hashes():
    with open(GOLDEN) as f:
        ref = json.load(f)
    for name in ("cfg1", "cfg2_d8"):
        assert gg.make_config(name).sha256() == ref[name], name


@pytest.mark.parametrize("name", ["cfg1", "s2d3", "stops", "perfect"])
def test_treeplex_well_formed(games, name):
    g = games[name]
    for p in range(2):
        par, first = g.inf_parent[p], g.inf_first_seq[p]
        assert first.shape[0] == g.n_inf[p] + 1
        assert first[0] == 1 and first[-1] == g.n_seq[p]
        assert np.all(np.diff(first) >= 1)
        assert np.all(par < first[:-1])
        assert np.all(par >= 0)


@pytest.mark.parametrize("name", ["cfg1", "s2d3", "stops", "perfect"])
def test_csc_is_csr_transpose(games, name):
    g = games[name]
    A = sp.csr_matrix((g.val, g.col_idx, g.row_ptr), shape=tuple(g.n_seq))
    B = sp.csc_matrix((g.val_csc, g.row_idx, g.col_ptr), shape=tuple(g.n_seq))
    assert (A != B).nnz == 0
    for ptr, idx in ((g.row_ptr, g.col_idx), (g.col_ptr, g.row_idx)):
        for i in range(ptr.shape[0] - 1):
            seg = idx[ptr[i]:ptr[i + 1]]
            assert np.all(np.diff(seg) > 0)


def _last_sequence(g, z, player, signal):
    """Walk from terminal z to the root; return the player's last sequence."""
    t = g.tree
    lookup = {(int(g.seq_node[player][i]), int(g.seq_signal[player][i]),
               int(g.seq_action[player][i])): i for i in range(1, g.n_seq[player])}
    cur = int(t.terminals[z])
    while t.parent[cur] >= 0:
        par = int(t.parent[cur])
        if (int(t.depth[par]) & 1) == player:
            return lookup[(par, signal, int(t.action[cur]))]
        cur = par
    return 0


@pytest.mark.parametrize("name", ["cfg1", "stops", "perfect"])
def test_payoff_matrix_by_paths(games, name):
    """A[s1_seq, s2_seq] = sum chance * u over terminals and signal pairs."""
    g = games[name]
    S1, S2 = g.S
    A = np.zeros(tuple(g.n_seq))
    for z in range(g.tree.n_terminals):
        for s1 in range(S1):
            r = _last_sequence(g, z, 0, s1)
            for s2 in range(S2):
                c = _last_sequence(g, z, 1, s2)
                A[r, c] += float(g.utility(np.array(z), np.array(s1), np.array(s2))) / (S1 * S2)
    B = sp.csr_matrix((g.val, g.col_idx, g.row_ptr), shape=tuple(g.n_seq)).toarray()
    np.testing.assert_allclose(B, A, rtol=0, atol=1e-15)


def test_showdown_ties_not_stored():
    g = gg.public_game(3, S=4, max_depth=3, branch_lo=2, branch_hi=2, p_stop=0.0,
                       payoff_kind="showdown")
    # every terminal contributes S*(S-1) nonzeros: ties are exact zeros
    assert g.nnz == g.tree.n_terminals * 4 * 3
    assert np.all(g.val != 0.0)


@pytest.mark.parametrize("S,depth,lo,hi", [(8, 6, 900, 1100), (16, 8, 9000, 11000)])
def test_showdown_sized(S, depth, lo, hi):
    """The size sweep's games: the terminal count falls in the window, every
    terminal contributes one nonzero per ordered pair of distinct signals
    (ties are exact zeros and are not stored), and the draw is repeatable."""
    g = gg.showdown_sized(S, depth, lo, hi, "sized")
    T = g.tree.n_terminals
    assert lo <= T <= hi
    assert g.nnz == T * S * (S - 1)
    h = gg.showdown_sized(S, depth, lo, hi, "sized")
    assert np.array_equal(g.val, h.val) and np.array_equal(g.col_idx, h.col_idx)
