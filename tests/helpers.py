"""Test helpers: renumbering games and comparing results."""
import numpy as np

import gamegen as gg


def dfs_renumber(game):
    """The same game with decision points numbered in depth-first preorder
    (still a valid topological order, but not level order), so the library
    must permute it internally."""
    n_inf = [int(v) for v in game.n_inf]
    new_par, new_first, new_of_old = [], [], []
    for p in range(2):
        par = game.inf_parent[p]
        first = game.inf_first_seq[p]
        kids = {}
        for j in range(n_inf[p]):
            kids.setdefault(int(par[j]), []).append(j)
        mapping = np.zeros(game.n_seq[p], np.int64)
        order = []
        nxt = [1]

        def visit(j):
            order.append(j)
            for a in range(int(first[j]), int(first[j + 1])):
                mapping[a] = nxt[0]
                nxt[0] += 1
            for a in range(int(first[j]), int(first[j + 1])):
                for c in kids.get(a, []):
                    visit(c)

        for j in kids.get(0, []):
            visit(j)
        # reverse the roots' subtrees too, so even level 0 changes order
        f, pa = [], []
        for j in order:
            f.append(mapping[first[j]])
            pa.append(mapping[par[j]] if par[j] > 0 else 0)
        f.append(game.n_seq[p])
        new_first.append(np.array(f, np.int32))
        new_par.append(np.array(pa, np.int32))
        new_of_old.append(mapping)
    r = np.repeat(np.arange(game.n_seq[0]), np.diff(game.row_ptr))
    rows = new_of_old[0][r]
    cols = new_of_old[1][game.col_idx]
    h = gg._from_triplets(game.name + "-dfs", list(game.n_seq), n_inf, new_par, new_first,
                          rows, cols, game.val)
    h.meta["new_of_old"] = new_of_old
    return h


def rel_inf(a, ref):
    """||a - ref||_inf / max(1, ||ref||_inf)."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(a - ref)) / max(1.0, float(np.max(np.abs(ref)))))


# Lines printed at the end of a test session (pytest_terminal_summary in
# conftest.py): the FP32 modes' errors against the FP64 oracle, so that
# every reported FP32 result carries its error even under `pytest -q`.
SESSION_REPORT = []


def report(line: str):
    print(line, flush=True)
    SESSION_REPORT.append(line)
