"""Seeded synthetic two-player zero-sum games in sequence form.

This module builds the *inputs* of the solver and nothing else: a public game
tree, private signals, terminal payoffs, and from them the two players'
treeplexes (tree-form sequential decision processes, Section 2.1 of the paper)
plus the sequence-form payoff matrix A in CSR and CSC.  It holds none of the
CFR arithmetic; both the CPU oracle and the GPU library consume its arrays.

Game model (the paper evaluates on OpenSpiel games that are not available
here; these synthetic games stand in for them):

* A public tree whose actions are seen by both players.  The owner of a node
  alternates with depth: player 1 at even depth, player 2 at odd depth.  The
  root is always internal.
* Each player privately observes a signal drawn uniformly and independently
  (S1 and S2 values), so chance reaches every signal pair with 1/(S1*S2).
* An information set (decision point) is (player, own signal, public node).
  Opponent actions and the player's own signal are observation points.
* Terminal payoffs u(z, s1, s2) are player 1's utility; player 2 gets -u.

Sequence-form payoff matrix: A[s1_seq, s2_seq] = sum over terminals z and
signal pairs of chance(s1,s2) * u(z,s1,s2), where sX_seq is player X's last
sequence on the path to z given its signal (the empty sequence 0 if it never
acted).  Exact zeros are not stored.

Sequence numbering (both players): sequence 0 is the empty sequence; then
decision levels in order (level = number of own earlier decisions); inside a
level, public nodes in breadth-first order, then signals, then actions.
This order is topological (every infoset's parent sequence precedes its own
sequences), and the columns of any payoff row (the opponent's sequences at
one public node, over all opponent signals) are one short contiguous run.

Random draws (numpy PCG64, one Generator per game): the public tree level by
level in breadth-first order (branching of every internal node of the level,
then one stop draw per child that is above the maximum depth), then the
payoffs over terminals in breadth-first order.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "PublicTree", "Game", "make_public_tree", "build_game", "public_game",
    "matrix_game", "cfg1", "cfg2", "cfg2_literal", "cfg3", "CONFIGS",
    "make_config",
]


# --------------------------------------------------------------------------
# Public tree
# --------------------------------------------------------------------------

@dataclass
class PublicTree:
    depth: np.ndarray        # int32 [n_nodes]
    parent: np.ndarray       # int32 [n_nodes], -1 at the root
    action: np.ndarray       # int32 [n_nodes], action index taken at parent
    child_first: np.ndarray  # int32 [n_nodes], first child id (-1 if terminal)
    n_child: np.ndarray      # int32 [n_nodes], 0 for terminals
    term_id: np.ndarray      # int32 [n_nodes], terminal index or -1
    terminals: np.ndarray    # int32 [T], node ids of terminals (BFS order)

    @property
    def n_nodes(self) -> int:
        return int(self.depth.shape[0])

    @property
    def n_terminals(self) -> int:
        return int(self.terminals.shape[0])

    def owner(self, node: int) -> int:
        return int(self.depth[node]) & 1


def make_public_tree(rng: np.random.Generator, max_depth: int,
                     branch_lo: int, branch_hi: int, p_stop: float,
                     fixed_branching: bool = False,
                     branch_p_hi: float | None = None) -> PublicTree:
    """Breadth-first random public tree.

    Each internal node draws its branching uniformly from
    {branch_lo..branch_hi} (or, with ``branch_p_hi``, branch_hi with that
    probability and branch_lo otherwise); each child above ``max_depth``
    becomes terminal with probability ``p_stop``; children at ``max_depth``
    are terminal.  The root never stops.
    """
    if max_depth < 1:
        raise ValueError("max_depth must be >= 1")
    depth = [np.zeros(1, np.int32)]
    parent = [np.full(1, -1, np.int32)]
    action = [np.full(1, -1, np.int32)]
    internal_levels = [np.zeros(1, np.int64)]   # internal node ids per depth
    nchild_of = {}                               # depth -> (ids, k)
    next_id = 1
    cur = np.zeros(1, np.int64)
    for d in range(max_depth):
        if cur.size == 0:
            break
        if fixed_branching:
            k = np.full(cur.size, branch_lo, np.int64)
        elif branch_p_hi is not None:
            k = np.where(rng.random(cur.size) < branch_p_hi, branch_hi, branch_lo).astype(np.int64)
        else:
            k = rng.integers(branch_lo, branch_hi + 1, size=cur.size)
        nchild_of[d] = (cur, k)
        n_new = int(k.sum())
        ids = np.arange(next_id, next_id + n_new, dtype=np.int64)
        next_id += n_new
        par = np.repeat(cur, k)
        starts = np.repeat(np.cumsum(k) - k, k)
        act = np.arange(n_new, dtype=np.int64) - starts
        depth.append(np.full(n_new, d + 1, np.int32))
        parent.append(par.astype(np.int32))
        action.append(act.astype(np.int32))
        if d + 1 < max_depth and p_stop > 0.0:
            stop = rng.random(n_new) < p_stop
        elif d + 1 < max_depth:
            stop = np.zeros(n_new, bool)
        else:
            stop = np.ones(n_new, bool)
        cur = ids[~stop]
        internal_levels.append(cur)
    depth = np.concatenate(depth)
    parent = np.concatenate(parent)
    action = np.concatenate(action)
    n = depth.shape[0]
    child_first = np.full(n, -1, np.int32)
    n_child = np.zeros(n, np.int32)
    # children of a depth's internal nodes are laid out contiguously, in order
    base = 1
    for d in sorted(nchild_of):
        ids, k = nchild_of[d]
        # children of depth-d nodes start right after all nodes of depth <= d
        first = base + np.cumsum(k) - k
        child_first[ids] = first.astype(np.int32)
        n_child[ids] = k.astype(np.int32)
        base += int(k.sum())
    is_term = n_child == 0
    terminals = np.nonzero(is_term)[0].astype(np.int32)
    term_id = np.full(n, -1, np.int32)
    term_id[terminals] = np.arange(terminals.size, dtype=np.int32)
    return PublicTree(depth, parent, action, child_first, n_child, term_id,
                      terminals)


# --------------------------------------------------------------------------
# Game container
# --------------------------------------------------------------------------

@dataclass
class Game:
    """Arrays in the layout the C-ABI (and the oracle) take.

    Per player p: ``n_seq[p]`` (sequence 0 = empty sequence), ``n_inf[p]``,
    ``inf_parent[p]`` (int32, parent sequence of each infoset) and
    ``inf_first_seq[p]`` (int32, n_inf+1 offsets; infoset j owns sequences
    [inf_first_seq[j], inf_first_seq[j+1])).  Payoff A (player 1's payoff,
    chance folded in) as CSR (row_ptr int64, col_idx int32, val float64) and
    CSC (col_ptr, row_idx, val_csc) of the same matrix.
    """
    name: str
    n_seq: list
    n_inf: list
    inf_parent: list
    inf_first_seq: list
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    col_ptr: np.ndarray
    row_idx: np.ndarray
    val_csc: np.ndarray
    # description used by independent checks (tree walks); may be None
    tree: PublicTree | None = None
    S: tuple = (1, 1)
    payoff_kind: str = ""
    payoff: np.ndarray | None = None       # iid: [T,S1,S2]; showdown: pot[T]
    seed: int | None = None
    meta: dict = field(default_factory=dict)
    # per player: node/signal/action of every sequence (for tree walks)
    seq_node: list | None = None
    seq_signal: list | None = None
    seq_action: list | None = None

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def utility(self, z: np.ndarray, s1: np.ndarray, s2: np.ndarray) -> np.ndarray:
        """Player 1's terminal payoff u(z, s1, s2) (terminal index z)."""
        return _utility(self.payoff_kind, self.payoff, z, s1, s2)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for p in range(2):
            h.update(np.int64(self.n_seq[p]).tobytes())
            h.update(np.int64(self.n_inf[p]).tobytes())
            h.update(np.ascontiguousarray(self.inf_parent[p]).tobytes())
            h.update(np.ascontiguousarray(self.inf_first_seq[p]).tobytes())
        for a in (self.row_ptr, self.col_idx, self.val,
                  self.col_ptr, self.row_idx, self.val_csc):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def summary(self) -> dict:
        return {
            "name": self.name, "seed": self.seed,
            "n_seq": [int(v) for v in self.n_seq],
            "n_inf": [int(v) for v in self.n_inf],
            "nnz": self.nnz,
            "terminals": (self.tree.n_terminals if self.tree is not None else None),
            "S": list(self.S),
        }


def _utility(kind, payoff, z, s1, s2):
    if kind == "iid":
        return payoff[z, s1, s2]
    if kind == "showdown":
        return np.sign(np.asarray(s1, np.int64) - np.asarray(s2, np.int64)) * payoff[z]
    if kind == "matrix":
        return payoff[s1, s2]
    raise ValueError(kind)


# --------------------------------------------------------------------------
# Treeplex construction for a public-tree game
# --------------------------------------------------------------------------

@dataclass
class _Plex:
    n_seq: int
    n_inf: int
    S: int
    inf_parent: np.ndarray
    inf_first_seq: np.ndarray
    level_base: np.ndarray   # first sequence index of each level (int64)
    level_nodes: list        # decision nodes of each level, breadth-first
    node_level: np.ndarray   # per public node: level if a decision node of p, else -1
    node_pos: np.ndarray     # per public node: actions of earlier nodes of its level
    node_k: np.ndarray       # per public node: number of actions
    seq_node: np.ndarray
    seq_signal: np.ndarray
    seq_action: np.ndarray


def _treeplex(tree: PublicTree, p: int, S: int) -> _Plex:
    """Player p's treeplex.  Inside a level the decision points are ordered
    node-major, signal-minor: sequence (n, s, a) of a level is
    level_base + S*pos(n) + s*k(n) + a.  Nodes that follow each other in the
    public tree are then neighbours for every signal, which keeps the
    columns of any payoff row (and the rows of any column) close together."""
    internal = tree.n_child > 0
    owned = internal & ((tree.depth & 1) == p)
    node_level = np.full(tree.n_nodes, -1, np.int64)
    node_pos = np.full(tree.n_nodes, -1, np.int64)
    node_k = tree.n_child.astype(np.int64)
    levels = []
    max_depth = int(tree.depth.max()) if tree.n_nodes else 0
    for d in range(p, max_depth + 1, 2):
        ids = np.nonzero(owned & (tree.depth == d))[0]
        if ids.size == 0:
            break
        levels.append(ids)
    level_base = np.zeros(len(levels), np.int64)
    inf_parent_parts, inf_first_parts = [], []
    seq_node_parts, seq_sig_parts, seq_act_parts = [], [], []
    base = 1
    for lv, ids in enumerate(levels):
        k = node_k[ids]
        K = int(k.sum())
        pos = np.cumsum(k) - k
        node_level[ids] = lv
        node_pos[ids] = pos
        level_base[lv] = base
        idx = np.repeat(np.arange(ids.size, dtype=np.int64), S)
        s = np.tile(np.arange(S, dtype=np.int64), ids.size)
        first = base + S * pos[idx] + s * k[idx]
        if lv == 0:
            par = np.zeros(ids.size * S, np.int64)
        else:
            pnode = tree.parent[ids].astype(np.int64)     # opponent node
            g = tree.parent[pnode].astype(np.int64)       # own previous node
            ag = tree.action[pnode].astype(np.int64)      # own action at g
            assert np.all(node_level[g] == lv - 1)
            par = level_base[lv - 1] + S * node_pos[g][idx] + s * node_k[g][idx] + ag[idx]
        inf_parent_parts.append(par)
        inf_first_parts.append(first)
        cnt = S * k
        block0 = np.repeat(np.cumsum(cnt) - cnt, cnt)
        local = np.arange(S * K, dtype=np.int64) - block0
        kk = np.repeat(k, cnt)
        seq_node_parts.append(np.repeat(ids, cnt))
        seq_sig_parts.append(local // kk)
        seq_act_parts.append(local % kk)
        base += S * K
    n_seq = base
    if inf_first_parts:
        inf_first = np.concatenate(inf_first_parts + [np.array([n_seq])])
        inf_parent = np.concatenate(inf_parent_parts)
        seq_node = np.concatenate([[-1]] + seq_node_parts)
        seq_signal = np.concatenate([[-1]] + seq_sig_parts)
        seq_action = np.concatenate([[-1]] + seq_act_parts)
    else:
        inf_first = np.array([n_seq])
        inf_parent = np.zeros(0, np.int64)
        seq_node = seq_signal = seq_action = np.array([-1])
    return _Plex(n_seq, inf_parent.shape[0], S, inf_parent.astype(np.int32),
                 inf_first.astype(np.int32), level_base, levels, node_level, node_pos,
                 node_k, seq_node.astype(np.int32), seq_signal.astype(np.int32),
                 seq_action.astype(np.int32))


def _last_slots(tree: PublicTree, plex: _Plex, p: int):
    """For every terminal: the level, node and action of player p's last
    sequence on its path (level -1 when player p never acts)."""
    z = tree.terminals.astype(np.int64)
    par = tree.parent[z].astype(np.int64)
    lvl = np.full(z.size, -1, np.int64)
    node = np.full(z.size, -1, np.int64)
    act = np.full(z.size, -1, np.int64)
    own_is_parent = (tree.depth[par] & 1) == p
    # the parent of z is p's node: (parent, action(z))
    m = own_is_parent
    lvl[m] = plex.node_level[par[m]]
    node[m] = par[m]
    act[m] = tree.action[z[m]]
    # else the grandparent is p's node: (grandparent, action(parent))
    m2 = ~own_is_parent & (tree.depth[par] >= 1)
    gp = tree.parent[par[m2]].astype(np.int64)
    lvl[m2] = plex.node_level[gp]
    node[m2] = gp
    act[m2] = tree.action[par[m2]]
    return lvl, node, act


def _seq_index(plex: _Plex, lvl, node, act, s):
    """Sequence index of (level, node, action, signal); 0 where lvl < 0."""
    lvl = np.asarray(lvl)
    if plex.level_base.shape[0] == 0:          # the player never acts
        return np.zeros(lvl.shape, np.int64)
    safe = np.where(lvl < 0, 0, lvl)
    nd = np.where(lvl < 0, 0, node)
    idx = (plex.level_base[safe] + plex.S * plex.node_pos[nd] +
           np.asarray(s, np.int64) * plex.node_k[nd] + act)
    return np.where(lvl < 0, 0, idx)


_CHUNK = 1 << 23   # payoff entries expanded at once


def _sorted_matrix(major: int, plex: list, slots: list, S: tuple,
                   ufun, chance: float):
    """Payoff matrix sorted along the ``major`` player's sequences (major=0
    gives the CSR of A, major=1 the CSR of A^T, i.e. the CSC of A).

    Every row is a sequence (n, s, a) of the major player; its entries come
    from the terminals whose major-player last sequence is (n, a), one per
    minor signal (or one entry summed over the minor signals when the minor
    player never acts on the path).  The pattern of a slot (n, a) does not
    depend on s, so it is built once and expanded for every signal.

    Returns (ptr int64[n_major+1], idx int32[nnz], val float64[nnz]).
    """
    mn = 1 - major
    PM, Pm = plex[major], plex[mn]
    SM, Sm = S[major], S[mn]
    lvM, ndM, acM = slots[major]
    lvm, ndm, acm = slots[mn]

    def u_of(z, sM, sm):
        if major == 0:
            return chance * ufun(z, sM, sm)
        return chance * ufun(z, sm, sM)

    def pair_sum(z, s1):
        # sum over player 2's signal of chance*u(z, s1, s2), always through
        # this one function so the CSR and the CSC entries agree bit for bit
        s2 = np.arange(S[1], dtype=np.int64)
        return (chance * ufun(z[:, None], s1[:, None], s2[None, :])).sum(axis=1)

    def pair_sum_p1(z, s2):
        s1 = np.arange(S[0], dtype=np.int64)
        return (chance * ufun(z[:, None], s1[None, :], s2[:, None])).sum(axis=1)

    def summed(z, sM):
        return pair_sum(z, sM) if major == 0 else pair_sum_p1(z, sM)

    chunks_idx, chunks_val, row_len = [], [], []

    # --- row 0 (major player's empty sequence): terminals where the major
    # player never acts; value summed over the major player's signal.
    zs = np.nonzero(lvM < 0)[0]
    if zs.size:
        zz = np.repeat(zs, Sm)
        sm = np.tile(np.arange(Sm, dtype=np.int64), zs.size)
        cols = _seq_index(Pm, lvm[zz], ndm[zz], acm[zz], sm)
        vals = pair_sum_p1(zz, sm) if major == 0 else pair_sum(zz, sm)
        order = np.lexsort((zz, cols))
        cols, vals = cols[order], vals[order]
        uc, inv = np.unique(cols, return_inverse=True)
        acc = np.zeros(uc.size)
        np.add.at(acc, inv, vals)
        keep = acc != 0.0
        chunks_idx.append(uc[keep]); chunks_val.append(acc[keep])
        row_len.append(np.array([int(keep.sum())]))
    else:
        row_len.append(np.array([0]))

    for lv, nodes in enumerate(PM.level_nodes):
        k = PM.node_k[nodes]
        K = int(k.sum())
        zl = np.nonzero(lvM == lv)[0]
        minor_none = lvm[zl] < 0
        z_full = zl[~minor_none]
        z_sum = zl[minor_none]
        pz = np.concatenate([np.repeat(z_full, Sm), z_sum])
        ps = np.concatenate([np.tile(np.arange(Sm, dtype=np.int64), z_full.size),
                             np.full(z_sum.size, -1, np.int64)])
        pslot = PM.node_pos[ndM[pz]] + acM[pz]
        pcol = np.where(ps < 0, 0, _seq_index(Pm, lvm[pz], ndm[pz], acm[pz], np.maximum(ps, 0)))
        order = np.lexsort((pcol, pslot))
        pz, ps, pslot, pcol = pz[order], ps[order], pslot[order], pcol[order]
        if pz.size > 1:
            dup = (pslot[1:] == pslot[:-1]) & (pcol[1:] == pcol[:-1])
            if dup.any():
                raise AssertionError("duplicate payoff entry in one row")
        pat_len = np.bincount(pslot, minlength=K)[:K].astype(np.int64)
        pat_ptr = np.zeros(K + 1, np.int64)
        np.cumsum(pat_len, out=pat_ptr[1:])
        # rows of this level in order: node-major, then signal, then action
        cnt = SM * k
        n_rows = int(cnt.sum())
        block0 = np.repeat(np.cumsum(cnt) - cnt, cnt)
        local = np.arange(n_rows, dtype=np.int64) - block0
        kk = np.repeat(k, cnt)
        row_sig = local // kk
        row_slot = np.repeat(PM.node_pos[nodes], cnt) + local % kk
        lens = pat_len[row_slot]
        r0 = 0
        while r0 < n_rows:
            # rows [r0, r1) holding about _CHUNK entries
            csum = np.cumsum(lens[r0:])
            r1 = r0 + max(1, int(np.searchsorted(csum, _CHUNK)))
            r1 = min(r1, n_rows)
            L = lens[r0:r1]
            tot = int(L.sum())
            starts = pat_ptr[row_slot[r0:r1]]
            ex = np.repeat(starts - (np.cumsum(L) - L), L) + np.arange(tot, dtype=np.int64)
            z = pz[ex]
            sm = ps[ex]
            sMv = np.repeat(row_sig[r0:r1], L)
            vals = np.empty(tot)
            f = sm >= 0
            vals[f] = u_of(z[f], sMv[f], sm[f])
            if not f.all():
                nf = ~f
                vals[nf] = summed(z[nf], sMv[nf])
            keep = vals != 0.0
            rid = np.repeat(np.arange(r1 - r0, dtype=np.int64), L)
            chunks_idx.append(pcol[ex][keep]); chunks_val.append(vals[keep])
            row_len.append(np.bincount(rid[keep], minlength=r1 - r0)[: r1 - r0])
            r0 = r1
    n_major = PM.n_seq
    lens_all = np.concatenate(row_len).astype(np.int64)
    assert lens_all.shape[0] == n_major, (lens_all.shape, n_major)
    ptr = np.zeros(n_major + 1, np.int64)
    np.cumsum(lens_all, out=ptr[1:])
    idx = (np.concatenate(chunks_idx) if chunks_idx else np.zeros(0)).astype(np.int32)
    val = (np.concatenate(chunks_val) if chunks_val else np.zeros(0)).astype(np.float64)
    return ptr, idx, val


def build_game(tree: PublicTree, S1: int, S2: int, payoff_kind: str,
               payoff: np.ndarray, name: str = "game", seed=None) -> Game:
    S = (S1, S2)
    plex = [_treeplex(tree, 0, S1), _treeplex(tree, 1, S2)]
    slots = [_last_slots(tree, plex[0], 0), _last_slots(tree, plex[1], 1)]
    chance = 1.0 / (S1 * S2)

    def ufun(z, s1, s2):
        return _utility(payoff_kind, payoff, z, s1, s2)

    row_ptr, col_idx, val = _sorted_matrix(0, plex, slots, S, ufun, chance)
    col_ptr, row_idx, val_csc = _sorted_matrix(1, plex, slots, S, ufun, chance)
    return Game(
        name=name,
        n_seq=[plex[0].n_seq, plex[1].n_seq],
        n_inf=[plex[0].n_inf, plex[1].n_inf],
        inf_parent=[plex[0].inf_parent, plex[1].inf_parent],
        inf_first_seq=[plex[0].inf_first_seq, plex[1].inf_first_seq],
        row_ptr=row_ptr, col_idx=col_idx, val=val,
        col_ptr=col_ptr, row_idx=row_idx, val_csc=val_csc,
        tree=tree, S=S, payoff_kind=payoff_kind, payoff=payoff, seed=seed,
        seq_node=[plex[0].seq_node, plex[1].seq_node],
        seq_signal=[plex[0].seq_signal, plex[1].seq_signal],
        seq_action=[plex[0].seq_action, plex[1].seq_action],
    )


def public_game(seed: int, S: int, max_depth: int, branch_lo: int, branch_hi: int,
                p_stop: float, payoff_kind: str = "iid", name: str = "game",
                fixed_branching: bool = False, S2: int | None = None,
                branch_p_hi: float | None = None) -> Game:
    """One seeded public-tree game (tree draws first, then payoffs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tree = make_public_tree(rng, max_depth, branch_lo, branch_hi, p_stop,
                            fixed_branching=fixed_branching, branch_p_hi=branch_p_hi)
    S1 = S
    S2 = S if S2 is None else S2
    T = tree.n_terminals
    if payoff_kind == "iid":
        payoff = rng.uniform(-1.0, 1.0, size=(T, S1, S2))
    elif payoff_kind == "showdown":
        payoff = rng.uniform(1.0, 8.0, size=T)
    else:
        raise ValueError(payoff_kind)
    return build_game(tree, S1, S2, payoff_kind, payoff, name=name, seed=seed)


# --------------------------------------------------------------------------
# Normal-form (matrix) games as one-infoset treeplexes
# --------------------------------------------------------------------------

def matrix_game(M, name: str = "matrix") -> Game:
    """A zero-sum matrix game: each player has a single decision point under
    the empty sequence; A[1+i, 1+j] = M[i, j] (row player maximises)."""
    M = np.asarray(M, np.float64)
    m, n = M.shape
    rows, cols, vals = [], [], []
    for i in range(m):
        for j in range(n):
            if M[i, j] != 0.0:
                rows.append(1 + i); cols.append(1 + j); vals.append(M[i, j])
    return _from_triplets(name, [m + 1, n + 1], [1, 1],
                          [np.zeros(1, np.int32), np.zeros(1, np.int32)],
                          [np.array([1, m + 1], np.int32), np.array([1, n + 1], np.int32)],
                          np.array(rows), np.array(cols), np.array(vals),
                          payoff_kind="matrix", payoff=M)


def _from_triplets(name, n_seq, n_inf, inf_parent, inf_first, rows, cols, vals,
                   payoff_kind="", payoff=None) -> Game:
    rows = np.asarray(rows, np.int64); cols = np.asarray(cols, np.int64)
    vals = np.asarray(vals, np.float64)
    o = np.lexsort((cols, rows))
    r, c, v = rows[o], cols[o], vals[o]
    row_ptr = np.zeros(n_seq[0] + 1, np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    o2 = np.lexsort((rows, cols))
    r2, c2, v2 = rows[o2], cols[o2], vals[o2]
    col_ptr = np.zeros(n_seq[1] + 1, np.int64)
    np.add.at(col_ptr, c2 + 1, 1)
    col_ptr = np.cumsum(col_ptr)
    return Game(name=name, n_seq=list(n_seq), n_inf=list(n_inf),
                inf_parent=[np.asarray(a, np.int32) for a in inf_parent],
                inf_first_seq=[np.asarray(a, np.int32) for a in inf_first],
                row_ptr=row_ptr, col_idx=c.astype(np.int32), val=v,
                col_ptr=col_ptr, row_idx=r2.astype(np.int32), val_csc=v2,
                payoff_kind=payoff_kind, payoff=payoff)


# --------------------------------------------------------------------------
# The benchmark configurations
# --------------------------------------------------------------------------

def cfg1() -> Game:
    """Tiny game: depth-4 binary public tree (16 terminals), 3 signals per
    player, U[-1,1] payoffs -> 144 payoff nonzeros."""
    return public_game(1, S=3, max_depth=4, branch_lo=2, branch_hi=2, p_stop=0.0,
                       payoff_kind="iid", name="cfg1-tiny", fixed_branching=True)


def _seed_select(start, lo, hi, S, max_depth, blo, bhi, p_stop, kind, name):
    seed = start
    while True:
        rng = np.random.Generator(np.random.PCG64(seed))
        tree = make_public_tree(rng, max_depth, blo, bhi, p_stop)
        if lo <= tree.n_terminals <= hi:
            break
        seed += 1
    g = public_game(seed, S=S, max_depth=max_depth, branch_lo=blo, branch_hi=bhi,
                    p_stop=p_stop, payoff_kind=kind, name=name)
    g.meta["seed_rule"] = f"first seed >= {start} with {lo} <= T <= {hi}"
    return g


def showdown_sized(S: int, max_depth: int, t_lo: int, t_hi: int, name: str,
                   start: int = 3000) -> Game:
    """The large game's generator (branching U{2,3,4}, no stop, showdown
    payoffs) at another size: S signals, the given depth, the first seed
    >= start whose tree has t_lo..t_hi terminals."""
    return _seed_select(start, t_lo, t_hi, S, max_depth, 2, 4, 0.0, "showdown", name)


def cfg2() -> Game:
    """Medium game: 13 signals, branching U{2,3}, stop 0.15 per non-root
    node, maximum depth 13 (the depth that reaches ~2e4 terminals),
    U[-1,1] payoffs, ~3.4e6 payoff nonzeros."""
    return _seed_select(2000, 18000, 22000, 13, 13, 2, 3, 0.15, "iid", "cfg2-medium")


def cfg2_literal() -> Game:
    """The medium configuration with its literal maximum depth of 8
    (a few hundred terminals)."""
    return public_game(2000, S=13, max_depth=8, branch_lo=2, branch_hi=3,
                       p_stop=0.15, payoff_kind="iid", name="cfg2-d8")


def cfg3() -> Game:
    """Large game: 32 signals, depth 10, branching U{2,3,4}, showdown payoffs
    sign(s1-s2)*pot with pot ~ U[1,8] per terminal, ~1e5 terminals,
    ~1e8 payoff nonzeros (ties are exact zeros and are not stored)."""
    return _seed_select(3000, 96000, 106000, 32, 10, 2, 4, 0.0, "showdown", "cfg3-large")


# --------------------------------------------------------------------------
# Many games of uneven size (batched solving and the request stream)
# --------------------------------------------------------------------------

def batch_specs(n: int = 256, seed: int = 4000, t_lo: float = 1e2, t_hi: float = 1e5,
                s_lo: int = 3, s_hi: int = 32, d_lo: int = 4, d_hi: int = 10) -> list:
    """Sizes of n games: signals S ~ U{s_lo..s_hi}, a target terminal count
    T log-uniform in [t_lo, t_hi], depth D ~ U{d_lo..d_hi}; every internal
    node branches to floor(T^(1/D)) or one more, the larger with probability
    T^(1/D) - floor(T^(1/D)), so the expected terminal count is T.  Game k
    takes seed `seed * 10 + k`; payoffs are U[-1,1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S = rng.integers(s_lo, s_hi + 1, size=n)
    T = np.exp(rng.uniform(np.log(t_lo), np.log(t_hi), size=n))
    D = rng.integers(d_lo, d_hi + 1, size=n)
    out = []
    for k in range(n):
        root = float(T[k]) ** (1.0 / int(D[k]))
        lo = max(1, int(np.floor(root)))
        out.append({"index": k, "seed": seed * 10 + k, "S": int(S[k]), "T_target": float(T[k]),
                    "depth": int(D[k]), "branch_lo": lo, "branch_p_hi": root - lo})
    return out


def batch_game(spec: dict) -> Game:
    g = public_game(spec["seed"], S=spec["S"], max_depth=spec["depth"],
                    branch_lo=spec["branch_lo"], branch_hi=spec["branch_lo"] + 1, p_stop=0.0,
                    payoff_kind="iid", name=f"batch-{spec['index']}",
                    branch_p_hi=spec["branch_p_hi"])
    g.meta["spec"] = dict(spec)
    return g


def batch_games(specs: list, workers: int = 16) -> list:
    """batch_game for every spec, on a pool of threads (each game draws from
    its own seed, so the games do not depend on the pool)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return list(ex.map(batch_game, specs))


def payoff_range(g: Game) -> float:
    """max - min of the terminal payoffs before chance weighting."""
    if g.payoff_kind == "showdown":
        return 2.0 * float(np.max(g.payoff))
    return float(np.max(g.payoff) - np.min(g.payoff))


def request_stream(n: int, rate: float, seed: int = 5000) -> list:
    """Poisson arrivals at `rate` per second: arrival times, game sizes from
    batch_specs' distribution, an exploitability target of 1e-2 or 1e-3 of
    the payoff range and CFR+ or DCFR, each with probability 1/2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n)
    rel = rng.choice([1e-2, 1e-3], size=n)
    var = rng.choice(["cfr+", "dcfr"], size=n)
    specs = batch_specs(n, seed=seed + 1)
    t = np.cumsum(gaps)
    return [{"arrival": float(t[k]), "spec": specs[k], "rel_target": float(rel[k]),
             "variant": str(var[k])} for k in range(n)]


CONFIGS = {"cfg1": cfg1, "cfg2": cfg2, "cfg2_d8": cfg2_literal, "cfg3": cfg3}


def make_config(name: str) -> Game:
    return CONFIGS[name]()
