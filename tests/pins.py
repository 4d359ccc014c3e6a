"""Independent checks the oracle is pinned against (test-side only).

* ``TreeWalkCFR``: classical CFR (Zinkevich et al.) by recursion over the
  public game tree and every chance outcome, with reach probabilities.  The
  paper states that classical and sequence-form CFR produce identical
  iterates (Section 2.1 and Section 5), so its iterates must equal the
  oracle's, which works on the sequence-form arrays instead.
* ``public_best_response``: a best response computed over the public tree
  and signals (not over the treeplex arrays).
* ``brute_force_best_response``: enumeration of pure strategies.
* ``lp_game_value``: the sequence-form linear program of Koller, Megiddo and
  von Stengel solved with HiGHS.
* ``minimax_value``: backward induction for perfect-information games.
"""
from __future__ import annotations

import itertools

import numpy as np


def _seq_lookup(game, p):
    """(node, signal, action) -> sequence index for player p."""
    table = {}
    sn, ss, sa = game.seq_node[p], game.seq_signal[p], game.seq_action[p]
    for i in range(1, game.n_seq[p]):
        table[(int(sn[i]), int(ss[i]), int(sa[i]))] = i
    return table


class TreeWalkCFR:
    """Classical tabular CFR on a public-tree game with private signals."""

    def __init__(self, game, variant="vanilla", mode="simultaneous", alpha=1.5,
                 beta=0.0, gamma=2.0, avg="default", inst_weight=None):
        self.g = game
        self.tree = game.tree
        self.S = game.S
        self.variant = variant
        self.mode = mode
        self.alpha, self.beta, self.gamma = alpha, beta, gamma
        self.avg = avg
        self.inst_weight = inst_weight   # optional f(t) scaling each instantaneous regret
        t = self.tree
        nb = int(t.n_child.max())
        self.nb = nb
        n = t.n_nodes
        # regrets / predictions / strategies per (node, signal, action)
        self.R = [np.zeros((n, self.S[p], nb)) for p in range(2)]
        self.M = [np.zeros((n, self.S[p], nb)) for p in range(2)]
        self.sigma = [self._rm(p) for p in range(2)]
        self.avg_seq = [np.zeros(game.n_seq[p]) for p in range(2)]
        self.W = 0.0
        self.t = 0
        self.lookup = [_seq_lookup(game, p) for p in range(2)]
        self.chance = 1.0 / (self.S[0] * self.S[1])

    # -- regret matching per information set ------------------------------
    def _rm(self, p):
        t = self.tree
        out = np.zeros_like(self.R[p])
        for node in range(t.n_nodes):
            k = int(t.n_child[node])
            if k == 0 or (int(t.depth[node]) & 1) != p:
                continue
            for s in range(self.S[p]):
                z = np.maximum(self.R[p][node, s, :k] + self.M[p][node, s, :k], 0.0)
                tot = z.sum()
                out[node, s, :k] = z / tot if tot > 0 else 1.0 / k
        return out

    # -- one traversal for one chance outcome -----------------------------
    def _walk(self, node, s1, s2, reach1, reach2, inst, updating):
        t = self.tree
        k = int(t.n_child[node])
        if k == 0:
            return float(self.g.utility(np.array(int(t.term_id[node])), np.array(s1),
                                        np.array(s2)))
        p = int(t.depth[node]) & 1
        s = s1 if p == 0 else s2
        strat = self.sigma[p][node, s, :k]
        c0 = int(t.child_first[node])
        vals = np.empty(k)
        for a in range(k):
            if p == 0:
                vals[a] = self._walk(c0 + a, s1, s2, reach1 * strat[a], reach2, inst, updating)
            else:
                vals[a] = self._walk(c0 + a, s1, s2, reach1, reach2 * strat[a], inst, updating)
        v = float(np.dot(strat, vals))
        if p in updating:
            cf = self.chance * (reach2 if p == 0 else reach1)
            sign = 1.0 if p == 0 else -1.0
            inst[p][node, s, :k] += cf * sign * (vals - v)
        return v

    def _instantaneous(self, updating):
        inst = [np.zeros_like(self.R[0]), np.zeros_like(self.R[1])]
        for s1 in range(self.S[0]):
            for s2 in range(self.S[1]):
                self._walk(0, s1, s2, 1.0, 1.0, inst, updating)
        return inst

    def _weight(self, t):
        kind = self.avg
        if kind == "default":
            kind = {"cfr+": "linear", "dcfr": "pow_gamma", "pcfr+": "quadratic"}.get(
                self.variant, "uniform")
        return {"uniform": 1.0, "linear": float(t), "quadratic": float(t) * t,
                "pow_gamma": float(t) ** self.gamma}[kind]

    def _apply(self, p, inst):
        t = self.t
        I = inst[p]
        if self.inst_weight is not None:
            I = I * self.inst_weight(t)
        R = self.R[p] + I
        if self.variant in ("cfr+", "pcfr+"):
            R = np.maximum(R, 0.0)
        elif self.variant == "dcfr":
            ta, tb = float(t) ** self.alpha, float(t) ** self.beta
            R = np.where(R > 0, R * (ta / (ta + 1)), np.where(R < 0, R * (tb / (tb + 1)), R))
        if self.variant in ("pcfr+", "pcfr"):
            self.M[p] = I.copy()
        self.R[p] = R

    def seq_strategy(self, p, sigma=None):
        """Sequence-form strategy of player p from behavioural strategies,
        by walking the public tree (own reach)."""
        sigma = self.sigma[p] if sigma is None else sigma
        t = self.tree
        x = np.zeros(self.g.n_seq[p])
        x[0] = 1.0
        own_reach = np.ones((t.n_nodes, self.S[p]))
        order = np.argsort(t.depth, kind="stable")
        for node in order:
            k = int(t.n_child[node])
            if k == 0:
                continue
            c0 = int(t.child_first[node])
            mine = (int(t.depth[node]) & 1) == p
            for s in range(self.S[p]):
                for a in range(k):
                    if mine:
                        pr = own_reach[node, s] * sigma[node, s, a]
                        x[self.lookup[p][(int(node), s, a)]] = pr
                    else:
                        pr = own_reach[node, s]
                    own_reach[c0 + a, s] = pr
        return x

    def step(self, n=1):
        for _ in range(n):
            self.t += 1
            w = self._weight(self.t)
            if self.mode == "simultaneous":
                inst = self._instantaneous({0, 1})
                x_played = [self.seq_strategy(0), self.seq_strategy(1)]
                self._apply(0, inst)
                self._apply(1, inst)
                self.sigma = [self._rm(0), self._rm(1)]
                for p in range(2):
                    self.avg_seq[p] += w * x_played[p]
            else:
                x1 = self.seq_strategy(0)
                inst = self._instantaneous({0})
                self._apply(0, inst)
                self.sigma[0] = self._rm(0)
                self.avg_seq[0] += w * x1
                y = self.seq_strategy(1)
                inst = self._instantaneous({1})
                self._apply(1, inst)
                self.sigma[1] = self._rm(1)
                self.avg_seq[1] += w * y
            self.W += w

    def regrets_seq(self, p):
        r = np.zeros(self.g.n_seq[p])
        for (node, s, a), i in self.lookup[p].items():
            r[i] = self.R[p][node, s, a]
        return r

    def average_seq(self, p):
        return self.avg_seq[p] / self.W if self.W > 0 else self.seq_strategy(p)


# ---------------------------------------------------------------------------
# Best responses
# ---------------------------------------------------------------------------

def public_best_response(game, player, opp_seq):
    """Best-response value of ``player`` against the opponent's sequence-form
    strategy, by a bottom-up pass over the public tree for every own signal.
    Player 0 maximises u, player 1 maximises -u."""
    t = game.tree
    opp = 1 - player
    lookup_opp = _seq_lookup(game, opp)
    S_me, S_op = game.S[player], game.S[opp]
    chance = 1.0 / (game.S[0] * game.S[1])
    sign = 1.0 if player == 0 else -1.0

    def opp_reach(node, s_op):
        # sequence-form probability of the opponent's last sequence on the path
        cur = node
        while t.parent[cur] >= 0:
            par = int(t.parent[cur])
            if (int(t.depth[par]) & 1) == opp:
                return opp_seq[lookup_opp[(par, s_op, int(t.action[cur]))]]
            cur = par
        return opp_seq[0]

    order = np.argsort(-t.depth, kind="stable")
    cv = np.zeros((t.n_nodes, S_me))
    for node in order:
        k = int(t.n_child[node])
        if k == 0:
            z = int(t.term_id[node])
            for s in range(S_me):
                acc = 0.0
                for so in range(S_op):
                    s1, s2 = (s, so) if player == 0 else (so, s)
                    u = float(game.utility(np.array(z), np.array(s1), np.array(s2)))
                    acc += chance * opp_reach(node, so) * sign * u
                cv[node, s] = acc
            continue
        c0 = int(t.child_first[node])
        kids = cv[c0:c0 + k]
        if (int(t.depth[node]) & 1) == player:
            cv[node] = kids.max(axis=0)
        else:
            cv[node] = kids.sum(axis=0)
    return float(cv[0].sum())


def brute_force_best_response(game, player, opp_seq):
    """max over the player's pure sequence-form strategies of its payoff
    (player 0: x^T A y_opp, player 1: -(x_opp^T A y))."""
    import scipy.sparse as sp
    A = sp.csr_matrix((game.val, game.col_idx, game.row_ptr),
                      shape=(game.n_seq[0], game.n_seq[1]))
    g = A @ opp_seq if player == 0 else -(A.T @ opp_seq)
    par = game.inf_parent[player]
    first = game.inf_first_seq[player]
    n_inf = game.n_inf[player]
    choices = [range(first[j + 1] - first[j]) for j in range(n_inf)]
    best = -np.inf
    for pick in itertools.product(*choices):
        x = np.zeros(game.n_seq[player])
        x[0] = 1.0
        for j in range(n_inf):
            x[first[j] + pick[j]] = x[par[j]]
        best = max(best, float(x @ g))
    return best


# ---------------------------------------------------------------------------
# Linear programs
# ---------------------------------------------------------------------------

def _constraints(game, p):
    n = game.n_seq[p]
    par = game.inf_parent[p]
    first = game.inf_first_seq[p]
    F = np.zeros((game.n_inf[p] + 1, n))
    f = np.zeros(game.n_inf[p] + 1)
    F[0, 0] = 1.0
    f[0] = 1.0
    for j in range(game.n_inf[p]):
        F[j + 1, first[j]:first[j + 1]] = 1.0
        F[j + 1, par[j]] = -1.0
    return F, f


def lp_game_value(game):
    """Game value max_x min_y x^T A y over the two sequence-form polytopes:
    max f2^T v  s.t.  F1 x = f1, x >= 0, F2^T v <= A^T x."""
    from scipy.optimize import linprog
    import scipy.sparse as sp
    A = sp.csr_matrix((game.val, game.col_idx, game.row_ptr),
                      shape=(game.n_seq[0], game.n_seq[1])).toarray()
    F1, f1 = _constraints(game, 0)
    F2, f2 = _constraints(game, 1)
    n1, m2 = game.n_seq[0], F2.shape[0]
    c = np.concatenate([np.zeros(n1), -f2])
    A_ub = np.hstack([-A.T, F2.T])
    b_ub = np.zeros(game.n_seq[1])
    A_eq = np.hstack([F1, np.zeros((F1.shape[0], m2))])
    bounds = [(0, None)] * n1 + [(None, None)] * m2
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=f1, bounds=bounds,
                  method="highs")
    assert res.status == 0, res.message
    return -res.fun, res.x[:n1]


def lp_best_response(game, player, opp_seq):
    """max over the player's sequence-form polytope of its payoff, by LP."""
    from scipy.optimize import linprog
    import scipy.sparse as sp
    A = sp.csr_matrix((game.val, game.col_idx, game.row_ptr),
                      shape=(game.n_seq[0], game.n_seq[1]))
    g = A @ opp_seq if player == 0 else -(A.T @ opp_seq)
    F, f = _constraints(game, player)
    res = linprog(-np.asarray(g), A_eq=F, b_eq=f,
                  bounds=[(0, None)] * game.n_seq[player], method="highs")
    assert res.status == 0, res.message
    return -res.fun


def minimax_value(game):
    """Backward induction on a perfect-information game (one signal each)."""
    t = game.tree
    assert game.S == (1, 1)
    order = np.argsort(-t.depth, kind="stable")
    val = np.zeros(t.n_nodes)
    for node in order:
        k = int(t.n_child[node])
        if k == 0:
            val[node] = float(game.utility(np.array(int(t.term_id[node])), np.array(0),
                                           np.array(0)))
            continue
        c0 = int(t.child_first[node])
        kids = val[c0:c0 + k]
        val[node] = kids.max() if (int(t.depth[node]) & 1) == 0 else kids.min()
    return float(val[0])
