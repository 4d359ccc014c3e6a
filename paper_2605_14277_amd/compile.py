"""Front end: a two-player zero-sum extensive-form game -> sequence-form arrays.

The paper's implementation takes its games through a game-state interface
(the OpenSpiel-compatible entry point of Sections 2.2 and 5).  This module
walks any object with that kind of state interface and emits what ``cfr_create`` and
``cfr_batch_add`` take: each player's treeplex (decision points with their
parent sequences and contiguous action ranges) and the payoff matrix A of
player 1 with chance folded in (Section 2.1: u1 = A y, u2 = -A^T x), as CSR
and CSC.

State interface (methods of the root state and of every state it reaches):

* ``is_terminal()`` -> bool; ``utility()`` -> player 1's payoff (terminal);
* ``is_chance()`` -> bool; ``chance_outcomes()`` -> [(outcome, probability)]
  with probabilities summing to 1 (chance nodes);
* ``current_player()`` -> 0 or 1; ``information_state()`` -> a hashable key
  of the acting player's information; ``legal_actions()`` -> a list of
  actions, the same list at every state of one information state;
* ``child(action_or_outcome)`` -> the next state.

Sequence form needs perfect recall: every state of one information state
must follow the same sequence of the acting player's own earlier
(information state, action) pairs; a violation raises ``ValueError``.

Numbering: decision points in order of first visit (depth first, children
in the listed order), each one's sequences consecutive, so every parent
sequence precedes its decision point's sequences.  Payoff entries reached
through several chance or opponent paths are summed; exact zeros are not
stored.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CompiledGame:
    """Arrays in the layout of ``cfr_game_desc`` (see include/cfr.h)."""
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
    infosets: list = field(default_factory=list)  # per player: information-state keys by index
    actions: list = field(default_factory=list)   # per player: action list of each decision point
    name: str = "compiled"

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def sequence(self, player: int, infoset, action) -> int:
        """Index of the sequence ending with `action` at `infoset`."""
        j = self.infosets[player].index(infoset)
        return int(self.inf_first_seq[player][j]) + list(self.actions[player][j]).index(action)


class _Plex:
    def __init__(self):
        self.key_index = {}    # information-state key -> decision point
        self.parent = []       # parent sequence of each decision point
        self.first = []        # first sequence of each decision point
        self.actions = []      # actions of each decision point
        self.keys = []
        self.n_seq = 1         # the empty sequence

    def visit(self, key, parent_seq: int, actions) -> int:
        j = self.key_index.get(key)
        acts = list(actions)
        if j is None:
            if not acts:
                raise ValueError(f"information state {key!r} has no legal action")
            j = len(self.parent)
            self.key_index[key] = j
            self.parent.append(parent_seq)
            self.first.append(self.n_seq)
            self.actions.append(acts)
            self.keys.append(key)
            self.n_seq += len(acts)
            return j
        if self.parent[j] != parent_seq:
            raise ValueError(f"information state {key!r} is reached after different own "
                             "earlier decisions (imperfect recall)")
        if self.actions[j] != acts:
            raise ValueError(f"information state {key!r} lists different actions at two states")
        return j


def compile_game(root, name: str = "compiled", prob_tol: float = 1e-12) -> CompiledGame:
    """Walks the game from `root` and returns its sequence-form arrays."""
    plex = [_Plex(), _Plex()]
    entries = {}
    # explicit stack: (state, own sequence of player 1, of player 2, chance reach)
    stack = [(root, 0, 0, 1.0)]
    while stack:
        state, s1, s2, reach = stack.pop()
        if state.is_terminal():
            u = float(state.utility())
            if not math.isfinite(u):
                raise ValueError("non-finite utility")
            entries[(s1, s2)] = entries.get((s1, s2), 0.0) + reach * u
            continue
        if state.is_chance():
            outs = list(state.chance_outcomes())
            total = sum(p for _, p in outs)
            if abs(total - 1.0) > prob_tol or any(p < 0 for _, p in outs):
                raise ValueError(f"chance probabilities sum to {total}, not 1")
            for o, p in reversed(outs):
                if p > 0:
                    stack.append((state.child(o), s1, s2, reach * p))
            continue
        pl = state.current_player()
        if pl not in (0, 1):
            raise ValueError(f"player {pl!r} is not 0 or 1")
        own = s1 if pl == 0 else s2
        acts = state.legal_actions()
        j = plex[pl].visit(state.information_state(), own, acts)
        first = plex[pl].first[j]
        kids = []
        for k, a in enumerate(plex[pl].actions[j]):
            seq = first + k
            kids.append((state.child(a), seq if pl == 0 else s1, seq if pl == 1 else s2, reach))
        stack.extend(reversed(kids))
    n_seq = [plex[0].n_seq, plex[1].n_seq]
    keys = sorted(k for k, v in entries.items() if v != 0.0)
    rows = np.array([k[0] for k in keys], dtype=np.int64)
    cols = np.array([k[1] for k in keys], dtype=np.int64)
    vals = np.array([entries[k] for k in keys], dtype=np.float64)
    row_ptr = np.zeros(n_seq[0] + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    o = np.lexsort((rows, cols))
    col_ptr = np.zeros(n_seq[1] + 1, np.int64)
    np.add.at(col_ptr, cols[o] + 1, 1)
    col_ptr = np.cumsum(col_ptr)
    inf_parent, inf_first = [], []
    for p in range(2):
        inf_parent.append(np.asarray(plex[p].parent, np.int32))
        inf_first.append(np.asarray(plex[p].first + [plex[p].n_seq], np.int32))
    return CompiledGame(n_seq=n_seq, n_inf=[len(plex[0].parent), len(plex[1].parent)],
                        inf_parent=inf_parent, inf_first_seq=inf_first, row_ptr=row_ptr,
                        col_idx=cols.astype(np.int32), val=vals, col_ptr=col_ptr,
                        row_idx=rows[o].astype(np.int32), val_csc=vals[o],
                        infosets=[plex[0].keys, plex[1].keys],
                        actions=[plex[0].actions, plex[1].actions], name=name)
