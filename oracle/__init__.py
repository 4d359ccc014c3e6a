"""CPU FP64 oracle for sequence-form CFR (ctypes wrapper over cfr_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The GPU library never imports,
links or calls it.

``build()`` compiles ``cfr_oracle.c`` with gcc (no floating-point
contraction) into ``liboracle.so`` next to this file, and the same source
with ``-fopenmp`` into ``liboracle_omp.so``: the all-core build, which runs
the same per-element arithmetic on every host core and gives bit-identical
results (``Oracle(game, parallel=True)``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cfr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

VARIANTS = {"vanilla": 0, "cfr+": 1, "dcfr": 2, "pcfr+": 3, "pcfr": 4}
MODES = {"simultaneous": 0, "alternating": 1}
KINDS = {"current": 0, "average": 1}
AVG = {"default": 0, "uniform": 1, "linear": 2, "quadratic": 3, "pow_gamma": 4}


def build(force: bool = True) -> str:
    for lib, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib):
            tmp = lib + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC",
                                   "-shared", *extra, SRC, "-o", tmp, "-lm"])
            os.replace(tmp, lib)
    return LIB


_libs = {}


def _load(parallel: bool = False):
    if parallel in _libs:
        return _libs[parallel]
    path = LIB_OMP if parallel else LIB
    if not os.path.exists(path):
        build(force=False)
    lib = C.CDLL(path)
    i64, i32p, f64p, vp = C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [i64, i64, i32p, i32p, i64, i64, i32p, i32p,
                               i64, C.POINTER(C.c_int64), i32p, f64p,
                               C.c_double, C.c_double, C.c_double, C.c_int, C.c_int]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_step.argtypes = [vp, i64, C.c_int, C.c_int]
    lib.orc_step.restype = C.c_int
    for f in ("orc_strategy",):
        getattr(lib, f).argtypes = [vp, C.c_int, C.c_int, f64p]
        getattr(lib, f).restype = C.c_int
    for f in ("orc_behavioral", "orc_regrets", "orc_prediction"):
        getattr(lib, f).argtypes = [vp, C.c_int, f64p]
        getattr(lib, f).restype = C.c_int
    lib.orc_last_observation.argtypes = [vp, C.c_int, f64p, f64p]
    lib.orc_exploitability.argtypes = [vp, C.c_int, f64p]
    lib.orc_exploitability.restype = C.c_int
    lib.orc_iteration.argtypes = [vp]
    lib.orc_iteration.restype = i64
    lib.orc_total_weight.argtypes = [vp]
    lib.orc_total_weight.restype = C.c_double
    lib.orc_best_response_to.argtypes = [vp, C.c_int, f64p]
    lib.orc_best_response_to.restype = C.c_double
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = C.c_int
    _libs[parallel] = lib
    return lib


def threads(parallel: bool = True) -> int:
    """Host threads the oracle's loops run on (1 for the plain build)."""
    return int(_load(parallel).orc_threads())


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Oracle:
    """Plain FP64 sequence-form CFR on a game's arrays (caller's numbering).
    parallel: the all-core build (same arithmetic, bit-identical results)."""

    def __init__(self, game, alpha: float = 1.5, beta: float = 0.0, gamma: float = 2.0,
                 avg: str = "default", literal_pcfr: bool = False, parallel: bool = False):
        lib = _load(parallel)
        self.threads = int(lib.orc_threads())
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        par = [arr(game.inf_parent[p], np.int32) for p in range(2)]
        first = [arr(game.inf_first_seq[p], np.int32) for p in range(2)]
        rp = arr(game.row_ptr, np.int64)
        ci = arr(game.col_idx, np.int32)
        va = arr(game.val, np.float64)
        self.n_seq = [int(game.n_seq[0]), int(game.n_seq[1])]
        self.n_inf = [int(game.n_inf[0]), int(game.n_inf[1])]
        self._h = lib.orc_create(
            self.n_seq[0], self.n_inf[0], _ptr(par[0], C.c_int32), _ptr(first[0], C.c_int32),
            self.n_seq[1], self.n_inf[1], _ptr(par[1], C.c_int32), _ptr(first[1], C.c_int32),
            int(ci.shape[0]), _ptr(rp, C.c_int64), _ptr(ci, C.c_int32), _ptr(va, C.c_double),
            float(alpha), float(beta), float(gamma), AVG[avg], int(literal_pcfr))
        if not self._h:
            raise MemoryError("orc_create failed")
        self._lib = lib

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int, variant: str = "vanilla", mode: str = "simultaneous"):
        rc = self._lib.orc_step(self._h, int(n), VARIANTS[variant], MODES[mode])
        if rc != 0:
            raise ValueError(f"orc_step failed ({rc})")

    @property
    def iteration(self) -> int:
        return int(self._lib.orc_iteration(self._h))

    @property
    def total_weight(self) -> float:
        return float(self._lib.orc_total_weight(self._h))

    def strategy(self, player: int, kind: str = "current") -> np.ndarray:
        out = np.empty(self.n_seq[player])
        self._lib.orc_strategy(self._h, player, KINDS[kind], _ptr(out, C.c_double))
        return out

    def behavioral(self, player: int) -> np.ndarray:
        out = np.empty(self.n_seq[player])
        self._lib.orc_behavioral(self._h, player, _ptr(out, C.c_double))
        return out

    def regrets(self, player: int) -> np.ndarray:
        out = np.empty(self.n_seq[player])
        self._lib.orc_regrets(self._h, player, _ptr(out, C.c_double))
        return out

    def prediction(self, player: int) -> np.ndarray:
        out = np.empty(self.n_seq[player])
        self._lib.orc_prediction(self._h, player, _ptr(out, C.c_double))
        return out

    def last_observation(self, player: int):
        q = np.empty(self.n_seq[player])
        v = np.empty(max(self.n_inf[player], 1))
        self._lib.orc_last_observation(self._h, player, _ptr(q, C.c_double), _ptr(v, C.c_double))
        return q, v[: self.n_inf[player]]

    def exploitability(self, kind: str = "average") -> dict:
        out = np.empty(5)
        self._lib.orc_exploitability(self._h, KINDS[kind], _ptr(out, C.c_double))
        return {"expl": out[0], "nash_conv": out[1], "br1": out[2], "br2": out[3],
                "value": out[4]}

    def best_response_to(self, player: int, opponent: np.ndarray) -> float:
        opp = np.ascontiguousarray(opponent, dtype=np.float64)
        return float(self._lib.orc_best_response_to(self._h, player, _ptr(opp, C.c_double)))
