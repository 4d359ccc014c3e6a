"""MI355X-native sequence-form CFR: Python binding of libcfr.so.

The binding only marshals arguments: every step of an iteration runs in the
library's HIP kernels.  PyTorch supplies device memory (one workspace
tensor) and the stream.  The functions carry the names of the C ABI in
``include/cfr.h``; ``Solver`` wraps them for convenience.

Importing this package loads the compiled library and raises ImportError if
it has not been built (``python paper_2605_14277_amd/build.py``); there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcfr.so")

CFR_OK, CFR_EINVAL, CFR_ENOMEM, CFR_EDEVICE, CFR_ESTATE, CFR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_acc64": 2}
VARIANTS = {"vanilla": 0, "cfr+": 1, "dcfr": 2, "pcfr+": 3, "pcfr": 4}
MODES = {"simultaneous": 0, "alternating": 1}
KINDS = {"current": 0, "average": 1}
AVG = {"default": 0, "uniform": 1, "linear": 2, "quadratic": 3, "pow_gamma": 4}
SPMV_ORDER = {"default": 0, "sequential": 1, "parallel": 2}
ERRORS = {CFR_EINVAL: "EINVAL", CFR_ENOMEM: "ENOMEM", CFR_EDEVICE: "EDEVICE",
          CFR_ESTATE: "ESTATE", CFR_EUNSUPPORTED: "EUNSUPPORTED"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python paper_2605_14277_amd/build.py` (there is no fallback path)")


class cfr_player_desc(C.Structure):
    _fields_ = [("n_seq", C.c_int64), ("n_inf", C.c_int64),
                ("inf_parent", C.POINTER(C.c_int32)), ("inf_first_seq", C.POINTER(C.c_int32))]


class cfr_game_desc(C.Structure):
    _fields_ = [("player", cfr_player_desc * 2), ("nnz", C.c_int64),
                ("row_ptr", C.POINTER(C.c_int64)), ("col_idx", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double)),
                ("col_ptr", C.POINTER(C.c_int64)), ("row_idx", C.POINTER(C.c_int32)),
                ("val_csc", C.POINTER(C.c_double))]


class cfr_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("dcfr_alpha", C.c_double), ("dcfr_beta", C.c_double),
                ("dcfr_gamma", C.c_double), ("avg_weight", C.c_int), ("stream", C.c_void_p),
                ("device", C.c_int), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("use_graph", C.c_int), ("spmv_order", C.c_int)]


_lib = C.CDLL(LIB_PATH)
_P = C.POINTER
_lib.cfr_options_default.argtypes = [_P(cfr_options)]
_lib.cfr_validate.argtypes = [_P(cfr_game_desc)]
_lib.cfr_workspace_size.argtypes = [_P(cfr_game_desc), _P(cfr_options), _P(C.c_size_t)]
_lib.cfr_create.argtypes = [_P(cfr_game_desc), _P(cfr_options), _P(C.c_void_p)]
_lib.cfr_step.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int]
_lib.cfr_strategy.argtypes = [C.c_void_p, C.c_int, C.c_int, _P(C.c_double), C.c_int64]
_lib.cfr_regrets.argtypes = [C.c_void_p, C.c_int, _P(C.c_double), C.c_int64]
_lib.cfr_exploitability.argtypes = [C.c_void_p, C.c_int, _P(C.c_double)]
_lib.cfr_iteration.argtypes = [C.c_void_p, _P(C.c_int64)]
_lib.cfr_kernel_timing.argtypes = [C.c_void_p, C.c_int]
_lib.cfr_kernel_stats.argtypes = [C.c_void_p, C.c_int, _P(C.c_int64), _P(C.c_double),
                                  _P(C.c_double)]
_lib.cfr_destroy.argtypes = [C.c_void_p]
_lib.cfr_last_error.restype = C.c_char_p
for _f in ("cfr_options_default", "cfr_validate", "cfr_workspace_size", "cfr_create", "cfr_step",
           "cfr_strategy", "cfr_regrets", "cfr_exploitability", "cfr_iteration",
           "cfr_kernel_timing", "cfr_kernel_stats", "cfr_destroy"):
    getattr(_lib, _f).restype = C.c_int


class CfrError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.cfr_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}")


def _check(rc: int, where: str):
    if rc != CFR_OK:
        raise CfrError(rc, where)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class GameArrays:
    """Holds contiguous, correctly typed copies of a game's arrays and the
    cfr_game_desc pointing at them (keep this object alive while in use)."""

    def __init__(self, game, with_csc: bool = True):
        def arr(a, dt):
            return np.ascontiguousarray(a, dtype=dt)

        self.par = [arr(game.inf_parent[p], np.int32) for p in range(2)]
        self.first = [arr(game.inf_first_seq[p], np.int32) for p in range(2)]
        self.row_ptr = arr(game.row_ptr, np.int64)
        self.col_idx = arr(game.col_idx, np.int32)
        self.val = arr(game.val, np.float64)
        self.n_seq = [int(game.n_seq[0]), int(game.n_seq[1])]
        self.n_inf = [int(game.n_inf[0]), int(game.n_inf[1])]
        d = cfr_game_desc()
        for p in range(2):
            d.player[p].n_seq = self.n_seq[p]
            d.player[p].n_inf = self.n_inf[p]
            d.player[p].inf_parent = self.par[p].ctypes.data_as(C.POINTER(C.c_int32))
            d.player[p].inf_first_seq = self.first[p].ctypes.data_as(C.POINTER(C.c_int32))
        d.nnz = int(self.col_idx.shape[0])
        d.row_ptr = self.row_ptr.ctypes.data_as(C.POINTER(C.c_int64))
        d.col_idx = self.col_idx.ctypes.data_as(C.POINTER(C.c_int32))
        d.val = _dptr(self.val)
        if with_csc and getattr(game, "col_ptr", None) is not None:
            self.col_ptr = arr(game.col_ptr, np.int64)
            self.row_idx = arr(game.row_idx, np.int32)
            self.val_csc = arr(game.val_csc, np.float64)
            d.col_ptr = self.col_ptr.ctypes.data_as(C.POINTER(C.c_int64))
            d.row_idx = self.row_idx.ctypes.data_as(C.POINTER(C.c_int32))
            d.val_csc = _dptr(self.val_csc)
        self.desc = d


# ---- C-ABI functions under their own names ---------------------------------

def cfr_options_default() -> cfr_options:
    o = cfr_options()
    _check(_lib.cfr_options_default(C.byref(o)), "cfr_options_default")
    return o


def cfr_validate(game_arrays: GameArrays) -> int:
    """Returns the status code (0 = valid); the message is cfr_last_error()."""
    return _lib.cfr_validate(C.byref(game_arrays.desc))


def cfr_last_error() -> str:
    return _lib.cfr_last_error().decode(errors="replace")


def cfr_workspace_size(game_arrays: GameArrays, opts: cfr_options) -> int:
    n = C.c_size_t(0)
    _check(_lib.cfr_workspace_size(C.byref(game_arrays.desc), C.byref(opts), C.byref(n)),
           "cfr_workspace_size")
    return int(n.value)


def cfr_create(game_arrays: GameArrays, opts: cfr_options) -> C.c_void_p:
    h = C.c_void_p()
    _check(_lib.cfr_create(C.byref(game_arrays.desc), C.byref(opts), C.byref(h)), "cfr_create")
    return h


def cfr_step(h, n: int, variant: int, mode: int):
    _check(_lib.cfr_step(h, int(n), int(variant), int(mode)), "cfr_step")


def cfr_strategy(h, player: int, kind: int, n_seq: int) -> np.ndarray:
    out = np.empty(n_seq)
    _check(_lib.cfr_strategy(h, player, kind, _dptr(out), n_seq), "cfr_strategy")
    return out


def cfr_regrets(h, player: int, n_seq: int) -> np.ndarray:
    out = np.empty(n_seq)
    _check(_lib.cfr_regrets(h, player, _dptr(out), n_seq), "cfr_regrets")
    return out


def cfr_exploitability(h, kind: int) -> np.ndarray:
    out = np.empty(5)
    _check(_lib.cfr_exploitability(h, kind, _dptr(out)), "cfr_exploitability")
    return out


def cfr_iteration(h) -> int:
    t = C.c_int64(0)
    _check(_lib.cfr_iteration(h, C.byref(t)), "cfr_iteration")
    return int(t.value)


def cfr_kernel_timing(h, enable: bool):
    _check(_lib.cfr_kernel_timing(h, int(bool(enable))), "cfr_kernel_timing")


def cfr_kernel_stats(h, kernel: int):
    n, ms, by = C.c_int64(0), C.c_double(0), C.c_double(0)
    _check(_lib.cfr_kernel_stats(h, kernel, C.byref(n), C.byref(ms), C.byref(by)),
           "cfr_kernel_stats")
    return int(n.value), float(ms.value), float(by.value)


def cfr_destroy(h):
    _check(_lib.cfr_destroy(h), "cfr_destroy")


# ---- convenience wrapper --------------------------------------------------------

class Solver:
    """One game on one GPU.  Device memory comes from a torch uint8 tensor;
    work is enqueued on torch's current stream of that device."""

    def __init__(self, game, precision: str = "fp64", device: int = 0, alpha: float = 1.5,
                 beta: float = 0.0, gamma: float = 2.0, avg: str = "default",
                 use_graph: bool = True, stream=None, with_csc: bool = True,
                 spmv_order: str = "default"):
        import torch
        self.torch = torch
        self.arrays = GameArrays(game, with_csc=with_csc)
        self.n_seq = list(self.arrays.n_seq)
        o = cfr_options_default()
        o.precision = PRECISIONS[precision]
        o.dcfr_alpha, o.dcfr_beta, o.dcfr_gamma = float(alpha), float(beta), float(gamma)
        o.avg_weight = AVG[avg]
        o.device = int(device)
        o.use_graph = int(bool(use_graph))
        o.spmv_order = SPMV_ORDER[spmv_order]
        dev = torch.device("cuda", int(device))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        o.stream = C.c_void_p(int(stream.cuda_stream))
        nbytes = cfr_workspace_size(self.arrays, o)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        o.workspace = C.c_void_p(int(self.workspace.data_ptr()))
        o.workspace_bytes = nbytes
        self.opts = o
        self.workspace_bytes = nbytes
        self.h = cfr_create(self.arrays, o)

    def step(self, n: int, variant: str = "vanilla", mode: str = "simultaneous"):
        cfr_step(self.h, n, VARIANTS[variant], MODES[mode])

    def strategy(self, player: int, kind: str = "current") -> np.ndarray:
        return cfr_strategy(self.h, player, KINDS[kind], self.n_seq[player])

    def regrets(self, player: int) -> np.ndarray:
        return cfr_regrets(self.h, player, self.n_seq[player])

    def exploitability(self, kind: str = "average") -> dict:
        out = cfr_exploitability(self.h, KINDS[kind])
        return {"expl": out[0], "nash_conv": out[1], "br1": out[2], "br2": out[3],
                "value": out[4]}

    @property
    def iteration(self) -> int:
        return cfr_iteration(self.h)

    def kernel_timing(self, enable: bool):
        cfr_kernel_timing(self.h, enable)

    def kernel_stats(self, kernel: int):
        return cfr_kernel_stats(self.h, kernel)

    def close(self):
        if getattr(self, "h", None):
            cfr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
