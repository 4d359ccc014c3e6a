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
# CFR_LIBRARY names another build of the same library (the address-sanitised
# host build the CPU tests load); by default the in-tree libcfr.so.
LIB_PATH = os.environ.get("CFR_LIBRARY") or os.path.join(_HERE, "libcfr.so")

CFR_OK, CFR_EINVAL, CFR_ENOMEM, CFR_EDEVICE, CFR_ESTATE, CFR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_acc64": 2}
VARIANTS = {"vanilla": 0, "cfr+": 1, "dcfr": 2, "pcfr+": 3, "pcfr": 4}
MODES = {"simultaneous": 0, "alternating": 1}
KINDS = {"current": 0, "average": 1}
AVG = {"default": 0, "uniform": 1, "linear": 2, "quadratic": 3, "pow_gamma": 4}
SPMV_ORDER = {"default": 0, "sequential": 1, "parallel": 2}
DOWN_PASS = {"default": 0, "levels": 1}
UP_PASS = {"default": 0, "levels": 1, "pairs": 2}
GAME_STATES = {0: "active", 1: "waiting", 2: "done"}
ERRORS = {CFR_EINVAL: "EINVAL", CFR_ENOMEM: "ENOMEM", CFR_EDEVICE: "EDEVICE",
          CFR_ESTATE: "ESTATE", CFR_EUNSUPPORTED: "EUNSUPPORTED"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python paper_2605_14277_amd/build.py` (there is no fallback path)")

# torch brings its own HIP runtime.  Loaded first, it also serves the
# library's libamdhip64 dependency, so the process has one runtime; if the
# library were loaded first, it would bind the system runtime, torch would
# then start a second one, and the library would find no device.
import torch  # noqa: E402,F401


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
                ("use_graph", C.c_int), ("spmv_order", C.c_int), ("down_pass", C.c_int), ("up_pass", C.c_int)]


class cfr_spmv_tiling(C.Structure):
    _fields_ = [("items", C.c_int * 2), ("rows", C.c_int * 2), ("vec", C.c_int * 2),
                ("perm", C.c_int * 2), ("xcd", C.c_int * 2)]


class cfr_batch_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("mode", C.c_int), ("spmv_order", C.c_int),
                ("max_games", C.c_int64), ("seq_capacity", C.c_int64 * 2),
                ("inf_capacity", C.c_int64 * 2), ("nnz_capacity", C.c_int64),
                ("check_every", C.c_int64), ("stream", C.c_void_p), ("device", C.c_int),
                ("use_graph", C.c_int), ("down_pass", C.c_int), ("async_admission", C.c_int),
                ("quad_capacity", C.c_int64)]


class cfr_game_params(C.Structure):
    _fields_ = [("variant", C.c_int), ("avg_weight", C.c_int), ("dcfr_alpha", C.c_double),
                ("dcfr_beta", C.c_double), ("dcfr_gamma", C.c_double),
                ("target_exploitability", C.c_double), ("max_iterations", C.c_int64)]


class cfr_game_status(C.Structure):
    _fields_ = [("state", C.c_int), ("reached_target", C.c_int), ("iterations", C.c_int64),
                ("evaluated_at", C.c_int64), ("exploitability", C.c_double)]


_lib = C.CDLL(LIB_PATH)
_P = C.POINTER
_lib.cfr_options_default.argtypes = [_P(cfr_options)]
_lib.cfr_validate.argtypes = [_P(cfr_game_desc)]
_lib.cfr_workspace_size.argtypes = [_P(cfr_game_desc), _P(cfr_options), _P(C.c_size_t)]
_lib.cfr_create.argtypes = [_P(cfr_game_desc), _P(cfr_options), _P(C.c_void_p)]
_lib.cfr_create_static.argtypes = [_P(cfr_game_desc), _P(cfr_options), _P(C.c_void_p)]
_lib.cfr_step.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int]
_lib.cfr_strategy.argtypes = [C.c_void_p, C.c_int, C.c_int, _P(C.c_double), C.c_int64]
_lib.cfr_regrets.argtypes = [C.c_void_p, C.c_int, _P(C.c_double), C.c_int64]
_lib.cfr_exploitability.argtypes = [C.c_void_p, C.c_int, _P(C.c_double), C.c_int64]
_lib.cfr_iteration.argtypes = [C.c_void_p, _P(C.c_int64)]
_lib.cfr_kernel_timing.argtypes = [C.c_void_p, C.c_int]
_lib.cfr_kernel_stats.argtypes = [C.c_void_p, C.c_int, _P(C.c_int64), _P(C.c_double),
                                  _P(C.c_double)]
_lib.cfr_state_size.argtypes = [C.c_void_p, _P(C.c_size_t)]
_lib.cfr_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
_lib.cfr_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
_lib.cfr_get_tiling.argtypes = [C.c_void_p, _P(cfr_spmv_tiling)]
_lib.cfr_set_tiling.argtypes = [C.c_void_p, _P(cfr_spmv_tiling)]
_lib.cfr_tune.argtypes = [C.c_void_p, C.c_int, _P(cfr_spmv_tiling)]
_lib.cfr_destroy.argtypes = [C.c_void_p]
_lib.cfr_last_error.restype = C.c_char_p
_lib.cfr_batch_options_default.argtypes = [_P(cfr_batch_options)]
_lib.cfr_game_params_default.argtypes = [_P(cfr_game_params)]
_lib.cfr_batch_game_size.argtypes = [_P(cfr_game_desc), _P(C.c_int64)]
_lib.cfr_batch_workspace_size.argtypes = [_P(cfr_batch_options), _P(C.c_size_t)]
_lib.cfr_batch_index_limits.argtypes = [_P(cfr_batch_options), _P(C.c_int)]
_lib.cfr_batch_create.argtypes = [_P(cfr_batch_options), _P(C.c_void_p)]
_lib.cfr_batch_add.argtypes = [C.c_void_p, _P(cfr_game_desc), _P(cfr_game_params), _P(C.c_int64)]
_lib.cfr_batch_run.argtypes = [C.c_void_p, C.c_int64, _P(C.c_int64)]
_lib.cfr_batch_run_begin.argtypes = [C.c_void_p]
_lib.cfr_batch_run_end.argtypes = [C.c_void_p, _P(C.c_int64)]
_lib.cfr_batch_run_ready.argtypes = [C.c_void_p, _P(C.c_int)]
_lib.cfr_batch_status.argtypes = [C.c_void_p, C.c_int64, _P(cfr_game_status)]
_lib.cfr_batch_strategy.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, _P(C.c_double),
                                    C.c_int64]
_lib.cfr_batch_exploitability.argtypes = [C.c_void_p, C.c_int64, C.c_int, _P(C.c_double),
                                            C.c_int64]
_lib.cfr_batch_remove.argtypes = [C.c_void_p, C.c_int64]
_lib.cfr_batch_get_tiling.argtypes = [C.c_void_p, _P(cfr_spmv_tiling)]
_lib.cfr_batch_set_tiling.argtypes = [C.c_void_p, _P(cfr_spmv_tiling)]
_lib.cfr_batch_tune.argtypes = [C.c_void_p, C.c_int, _P(cfr_spmv_tiling)]
_lib.cfr_batch_kernel_timing.argtypes = [C.c_void_p, C.c_int]
_lib.cfr_batch_kernel_stats.argtypes = [C.c_void_p, C.c_int, _P(C.c_int64), _P(C.c_double),
                                        _P(C.c_double)]
_lib.cfr_batch_destroy.argtypes = [C.c_void_p]
_lib.cfr_prepare.argtypes = [_P(cfr_game_desc), C.c_int, _P(C.c_void_p)]
_lib.cfr_batch_host_stats.argtypes = [C.c_void_p, _P(C.c_double)]
_lib.cfr_prepared_size.argtypes = [C.c_void_p, _P(C.c_int64)]
_lib.cfr_prepare_quads.argtypes = [C.c_void_p, _P(C.c_int)]
_lib.cfr_batch_add_prepared.argtypes = [C.c_void_p, C.c_void_p, _P(cfr_game_params),
                                        _P(C.c_int64)]
_lib.cfr_prepared_destroy.argtypes = [C.c_void_p]
for _f in ("cfr_options_default", "cfr_validate", "cfr_workspace_size", "cfr_create",
           "cfr_create_static", "cfr_step",
           "cfr_strategy", "cfr_regrets", "cfr_exploitability", "cfr_iteration",
           "cfr_kernel_timing", "cfr_kernel_stats", "cfr_get_tiling", "cfr_set_tiling",
           "cfr_state_size", "cfr_get_state", "cfr_set_state",
           "cfr_tune", "cfr_destroy", "cfr_batch_options_default", "cfr_game_params_default",
           "cfr_batch_game_size", "cfr_batch_workspace_size", "cfr_batch_create",
           "cfr_batch_add", "cfr_batch_run", "cfr_batch_run_begin", "cfr_batch_run_end",
           "cfr_batch_run_ready",
           "cfr_batch_status", "cfr_batch_strategy",
           "cfr_batch_exploitability", "cfr_batch_remove", "cfr_batch_get_tiling",
           "cfr_batch_set_tiling", "cfr_batch_tune", "cfr_batch_kernel_timing",
           "cfr_batch_kernel_stats", "cfr_batch_destroy", "cfr_prepare", "cfr_prepared_size",
           "cfr_batch_add_prepared", "cfr_prepared_destroy", "cfr_batch_host_stats",
           "cfr_prepare_quads", "cfr_batch_index_limits"):
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


def cfr_create_static(game_arrays: GameArrays, opts: cfr_options) -> C.c_void_p:
    h = C.c_void_p()
    _check(_lib.cfr_create_static(C.byref(game_arrays.desc), C.byref(opts), C.byref(h)),
           "cfr_create_static")
    return h


# bytes of the library's static per-device workspace (cfr_create_static)
STATIC_WORKSPACE_BYTES = 64 << 20


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
    _check(_lib.cfr_exploitability(h, kind, _dptr(out), 5), "cfr_exploitability")
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


def cfr_get_state(h) -> bytes:
    n = C.c_size_t(0)
    _check(_lib.cfr_state_size(h, C.byref(n)), "cfr_state_size")
    buf = C.create_string_buffer(int(n.value))
    _check(_lib.cfr_get_state(h, buf, n), "cfr_get_state")
    return buf.raw


def cfr_set_state(h, state: bytes):
    buf = C.create_string_buffer(state, len(state))
    _check(_lib.cfr_set_state(h, buf, len(state)), "cfr_set_state")


def _tiling_dict(t: cfr_spmv_tiling) -> dict:
    return {"items": [int(t.items[0]), int(t.items[1])], "rows": [int(t.rows[0]), int(t.rows[1])],
            "vec": [int(t.vec[0]), int(t.vec[1])], "perm": [int(t.perm[0]), int(t.perm[1])],
            "xcd": [int(t.xcd[0]), int(t.xcd[1])]}


def _tiling_struct(d: dict) -> cfr_spmv_tiling:
    t = cfr_spmv_tiling()
    for w in range(2):
        t.items[w] = int(d["items"][w])
        t.rows[w] = int(d["rows"][w])
        t.vec[w] = int(d.get("vec", [1, 1])[w])
        t.perm[w] = int(d.get("perm", [0, 0])[w])
        t.xcd[w] = int(d.get("xcd", [1, 1])[w])
    return t


def cfr_get_tiling(h) -> dict:
    t = cfr_spmv_tiling()
    _check(_lib.cfr_get_tiling(h, C.byref(t)), "cfr_get_tiling")
    return _tiling_dict(t)


def cfr_set_tiling(h, tiling: dict):
    t = _tiling_struct(tiling)
    _check(_lib.cfr_set_tiling(h, C.byref(t)), "cfr_set_tiling")


def cfr_tune(h, reps: int = 10) -> dict:
    t = cfr_spmv_tiling()
    _check(_lib.cfr_tune(h, int(reps), C.byref(t)), "cfr_tune")
    return _tiling_dict(t)


def cfr_destroy(h):
    _check(_lib.cfr_destroy(h), "cfr_destroy")


def cfr_batch_options_default() -> cfr_batch_options:
    o = cfr_batch_options()
    _check(_lib.cfr_batch_options_default(C.byref(o)), "cfr_batch_options_default")
    return o


def cfr_game_params_default() -> cfr_game_params:
    g = cfr_game_params()
    _check(_lib.cfr_game_params_default(C.byref(g)), "cfr_game_params_default")
    return g


def cfr_batch_game_size(game_arrays: GameArrays) -> np.ndarray:
    out = np.zeros(5, dtype=np.int64)
    _check(_lib.cfr_batch_game_size(C.byref(game_arrays.desc),
                                    out.ctypes.data_as(C.POINTER(C.c_int64))),
           "cfr_batch_game_size")
    return out


def cfr_batch_workspace_size(opts: cfr_batch_options) -> int:
    n = C.c_size_t(0)
    _check(_lib.cfr_batch_workspace_size(C.byref(opts), C.byref(n)), "cfr_batch_workspace_size")
    return int(n.value)


def cfr_batch_index_limits(opts: cfr_batch_options) -> dict:
    out = (C.c_int * 4)()
    _check(_lib.cfr_batch_index_limits(C.byref(opts), out), "cfr_batch_index_limits")
    return {"slots": [bool(out[0]), bool(out[1])], "quads": [bool(out[2]), bool(out[3])]}


def cfr_batch_create(opts: cfr_batch_options) -> C.c_void_p:
    h = C.c_void_p()
    _check(_lib.cfr_batch_create(C.byref(opts), C.byref(h)), "cfr_batch_create")
    return h


def cfr_batch_add(h, game_arrays: GameArrays, params: cfr_game_params) -> int:
    """Returns the game's id, or raises CfrError (code CFR_ENOMEM when the
    game does not fit the free capacity)."""
    i = C.c_int64(-1)
    _check(_lib.cfr_batch_add(h, C.byref(game_arrays.desc), C.byref(params), C.byref(i)),
           "cfr_batch_add")
    return int(i.value)


def cfr_batch_run(h, n: int) -> int:
    k = C.c_int64(0)
    _check(_lib.cfr_batch_run(h, int(n), C.byref(k)), "cfr_batch_run")
    return int(k.value)


def cfr_batch_run_begin(h):
    _check(_lib.cfr_batch_run_begin(h), "cfr_batch_run_begin")


def cfr_batch_run_ready(h) -> bool:
    r = C.c_int(0)
    _check(_lib.cfr_batch_run_ready(h, C.byref(r)), "cfr_batch_run_ready")
    return bool(r.value)


def cfr_batch_run_end(h) -> int:
    k = C.c_int64(0)
    _check(_lib.cfr_batch_run_end(h, C.byref(k)), "cfr_batch_run_end")
    return int(k.value)


def cfr_batch_status(h, gid: int) -> dict:
    s = cfr_game_status()
    _check(_lib.cfr_batch_status(h, int(gid), C.byref(s)), "cfr_batch_status")
    return {"state": GAME_STATES[int(s.state)], "reached_target": bool(s.reached_target),
            "iterations": int(s.iterations), "evaluated_at": int(s.evaluated_at),
            "expl": float(s.exploitability)}


def cfr_batch_strategy(h, gid: int, player: int, kind: int, n_seq: int) -> np.ndarray:
    out = np.empty(n_seq)
    _check(_lib.cfr_batch_strategy(h, int(gid), player, kind, _dptr(out), n_seq),
           "cfr_batch_strategy")
    return out


def cfr_batch_exploitability(h, gid: int, kind: int) -> np.ndarray:
    out = np.empty(5)
    _check(_lib.cfr_batch_exploitability(h, int(gid), kind, _dptr(out), 5),
           "cfr_batch_exploitability")
    return out


def cfr_batch_remove(h, gid: int):
    _check(_lib.cfr_batch_remove(h, int(gid)), "cfr_batch_remove")


def cfr_batch_get_tiling(h) -> dict:
    t = cfr_spmv_tiling()
    _check(_lib.cfr_batch_get_tiling(h, C.byref(t)), "cfr_batch_get_tiling")
    return _tiling_dict(t)


def cfr_batch_set_tiling(h, tiling: dict):
    t = _tiling_struct(tiling)
    _check(_lib.cfr_batch_set_tiling(h, C.byref(t)), "cfr_batch_set_tiling")


def cfr_batch_tune(h, reps: int = 10) -> dict:
    t = cfr_spmv_tiling()
    _check(_lib.cfr_batch_tune(h, int(reps), C.byref(t)), "cfr_batch_tune")
    return _tiling_dict(t)


def cfr_batch_kernel_timing(h, enable: bool):
    _check(_lib.cfr_batch_kernel_timing(h, int(bool(enable))), "cfr_batch_kernel_timing")


def cfr_batch_kernel_stats(h, kernel: int):
    n, ms, by = C.c_int64(0), C.c_double(0), C.c_double(0)
    _check(_lib.cfr_batch_kernel_stats(h, kernel, C.byref(n), C.byref(ms), C.byref(by)),
           "cfr_batch_kernel_stats")
    return int(n.value), float(ms.value), float(by.value)


HOST_STATS = ("tables", "graph", "evaluate", "enqueue", "add", "remove", "quads")


def cfr_batch_host_stats(h) -> dict:
    n = len(HOST_STATS)
    out = np.zeros(2 * n)
    _check(_lib.cfr_batch_host_stats(h, _dptr(out)), "cfr_batch_host_stats")
    return {k: {"seconds": float(out[i]), "calls": int(out[n + i])}
            for i, k in enumerate(HOST_STATS)}


def cfr_batch_destroy(h):
    _check(_lib.cfr_batch_destroy(h), "cfr_batch_destroy")


# ---- convenience wrapper --------------------------------------------------------

class _Untuned:
    """A Solver or Batch seen by the tuning cache: its tiling, and the plain
    autotuner (so the cache does not recurse into itself)."""

    def __init__(self, obj, tune_fn):
        self._obj, self._tune = obj, tune_fn

    @property
    def tiling(self):
        return self._obj.tiling

    @tiling.setter
    def tiling(self, t):
        self._obj.tiling = t

    def tune(self, reps):
        return self._tune(self._obj.h, reps)


class Solver:
    """One game on one GPU.  Device memory comes from a torch uint8 tensor;
    work is enqueued on torch's current stream of that device.  With
    static_workspace=True the solver is made by cfr_create_static instead: no
    device memory is allocated for it (its state lives in the library's static
    per-device array) and iterations are launched without a graph."""

    def __init__(self, game, precision: str = "fp64", device: int = 0, alpha: float = 1.5,
                 beta: float = 0.0, gamma: float = 2.0, avg: str = "default",
                 use_graph: bool = True, stream=None, with_csc: bool = True,
                 spmv_order: str = "default", down_pass: str = "default",
                 up_pass: str = "default", static_workspace: bool = False):
        import torch
        self.torch = torch
        self.arrays = GameArrays(game, with_csc=with_csc)
        self.n_seq = list(self.arrays.n_seq)
        self.precision = precision
        self.nnz = int(game.nnz)
        o = cfr_options_default()
        o.precision = PRECISIONS[precision]
        o.dcfr_alpha, o.dcfr_beta, o.dcfr_gamma = float(alpha), float(beta), float(gamma)
        o.avg_weight = AVG[avg]
        o.device = int(device)
        o.use_graph = int(bool(use_graph))
        o.spmv_order = SPMV_ORDER[spmv_order]
        o.down_pass = DOWN_PASS[down_pass]
        o.up_pass = UP_PASS[up_pass]
        dev = torch.device("cuda", int(device))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        o.stream = C.c_void_p(int(stream.cuda_stream))
        nbytes = cfr_workspace_size(self.arrays, o)
        if static_workspace:
            self.opts, self.workspace, self.workspace_bytes = o, None, nbytes
            self.h = cfr_create_static(self.arrays, o)
            return
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

    def get_state(self) -> bytes:
        """Checkpoint image of the solver's state (see cfr_get_state)."""
        return cfr_get_state(self.h)

    def set_state(self, state: bytes):
        cfr_set_state(self.h, state)

    @property
    def tiling(self) -> dict:
        return cfr_get_tiling(self.h)

    @tiling.setter
    def tiling(self, t: dict):
        cfr_set_tiling(self.h, t)

    def tune(self, reps: int = 10, cache: str | None = None) -> dict:
        """Autotunes the product tiling; with `cache` (a JSON file path), a
        tiling stored there for this game's size bucket is taken instead,
        and a new choice is stored."""
        if cache is not None:
            from .tuning import size_key, tune_cached
            key = size_key("solver", self.precision, self.nnz, self.n_seq, 1, LIB_PATH)
            return tune_cached(_Untuned(self, cfr_tune), key, cache, reps)[0]
        return cfr_tune(self.h, reps)

    def close(self):
        if getattr(self, "h", None):
            cfr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many games solved together on one GPU (library-owned workspace, work
    on torch's current stream of the device).  Capacities are in index
    units (cfr_batch_game_size); games are added with their own regret
    minimiser and stopping rule and run with checks every `check_every`
    iterations."""

    def __init__(self, seq_capacity, inf_capacity, nnz_capacity: int, max_games: int = 256,
                 precision: str = "fp32_acc64", mode: str = "alternating",
                 check_every: int = 10, device: int = 0, use_graph: bool = True, stream=None,
                 spmv_order: str = "default", down_pass: str = "default",
                 async_admission: bool = False, quad_capacity: int = 0):
        import torch
        o = cfr_batch_options_default()
        o.precision = PRECISIONS[precision]
        o.mode = MODES[mode]
        o.spmv_order = SPMV_ORDER[spmv_order]
        o.max_games = int(max_games)
        for p in range(2):
            o.seq_capacity[p] = int(seq_capacity[p])
            o.inf_capacity[p] = int(inf_capacity[p])
        o.nnz_capacity = int(nnz_capacity)
        o.check_every = int(check_every)
        o.device = int(device)
        o.use_graph = int(bool(use_graph))
        o.down_pass = DOWN_PASS[down_pass]
        o.async_admission = int(bool(async_admission))
        o.quad_capacity = int(quad_capacity)
        dev = torch.device("cuda", int(device))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        o.stream = C.c_void_p(int(stream.cuda_stream))
        self.opts = o
        self.workspace_bytes = cfr_batch_workspace_size(o)
        self.h = cfr_batch_create(o)
        self.precision = precision
        self.n_seq = {}
        self.nnz = {}

    @staticmethod
    def game_size(game) -> np.ndarray:
        return cfr_batch_game_size(GameArrays(game, with_csc=False))

    def add(self, game, variant: str = "pcfr+", target: float = 0.0, max_iterations: int = 0,
            avg: str = "default", alpha: float = 1.5, beta: float = 0.0,
            gamma: float = 2.0) -> int:
        arrays = GameArrays(game)
        gp = cfr_game_params_default()
        gp.variant = VARIANTS[variant]
        gp.avg_weight = AVG[avg]
        gp.dcfr_alpha, gp.dcfr_beta, gp.dcfr_gamma = float(alpha), float(beta), float(gamma)
        gp.target_exploitability = float(target)
        gp.max_iterations = int(max_iterations)
        gid = cfr_batch_add(self.h, arrays, gp)
        self.n_seq[gid] = list(arrays.n_seq)
        self.nnz[gid] = int(game.nnz)
        return gid

    def run(self, n: int) -> int:
        return cfr_batch_run(self.h, n)

    def run_begin(self):
        """Enqueues one check period and returns (cfr_batch_run_begin)."""
        cfr_batch_run_begin(self.h)

    def run_end(self) -> int:
        """Waits for the check period begun and applies its check."""
        return cfr_batch_run_end(self.h)

    def run_ready(self) -> bool:
        """True when run_end would not wait."""
        return cfr_batch_run_ready(self.h)

    def status(self, gid: int) -> dict:
        return cfr_batch_status(self.h, gid)

    def strategy(self, gid: int, player: int, kind: str = "average") -> np.ndarray:
        return cfr_batch_strategy(self.h, gid, player, KINDS[kind], self.n_seq[gid][player])

    def exploitability(self, gid: int, kind: str = "average") -> dict:
        out = cfr_batch_exploitability(self.h, gid, KINDS[kind])
        return {"expl": out[0], "nash_conv": out[1], "br1": out[2], "br2": out[3],
                "value": out[4]}

    def remove(self, gid: int):
        cfr_batch_remove(self.h, gid)
        self.n_seq.pop(gid, None)
        self.nnz.pop(gid, None)

    @property
    def tiling(self) -> dict:
        return cfr_batch_get_tiling(self.h)

    @tiling.setter
    def tiling(self, t: dict):
        cfr_batch_set_tiling(self.h, t)

    def tune(self, reps: int = 10, cache: str | None = None) -> dict:
        """Autotunes the product tiling on the games held; with `cache` (a
        JSON file path), a tiling stored there for this batch's size bucket
        (total nonzeros and sequences, game count) is taken instead, and a
        new choice is stored."""
        if cache is not None:
            from .tuning import size_key, tune_cached
            nnz = sum(self.nnz.values())
            seq = [sum(v[p] for v in self.n_seq.values()) for p in range(2)]
            key = size_key("batch", self.precision, nnz, seq, len(self.n_seq), LIB_PATH)
            return tune_cached(_Untuned(self, cfr_batch_tune), key, cache, reps)[0]
        return cfr_batch_tune(self.h, reps)

    def kernel_timing(self, enable: bool):
        cfr_batch_kernel_timing(self.h, enable)

    def host_stats(self) -> dict:
        return cfr_batch_host_stats(self.h)

    def kernel_stats(self, kernel: int):
        return cfr_batch_kernel_stats(self.h, kernel)

    def close(self):
        if getattr(self, "h", None):
            cfr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
