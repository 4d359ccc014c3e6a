"""Serving loop with continuous batching on one GPU.

Requests (a game, a regret minimiser, an exploitability target, an
iteration limit) arrive over time.  Arriving games are prepared on worker
threads (``cfr_prepare``: validation, level order, float conversion; no
device work, and ctypes releases the GIL), so preparation overlaps the
device's iterations.  At each check boundary the loop admits waiting
requests in arrival order while they fit the batch's free slots and device
ranges (``cfr_batch_add_prepared`` returns CFR_ENOMEM otherwise), begins one
check period of every game in the batch (``cfr_batch_run_begin``), and
when it has ended (``cfr_batch_run_end``) frees the games that met their
stopping rule.  Optionally small games are served by a second batch on a
stream of its own.  Admission at check boundaries keeps
every game's iterates and checks identical to the game solved alone.  A
request that cannot be served (a malformed game, or one larger than the
whole batch) is answered as rejected, with the library's error code, and
the loop serves the others on.

The device capacity is sized from a byte budget (``capacities_for_bytes``)
with the index-unit proportions of the expected request mix.
"""
from __future__ import annotations

import ctypes as C
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import (AVG, CFR_ENOMEM, PRECISIONS, VARIANTS, Batch, CfrError, GameArrays, _check, _lib,
               cfr_batch_options_default, cfr_batch_workspace_size, cfr_game_params_default)


class Prepared:
    """A game prepared on the host for batches of one precision."""

    def __init__(self, game, precision: str = "fp32_acc64", quads=None):
        arrays = GameArrays(game)
        self.precision = precision
        self.n_seq = list(arrays.n_seq)
        h = C.c_void_p()
        _check(_lib.cfr_prepare(C.byref(arrays.desc), PRECISIONS[precision], C.byref(h)),
               "cfr_prepare")
        self.h = h
        units = np.zeros(5, dtype=np.int64)
        _check(_lib.cfr_prepared_size(h, units.ctypes.data_as(C.POINTER(C.c_int64))),
               "cfr_prepared_size")
        self.units = units
        if quads is not None:
            self.prepare_quads(quads)

    def prepare_quads(self, perm):
        """Quad copies of both products (stream form 3) in column orders
        perm = (A y, A^T x) (0: as numbered, 1: first-touch), built here on
        the host so that admission only copies them."""
        arr = (C.c_int * 2)(int(perm[0]), int(perm[1]))
        _check(_lib.cfr_prepare_quads(self.h, arr), "cfr_prepare_quads")

    def close(self):
        if getattr(self, "h", None):
            _lib.cfr_prepared_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def add_prepared(batch: Batch, prep: Prepared, variant: str, target: float = 0.0,
                 max_iterations: int = 0, avg: str = "default", alpha: float = 1.5,
                 beta: float = 0.0, gamma: float = 2.0) -> int:
    gp = cfr_game_params_default()
    gp.variant = VARIANTS[variant]
    gp.avg_weight = AVG[avg]
    gp.dcfr_alpha, gp.dcfr_beta, gp.dcfr_gamma = float(alpha), float(beta), float(gamma)
    gp.target_exploitability = float(target)
    gp.max_iterations = int(max_iterations)
    gid = C.c_int64(-1)
    _check(_lib.cfr_batch_add_prepared(batch.h, prep.h, C.byref(gp), C.byref(gid)),
           "cfr_batch_add_prepared")
    batch.n_seq[int(gid.value)] = list(prep.n_seq)
    batch.nnz[int(gid.value)] = int(prep.units[4])
    return int(gid.value)


def capacities_for_bytes(budget: int, mix_units, max_games: int, precision: str = "fp32_acc64"):
    """Largest capacities in the proportions of `mix_units` (the summed
    index units of a representative set of games) whose batch workspace
    fits `budget` bytes.  Returns (seq[2], inf[2], nnz)."""
    mix = np.asarray(mix_units, dtype=np.float64)

    def caps(scale):
        u = np.maximum(np.ceil(mix * scale), [2, 2, 1, 1, 0]).astype(np.int64)
        return [int(u[0]), int(u[1])], [int(u[2]), int(u[3])], int(u[4])

    def size(scale):
        o = cfr_batch_options_default()
        o.precision = PRECISIONS[precision]
        o.max_games = int(max_games)
        seq, inf, nnz = caps(scale)
        for p in range(2):
            o.seq_capacity[p] = seq[p]
            o.inf_capacity[p] = inf[p]
        o.nnz_capacity = nnz
        return cfr_batch_workspace_size(o)

    lo, hi = 0.0, 1.0
    while size(hi) <= budget:
        lo, hi = hi, hi * 2
    for _ in range(50):
        mid = (lo + hi) / 2
        if size(mid) <= budget:
            lo = mid
        else:
            hi = mid
    return caps(lo)


class _Lane:
    """One batch of the server with its own queue of admitted-to-be requests
    and its games in flight."""

    def __init__(self, batch: Batch, capacity, nnz_limit, solo: int = 0, admit_after: float = 0.0):
        self.batch = batch
        self.capacity = capacity  # index units of the whole batch
        self.nnz_limit = nnz_limit  # requests with at most this many nonzeros (None: any)
        # with `solo` games in flight, a waiting request is admitted beside
        # them only once it has waited `admit_after` seconds (0: no limit)
        self.solo = solo
        self.admit_after = admit_after
        self.waiting = deque()  # appended by the serving thread, taken by the lane's
        self.inflight = {}
        self.running = False  # a check period has been begun and not ended
        self.wake = threading.Event()  # a request has been routed to the lane


class Server:
    """Continuous batching over one Batch, or two: with `small` (a dict with
    seq_capacity, inf_capacity, nnz_capacity, max_games, nnz_limit and
    optionally quad_capacity) requests whose game has at most nnz_limit
    payoff nonzeros go to a second batch on a stream of its own, so that
    small games iterate without waiting for the large games' launches (in one
    batch every game advances one iteration per iteration of the whole
    batch).  Each lane runs its check periods asynchronously
    (cfr_batch_run_begin / cfr_batch_run_end, polled with
    cfr_batch_run_ready) from a host thread of its own, so the admissions,
    table builds and uploads of one lane overlap the other lane's iterations
    and host work; the serving thread takes arrivals and routes them.  With `solo` the lane that
    takes any request holds that many games and admits another beside them
    only once it has waited `admit_after` seconds: at light load large games
    run on their own (in a batch each game advances one iteration per
    iteration of the whole batch, so a large game shares the device's
    bandwidth with every other), while a queue that builds up under load
    brings batching back."""

    def __init__(self, seq_capacity, inf_capacity, nnz_capacity, max_games: int = 256,
                 precision: str = "fp32_acc64", check_every: int = 10, workers: int = 8,
                 device: int = 0, async_admission: bool = True, tiling: dict | None = None,
                 quad_capacity: int = 0, small: dict | None = None, solo: int = 0,
                 admit_after: float = 0.0):
        import torch
        # column orders of the quad copies that arriving requests get built
        # on the worker threads (stream form 3 on some product), else None
        self.quad_perm = None
        if tiling is not None and 3 in tiling["vec"]:
            self.quad_perm = tuple(int(v) for v in tiling["perm"])

        def lane(seq, inf, nnz, games, qcap, limit, stream, solo_=0, after=0.0):
            # asynchronous admission: a request's copies to the device overlap
            # the iterations of the requests already running
            b = Batch(seq, inf, nnz, max_games=games, precision=precision, mode="alternating",
                      check_every=check_every, device=device, async_admission=async_admission,
                      quad_capacity=qcap, stream=stream)
            if tiling is not None:
                b.tiling = tiling
            cap = np.array([seq[0], seq[1], inf[0], inf[1], nnz], dtype=np.int64)
            return _Lane(b, cap, limit, solo_, after)

        self.lanes = []
        if small is not None:
            st = torch.cuda.Stream(device=torch.device("cuda", int(device)))
            self.lanes.append(lane(small["seq_capacity"], small["inf_capacity"],
                                   small["nnz_capacity"], small["max_games"],
                                   small.get("quad_capacity", 0), small["nnz_limit"], st))
        self.lanes.append(lane(seq_capacity, inf_capacity, nnz_capacity, max_games, quad_capacity,
                               None, None, solo, admit_after))
        self.batch = self.lanes[-1].batch  # the lane that takes any request
        self.precision = precision
        self.check_every = check_every
        self.workers = workers

    def host_stats(self) -> dict:
        """Host time and calls per activity, summed over the lanes."""
        tot = {}
        for ln in self.lanes:
            for k, v in ln.batch.host_stats().items():
                t = tot.setdefault(k, {"seconds": 0.0, "calls": 0})
                t["seconds"] += v["seconds"]
                t["calls"] += v["calls"]
        return tot

    def _lane_for(self, units) -> _Lane:
        for ln in self.lanes:
            if ln.nnz_limit is not None and units[4] <= ln.nnz_limit and \
                    np.all(np.asarray(units) <= ln.capacity):
                return ln
        return self.lanes[-1]

    def serve(self, requests, keep_strategies: bool = False, prepared=None) -> list:
        """Serves `requests` in real time: a list of dicts with "arrival"
        (seconds from the start, ascending), "game" (or an index into
        `prepared`, a list of Prepared games: "prepared"), "variant",
        "target" and "max_iterations".  Returns one record per request:
        arrival, admitted, finished, latency, iterations, expl,
        reached_target, state and lane (0 for the small-game lane when there
        is one) (and the average strategies with keep_strategies).  state is
        "done" for a solved request; a request that cannot be served is
        answered with state "rejected" (its game is malformed: the library's
        error code and message in "code" and "error"; or it is larger than
        the whole batch: CFR_ENOMEM) and the loop goes on serving the
        others."""
        n = len(requests)
        out = [None] * n
        futures = [None] * n
        pool = ThreadPoolExecutor(max_workers=self.workers)
        clock = time.perf_counter
        t0 = clock()
        next_arrival = 0
        arrived = deque()  # arrived, not yet routed to a lane (preparation running)

        def reject(k, code, msg):
            now = clock() - t0
            out[k] = {"arrival": requests[k]["arrival"], "admitted": None, "finished": now,
                      "latency": now - requests[k]["arrival"], "iterations": 0, "expl": None,
                      "reached_target": 0, "state": "rejected", "code": code, "error": msg,
                      "lane": None}

        def collect(li, ln):
            now = clock() - t0
            for gid in list(ln.inflight):
                st = ln.batch.status(gid)
                if st["state"] != "done":
                    continue
                k, admitted, _ = ln.inflight.pop(gid)
                rec = {"arrival": requests[k]["arrival"], "admitted": admitted,
                       "finished": now, "latency": now - requests[k]["arrival"],
                       "iterations": st["iterations"], "expl": st["expl"],
                       "reached_target": st["reached_target"], "state": "done", "lane": li}
                if keep_strategies:
                    rec["strategy"] = [ln.batch.strategy(gid, p, "average") for p in range(2)]
                ln.batch.remove(gid)
                out[k] = rec

        def admit(ln):
            # admit in arrival order while the head fits
            while ln.waiting:
                k, prep = ln.waiting[0]
                r = requests[k]
                if ln.solo and len(ln.inflight) >= ln.solo and \
                        clock() - t0 - r["arrival"] < ln.admit_after:
                    break  # the lane is busy and the head has not waited long enough
                if np.any(np.asarray(prep.units) > ln.capacity):
                    ln.waiting.popleft()
                    reject(k, CFR_ENOMEM, "the game is larger than the whole batch")
                    continue
                try:
                    gid = add_prepared(ln.batch, prep, r["variant"], r["target"],
                                       r["max_iterations"])
                except CfrError as e:
                    if e.code == CFR_ENOMEM and ln.inflight:
                        break  # waits for games in flight to free space
                    ln.waiting.popleft()
                    reject(k, e.code, str(e))
                    continue
                ln.waiting.popleft()
                # the prepared game stays referenced while its copies may run
                ln.inflight[gid] = (k, clock() - t0, prep)

        routed_all = threading.Event()  # every request has been routed (or rejected)
        abort = threading.Event()
        errors = []

        def lane_loop(li, ln):
            # one host thread per lane: its admissions, table builds and
            # uploads (library calls, which release the interpreter lock)
            # overlap the other lane's
            try:
                while not abort.is_set():
                    if ln.running:
                        while not ln.batch.run_ready():
                            time.sleep(5e-5)  # the check period is still on the device
                        ln.batch.run_end()
                        ln.running = False
                        collect(li, ln)
                    admit(ln)
                    if ln.inflight:
                        ln.batch.run_begin()
                        ln.running = True
                        continue
                    ln.wake.clear()
                    if ln.waiting:
                        continue
                    if routed_all.is_set():
                        break
                    ln.wake.wait(0.01)
            except BaseException as e:  # reported by the serving thread
                errors.append(e)
                abort.set()
            finally:
                if ln.running:
                    ln.running = False
                    ln.batch.run_end()

        threads = [threading.Thread(target=lane_loop, args=(li, ln), daemon=True)
                   for li, ln in enumerate(self.lanes)]
        for th in threads:
            th.start()
        try:
            while (next_arrival < n or arrived) and not abort.is_set():
                now = clock() - t0
                while next_arrival < n and requests[next_arrival]["arrival"] <= now:
                    k = next_arrival
                    r = requests[k]
                    if "prepared" in r:
                        futures[k] = prepared[r["prepared"]]
                    else:
                        futures[k] = pool.submit(Prepared, r["game"], self.precision,
                                                 self.quad_perm)
                    arrived.append(k)
                    next_arrival += 1
                # route prepared requests, in arrival order, to their lanes
                while arrived:
                    k = arrived[0]
                    f = futures[k]
                    if not isinstance(f, Prepared) and not f.done():
                        break
                    arrived.popleft()
                    try:
                        prep = f if isinstance(f, Prepared) else f.result()
                    except CfrError as e:  # the game failed validation
                        reject(k, e.code, str(e))
                        continue
                    ln = self._lane_for(prep.units)
                    ln.waiting.append((k, prep))
                    ln.wake.set()
                if arrived:
                    time.sleep(0.0005)  # the head is still being prepared
                elif next_arrival < n:
                    time.sleep(min(0.01, max(0.0, requests[next_arrival]["arrival"] -
                                             (clock() - t0))))
        except BaseException:
            abort.set()
            raise
        finally:
            routed_all.set()
            for ln in self.lanes:
                ln.wake.set()
            for th in threads:
                th.join()
            pool.shutdown(wait=True)
        if errors:
            raise errors[0]
        return out

    def close(self):
        for ln in self.lanes:
            ln.batch.close()


def sequential_latencies(arrivals, service_times):
    """Latencies of one-at-a-time FIFO service with the given per-request
    service times (a single server: each request starts when it has arrived
    and the previous one has finished)."""
    free = 0.0
    lat = []
    for a, s in zip(arrivals, service_times):
        start = max(a, free)
        free = start + s
        lat.append(free - a)
    return np.array(lat)
