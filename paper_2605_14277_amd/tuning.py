"""Autotuner results kept in a JSON file, keyed by size bucket.

A product tiling chosen by the autotuner (cfr_tune / cfr_batch_tune) depends
on the shape of the work: the precision, the number of nonzeros and the
lengths of the two strategy vectors (and, for a batch, how many games share
the launches).  Those are bucketed by powers of two, together with a digest
of the built library (a rebuilt kernel invalidates every entry), and the
choice for a bucket is stored so that a later solver or batch of the same
bucket takes it without timing anything.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

_LIB_DIGEST = None


def library_digest(path: str) -> str:
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        h = hashlib.sha256()
        with open(path, "rb") as fh:
            for chunk in iter(lambda: fh.read(1 << 20), b""):
                h.update(chunk)
        _LIB_DIGEST = h.hexdigest()[:16]
    return _LIB_DIGEST


def _bucket(v) -> int:
    return int(round(math.log2(max(int(v), 1))))


def size_key(kind: str, precision: str, nnz: int, n_seq, games: int, lib_path: str) -> str:
    """Bucket of a workload: kind ("solver" or "batch"), precision, and the
    nearest powers of two of its nonzeros, of each player's sequences and of
    its game count."""
    return (f"{kind}|{precision}|nnz 2^{_bucket(nnz)}|seq 2^{_bucket(n_seq[0])},"
            f"2^{_bucket(n_seq[1])}|games 2^{_bucket(games)}|lib {library_digest(lib_path)}")


def tune_cached(obj, key: str, path: str, reps: int) -> tuple[dict, bool]:
    """The cached tiling for `key` applied to `obj` (a Solver or Batch), or
    the autotuner's choice, stored under `key`.  Returns (tiling, hit)."""
    cache = {}
    if os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    if key in cache:
        obj.tiling = cache[key]
        return obj.tiling, True
    tiling = obj.tune(reps)
    cache[key] = tiling
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return tiling, False
