"""Builds libcfr.so (the HIP kernels and the C ABI) for gfx950, in-tree.

The three sources compile in parallel into objects under ``_build/`` and
link into ``libcfr.so``.  The same host sources are also compiled with the
address sanitiser on the host side only and linked with the same kernel
object into ``libcfr_asan.so``, which the CPU tests load (through
``CFR_LIBRARY``) to run the library's host paths (validation, level
planning, prepared images and their quad copies) under the sanitiser.  The
device code of both libraries is the same object.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcfr.so")
LIB_ASAN = os.path.join(PKG, "libcfr_asan.so")
OBJ = os.path.join(ROOT, "_build")
SOURCES = ["cfr_api.hip", "cfr_engine.hip", "cfr_kernels.hip"]
HOST_SOURCES = ["cfr_api.hip", "cfr_engine.hip"]  # no kernels in these

COMMON = ["--offload-arch=gfx950", "-std=c++17", "-fPIC",
          # sums are taken in a fixed order without contraction, so the FP64
          # path rounds exactly like a plain sequential evaluation
          "-ffp-contract=off",
          # no packed FP32 instructions
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC]
# host-side sanitiser only (the device code is not instrumented)
ASAN = ["-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer", "-g"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def asan_runtime() -> str | None:
    """The compiler's address-sanitiser runtime (preloaded by the process
    that loads libcfr_asan.so), or None."""
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return cands[-1] if cands else None


def _run_all(cmds, verbose):
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append((cmd, subprocess.Popen(cmd)))
    bad = [cmd for cmd, p in procs if p.wait() != 0]
    if bad:
        raise subprocess.CalledProcessError(1, bad[0])


def build(verbose: bool = False, asan: bool = True) -> str:
    """Compiles every source for gfx950 and links libcfr.so (and, with asan,
    libcfr_asan.so); always recompiles."""
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    obj = {s: os.path.join(OBJ, s.replace(".hip", ".o")) for s in SOURCES}
    obj_asan = {s: os.path.join(OBJ, s.replace(".hip", "_asan.o")) for s in HOST_SOURCES}
    cmds = [[cc, *COMMON, "-O3", "-c", os.path.join(CSRC, s), "-o", obj[s]] for s in SOURCES]
    if asan:
        cmds += [[cc, *COMMON, "-O1", *ASAN, "-c", os.path.join(CSRC, s), "-o", obj_asan[s]]
                 for s in HOST_SOURCES]
    _run_all(cmds, verbose)
    tmp = LIB + ".tmp"
    _run_all([[cc, "--offload-arch=gfx950", "-shared", "-fPIC", *[obj[s] for s in SOURCES],
               "-o", tmp]], verbose)
    os.replace(tmp, LIB)
    if asan:
        tmp = LIB_ASAN + ".tmp"
        _run_all([[cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan",
                   "-Xarch_host", "-fsanitize=address",
                   *[obj_asan[s] for s in HOST_SOURCES], obj["cfr_kernels.hip"], "-o", tmp]],
                 verbose)
        os.replace(tmp, LIB_ASAN)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
