"""Throughput of sequence-form CFR on one MI355X.

Default workload: the large synthetic game (32 signals per player, depth-10
public tree with branching U{2,3,4}, showdown payoffs, ~1e5 public terminals,
~1.0e8 payoff nonzeros), DCFR(alpha=1.5, beta=0, gamma=2) with alternating
updates, FP32 payoffs/strategies with FP64 regret and average accumulators.
One step = one full CFR iteration (both payoff products, both players'
bottom-up and top-down sweeps, the regret update, regret matching and the
average-strategy accumulation), with the game already resident in HBM.

Prints one JSON line: iterations/s, plus nnz*iterations/s, whole-iteration
algorithmic GB/s, a roofline entry for the dominant kernel (the payoff
product, timed with HIP events on the solver's stream) and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """Digest of the payoff-product kernel's source and of its tiling
    constants: the committed HBM-traffic figures are valid only for the
    kernel they were measured on."""
    csrc = os.path.join(ROOT, "paper_2605_14277_amd", "csrc")
    with open(os.path.join(csrc, "cfr_kernels.hip")) as fh:
        text = fh.read()
    start = text.index("// SEQ: every row is summed strictly left to right")
    end = text.index("// ----", start)
    h = hashlib.sha256(text[start:end].encode())
    with open(os.path.join(csrc, "cfr_internal.h")) as fh:
        for line in fh:
            if "SPMV" in line or "kSpmv" in line:
                h.update(line.encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, digest: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "spmv_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    ent = rec.get(kernel)
    if not ent or ent.get("kernel_digest") != digest:
        return None
    return ent.get("bytes_per_launch")


def algorithmic_bytes_per_iteration(g, vbytes: int, abytes: int, predictive: bool) -> float:
    """Bytes one iteration must move at minimum: both payoff streams (index +
    value), row pointers, each gathered vector once and each product's output
    once, and per sequence: regret and average read-modify-write in the
    accumulator type, the utility read, the behavioural strategy written and
    read, the strategy written, one int32 of treeplex structure (plus the
    prediction's read and write for predictive variants)."""
    n1, n2 = g.n_seq
    payoff = 2 * g.nnz * (4 + vbytes) + 4 * (n1 + 1) + 4 * (n2 + 1)
    vectors = 2 * (n1 + n2) * vbytes
    per_seq = 4 * abytes + 4 * vbytes + 4 + (2 * abytes if predictive else 0)
    return float(payoff + vectors + (n1 + n2) * per_seq)


def cpu_baseline(g, variant, mode, budget_s: float):
    import oracle
    o = oracle.Oracle(g)
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step(1, variant, mode)
        n += 1
        el = time.perf_counter() - t0
        if (el >= budget_s and n >= 2) or n >= 200:
            break
    o.close()
    return n, el


def copy_probe(torch, nbytes: int = 1600 << 20, reps: int = 5):
    """A plain copy of known size: each launch reads and writes nbytes."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                      "ms_per_copy": ms, "copy_GBs": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="cfg3", choices=["cfg1", "cfg2", "cfg2_d8", "cfg3"])
    ap.add_argument("--variant", default=None)
    ap.add_argument("--mode", default=None)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--spmv-order", default="default", choices=["default", "sequential", "parallel"])
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain device copy of 1.6 GiB (the HBM reference that "
                         "scales the FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        log("bench.py measures one GPU only: this build has no multi-GPU path "
            "(the sharding design is described in DESIGN.md). Run with --gpus 1.")
        sys.exit(2)

    import torch

    if args.copy_probe:
        copy_probe(torch)
        return

    import gamegen as gg
    import paper_2605_14277_amd as cfr

    defaults = {"cfg1": ("vanilla", "simultaneous", "fp64"),
                "cfg2": ("cfr+", "alternating", "fp64"),
                "cfg2_d8": ("cfr+", "alternating", "fp64"),
                "cfg3": ("dcfr", "alternating", "fp32_acc64")}[args.config]
    variant = args.variant or defaults[0]
    mode = args.mode or defaults[1]
    precision = args.precision or defaults[2]

    t0 = time.perf_counter()
    g = gg.make_config(args.config)
    log(f"[bench] game {args.config}: {g.summary()} built in {time.perf_counter() - t0:.1f}s")
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    s = cfr.Solver(g, precision=precision, device=0, use_graph=not args.no_graph,
                   spmv_order=args.spmv_order)
    torch.cuda.synchronize()
    log(f"[bench] cfr_create {time.perf_counter() - t0:.1f}s, workspace {s.workspace_bytes / 1e9:.2f} GB")

    s.step(args.warmup, variant, mode)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")

    stream = s.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    s.step(args.steps, variant, mode)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    its = 1000.0 / ms_per_step
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step (wall {wall:.3f}s)")

    # per-kernel timing of the payoff products over a second timed region
    s.kernel_timing(True)
    kt_steps = max(10, min(args.steps, 100))
    s.step(kt_steps, variant, mode)
    torch.cuda.synchronize()
    stats = []
    for k, name in ((0, "spmv_csr"), (1, "spmv_csc")):
        n, tot, by = s.kernel_stats(k)
        stats.append((tot, name, n, by))
    s.kernel_timing(False)
    stats.sort(reverse=True)
    tot, kname, nl, by = stats[0]
    avg_ms = tot / nl
    achieved = by / (avg_ms * 1e-3) / 1e9
    digest = kernel_source_digest()
    traffic = measured_traffic(kname, digest)
    e = s.exploitability("average")
    log(f"[bench] {kname}: {nl} launches, {avg_ms * 1e3:.1f} us avg, {achieved:.0f} GB/s "
        f"(algorithmic); expl after {s.iteration} it = {e['expl']:.4g}")

    vbytes = 8 if precision == "fp64" else 4
    abytes = 4 if precision == "fp32" else 8
    alg = algorithmic_bytes_per_iteration(g, vbytes, abytes, variant in ("pcfr+", "pcfr"))

    cpu = None
    if not args.no_cpu_baseline:
        n_cpu, el = cpu_baseline(g, variant, mode, args.cpu_budget)
        cpu = {"value": n_cpu / el, "unit": "iter/s", "cores": 1, "kind": "oracle",
               "sample": f"{n_cpu} iterations of the same workload ({args.config}, {variant}, "
                         f"{mode}) by the single-threaded FP64 C oracle, {el:.1f}s"}
        log(f"[bench] cpu oracle {n_cpu} it in {el:.1f}s")

    out = {
        "metric": "CFR iters/s + HBM GB/s at 1e8 nnz",
        "value": its,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_acc64": "f32+f64acc"}[precision],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {g.name}, {variant}, {mode}, {precision}",
                   "nnz": g.nnz, "n_seq": list(g.n_seq), "terminals": g.tree.n_terminals
                   if g.tree is not None else None, "graph": not args.no_graph},
        "nnz_iters_per_s": g.nnz * its,
        "algorithmic_gb_per_iter": alg / 1e9,
        "iteration_gbs": alg / (ms_per_step * 1e-3) / 1e9,
        "iteration_hbm_frac": alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_us": avg_ms * 1e3,
                     "bytes_per_launch": by},
        "cpu_baseline": cpu,
        "expl_average": e["expl"],
    }
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
