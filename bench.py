"""Throughput of sequence-form CFR on one MI355X.

Default workload: the large synthetic game (32 signals per player, depth-10
public tree with branching U{2,3,4}, showdown payoffs, ~1e5 public terminals,
~1.0e8 payoff nonzeros), DCFR(alpha=1.5, beta=0, gamma=2) with alternating
updates, FP32 payoffs/strategies with FP64 regret and average accumulators.
One step = one full CFR iteration (both payoff products, both players'
bottom-up and top-down sweeps, the regret update, regret matching and the
average-strategy accumulation), with the game already resident in HBM.

Prints one JSON line: iterations/s (the timed steps in five consecutive
event-bracketed regions: mean, SEM and median per region), nnz*iterations/s,
the bytes the iteration streams and their rate, a roofline entry for the
dominant kernel (the slower payoff product, timed per launch with HIP events
the launch itself sets), the all-core CPU oracle run to the same iteration
count (its rate is the CPU baseline; its exploitability gives the GPU's
error) beside a single-threaded sample, the same game in FP64, and the
batched and served records (many games of uneven size solved together
against the same games one at a time, and against plain CFR).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
DTYPES = {"fp64": "f64", "fp32": "f32", "fp32_acc64": "f32+f64acc"}


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
    # the definitions of the constants and macros the kernel uses
    defs = re.compile(r"^\s*(constexpr\s+\S+\s+(kSpmv\w*|kStreamPad|kQuadMaskShift|"
                      r"kQuadIndexMask)\s*=|#define\s+CFR_SPMV\w*|#ifndef\s+CFR_SPMV\w*|"
                      r"__host__ __device__ constexpr int spmv_block_cap\(int items\))")
    with open(os.path.join(csrc, "cfr_internal.h")) as fh:
        for line in fh:
            if defs.match(line):
                h.update(line.encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, digest: str, tiling: dict):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source with the same tiling; else
    None."""
    path = os.path.join(ROOT, "profiles", "spmv_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    ent = rec.get(kernel)
    if not ent or ent.get("kernel_digest") != digest or ent.get("tiling") != tiling:
        return None
    return ent.get("bytes_per_launch")


def sweep_bytes_per_sequence(vbytes: int, abytes: int, predictive: bool) -> int:
    """Per sequence and iteration: regret and average read-modify-write in
    the accumulator type, the utility read, the behavioural strategy written
    and read, the strategy written, one int32 of treeplex structure (plus
    the prediction's read and write for predictive variants)."""
    return 4 * abytes + 4 * vbytes + 4 + (2 * abytes if predictive else 0)


def element_product_bytes(g, w: int, vbytes: int) -> float:
    """Bytes of one payoff product in the element stream (index and value per
    nonzero), row pointers, the gathered vector once and the output once."""
    rows, cols = g.n_seq[w], g.n_seq[1 - w]
    return float(g.nnz * (4 + vbytes) + 4 * (rows + 1) + vbytes * (cols + rows))


def iteration_bytes(g, vbytes: int, abytes: int, predictive: bool, product_bytes=None) -> float:
    """Bytes one iteration moves at minimum: the two products (element
    streams when product_bytes is None, else the bytes each launch's own
    stream form reads, as the library counts them) and the sweeps."""
    if product_bytes is None:
        product_bytes = [element_product_bytes(g, w, vbytes) for w in (0, 1)]
    n1, n2 = g.n_seq
    return float(sum(product_bytes) + (n1 + n2) * sweep_bytes_per_sequence(vbytes, abytes,
                                                                            predictive))


def host_cpu() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def oracle_sample(g, variant, mode, budget_s: float, parallel: bool, max_iters: int = 200,
                  **kw):
    """Iterations of the oracle (plain or all-core build) within about
    budget_s seconds (at least two); returns (iterations, seconds, threads)."""
    import oracle
    o = oracle.Oracle(g, parallel=parallel, **kw)
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step(1, variant, mode)
        n += 1
        el = time.perf_counter() - t0
        if (el >= budget_s and n >= 2) or n >= max_iters:
            break
    th = o.threads
    o.close()
    return n, el, th


def oracle_to(g, variant, mode, iters: int, **kw):
    """The all-core oracle run for exactly `iters` iterations: (seconds,
    threads, exploitability record of its average profile)."""
    import oracle
    o = oracle.Oracle(g, parallel=True, **kw)
    t0 = time.perf_counter()
    o.step(iters, variant, mode)
    el = time.perf_counter() - t0
    e = o.exploitability("average")
    th = o.threads
    o.close()
    return el, th, {k: float(v) for k, v in e.items()}


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


def parse_tiling(text: str) -> dict:
    """'items_Ay,items_ATx:rows_Ay,rows_ATx[:vec_Ay,vec_ATx[:perm_Ay,perm_ATx[:xcd_Ay,xcd_ATx]]]'."""
    parts = text.split(":")
    return {"items": [int(v) for v in parts[0].split(",")],
            "rows": [int(v) for v in parts[1].split(",")],
            "vec": [int(v) for v in parts[2].split(",")] if len(parts) > 2 else [1, 1],
            "perm": [int(v) for v in parts[3].split(",")] if len(parts) > 3 else [0, 0],
            "xcd": [int(v) for v in parts[4].split(",")] if len(parts) > 4 else [1, 1]}


def timed_steps(torch, s, steps: int, variant: str, mode: str, regions: int = 5) -> dict:
    """Exactly `steps` iterations on the solver's stream, synchronised on both
    sides, split into up to `regions` consecutive regions bracketed by HIP
    events (recorded between graph launches, so the device never waits for
    the host between regions).  Returns the total and per-region ms/step."""
    regions = max(1, min(regions, steps))
    sizes = [steps // regions + (1 if i < steps % regions else 0) for i in range(regions)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(regions + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev[0].record(s.stream)
    for i, n in enumerate(sizes):
        s.step(n, variant, mode)
        ev[i + 1].record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    per = [ev[i].elapsed_time(ev[i + 1]) / n for i, n in enumerate(sizes)]
    total = ev[0].elapsed_time(ev[-1])
    mean = sum(per) / len(per)
    sem = (math.sqrt(sum((p - mean) ** 2 for p in per) / (len(per) - 1) / len(per))
           if len(per) > 1 else 0.0)
    med = sorted(per)[len(per) // 2] if len(per) % 2 else \
        0.5 * (sorted(per)[len(per) // 2 - 1] + sorted(per)[len(per) // 2])
    return {"ms_per_step": total / steps, "wall_s": wall, "regions": len(per),
            "region_steps": sizes, "region_ms_per_step": per, "mean_ms": mean, "sem_ms": sem,
            "median_ms": med}


def product_timing(torch, s, steps: int, variant: str, mode: str):
    """Per-launch HIP-event timing of both products over `steps` iterations:
    [(mean ms per launch, launches, bytes per launch of the stream form in
    use)] for A y and A^T x."""
    s.kernel_timing(True)
    s.step(steps, variant, mode)
    torch.cuda.synchronize()
    out = []
    for k in (0, 1):
        n, tot, by = s.kernel_stats(k)
        out.append((tot / n, n, by))
    s.kernel_timing(False)
    return out


def solve_alone(cfr, g, variant, target, max_it, K, precision, tiling=None):
    """One game solved alone with the same stopping rule as in a batch:
    checks every K iterations, stop at exploitability <= target or max_it.
    With a tiling, the solver uses it too; its set-up (the quad copies of
    stream form 3) happens before the timed solve, as the game's creation
    does."""
    s = cfr.Solver(g, precision=precision)
    if tiling is not None:
        s.tiling = tiling
        s.exploitability("current")  # builds the tables (and quad copies) untimed
    t0 = time.perf_counter()
    while True:
        s.step(K, variant, "alternating")
        e = s.exploitability("average")["expl"]
        if e <= target or s.iteration >= max_it:
            break
    el = time.perf_counter() - t0
    it = s.iteration
    s.close()
    return el, it, e


def solver_line(torch, cfr, g, precision, variant, mode, steps, warmup, tiling=None,
                tune=True, graph=True, spmv_order="default"):
    """Creates a solver, tunes (or sets) its tiling, warms up, times `steps`
    iterations and both products per launch.  Returns (solver, record)."""
    t0 = time.perf_counter()
    s = cfr.Solver(g, precision=precision, device=0, use_graph=graph, spmv_order=spmv_order)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    tune_s = None
    if tiling is not None:
        s.tiling = tiling
    elif tune:
        t0 = time.perf_counter()
        s.tune(reps=10)
        tune_s = time.perf_counter() - t0
    s.step(warmup, variant, mode)
    torch.cuda.synchronize()
    tm = timed_steps(torch, s, steps, variant, mode)
    prod = product_timing(torch, s, max(10, min(steps, 100)), variant, mode)
    vbytes = 8 if precision == "fp64" else 4
    abytes = 4 if precision == "fp32" else 8
    pred = variant in ("pcfr+", "pcfr")
    # the slower product is the dominant kernel
    w = 0 if prod[0][0] >= prod[1][0] else 1
    ms_l, n_l, fmt_by = prod[w]
    streamed = iteration_bytes(g, vbytes, abytes, pred, [p[2] for p in prod])
    alg = iteration_bytes(g, vbytes, abytes, pred)
    rec = {"precision": precision, "iters_per_s": 1e3 / tm["ms_per_step"],
           "ms_per_step": tm["ms_per_step"], "timing": tm, "tiling": s.tiling,
           "tuned": tune_s is not None, "create_s": create_s, "tune_s": tune_s,
           "workspace_gb": s.workspace_bytes / 1e9,
           "products": [{"kernel": k, "avg_launch_us": prod[i][0] * 1e3, "launches": prod[i][1],
                         "bytes_per_launch": prod[i][2],
                         "gbs": prod[i][2] / (prod[i][0] * 1e-3) / 1e9,
                         "element_bytes_per_launch": element_product_bytes(g, i, vbytes)}
                        for i, k in enumerate(("spmv_csr", "spmv_csc"))],
           "dominant": w, "streamed_gb_per_iter": streamed / 1e9,
           "algorithmic_gb_per_iter": alg / 1e9,
           "iteration_gbs": streamed / (tm["ms_per_step"] * 1e-3) / 1e9,
           "iteration_hbm_frac": streamed / (tm["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "kernel_ms": ms_l, "kernel_bytes": fmt_by}
    return s, rec


def bench_large(args, torch):
    """The large game (default), or another single-game configuration."""
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
    tiling = parse_tiling(args.tiling) if args.tiling else None
    s, rec = solver_line(torch, cfr, g, precision, variant, mode, args.steps, args.warmup,
                         tiling=tiling, tune=not args.no_tune, graph=not args.no_graph,
                         spmv_order=args.spmv_order)
    tm = rec["timing"]
    log(f"[bench] product tiling {rec['tiling']}" + (f" (autotuner, {rec['tune_s']:.1f}s)"
                                                     if rec["tune_s"] else ""))
    log(f"[bench] timed {args.steps} steps: {tm['ms_per_step']:.4f} ms/step; regions "
        f"{tm['mean_ms']:.4f} +- {tm['sem_ms']:.4f} ms (median {tm['median_ms']:.4f})")
    # the error against the oracle is taken at the stated horizon (the
    # configs' 1000 iterations): the solver continues untimed to it
    if args.error_iterations > s.iteration:
        s.step(args.error_iterations - s.iteration, variant, mode)
    t_gpu = s.iteration
    e_gpu = {k: float(v) for k, v in s.exploitability("average").items()}
    s.close()

    w = rec["dominant"]
    kname = rec["products"][w]["kernel"]
    ms_l, fmt_by = rec["kernel_ms"], rec["kernel_bytes"]
    el_by = rec["products"][w]["element_bytes_per_launch"]
    achieved = fmt_by / (ms_l * 1e-3) / 1e9
    traffic = measured_traffic(kname, kernel_source_digest(), rec["tiling"])
    log(f"[bench] {kname}: {rec['products'][w]['launches']} launches, {ms_l * 1e3:.1f} us avg, "
        f"{achieved:.0f} GB/s of the bytes its stream form reads ({achieved / HBM_PEAK_GBS:.3f} "
        f"of 8 TB/s); element-stream equivalent {el_by / (ms_l * 1e-3) / 1e9:.0f} GB/s")

    # CPU: the all-core oracle to the GPU's iteration count (the baseline,
    # and the GPU's error at equal iterations), and a single-threaded sample
    cpu, err = None, None
    if not args.no_cpu_baseline:
        el, th, e_orc = oracle_to(g, variant, mode, t_gpu)
        err = {k: abs(e_gpu[k] - e_orc[k]) for k in ("expl", "nash_conv", "br1", "br2", "value")}
        err.update({"iterations": t_gpu, "gpu_expl": e_gpu["expl"], "oracle_expl": e_orc["expl"]})
        log(f"[bench] all-core oracle ({th} threads): {t_gpu} it in {el:.1f}s; expl gpu "
            f"{e_gpu['expl']:.6g} oracle {e_orc['expl']:.6g} |d| {err['expl']:.2e}")
        n1, el1, _ = oracle_sample(g, variant, mode, args.cpu_budget, parallel=False)
        log(f"[bench] single-threaded oracle: {n1} it in {el1:.1f}s")
        cpu = {"value": t_gpu / el, "unit": "iter/s", "cores": th, "kind": "oracle",
               "sample": f"{t_gpu} iterations of the same workload ({args.config}, {variant}, "
                         f"{mode}, from t=0) by the all-core FP64 C oracle (OpenMP build, "
                         f"{th} threads), {el:.1f}s",
               "single_thread": {"value": n1 / el1, "unit": "iter/s", "cores": 1,
                                 "sample": f"{n1} iterations by the plain build, {el1:.1f}s"},
               "host": host_cpu()}

    fp64 = None
    if args.config == "cfg3" and precision != "fp64" and not args.no_fp64:
        s64, r64 = solver_line(torch, cfr, g, "fp64", variant, mode, args.steps, args.warmup,
                               tune=not args.no_tune)
        s64.close()
        w64 = r64["dominant"]
        fp64 = {"iters_per_s": r64["iters_per_s"], "ms_per_step": r64["ms_per_step"],
                "ms_mean": r64["timing"]["mean_ms"], "ms_sem": r64["timing"]["sem_ms"],
                "ms_median": r64["timing"]["median_ms"], "tiling": r64["tiling"],
                "dominant_kernel": r64["products"][w64]["kernel"],
                "dominant_us": r64["kernel_ms"] * 1e3,
                "dominant_frac": r64["kernel_bytes"] / (r64["kernel_ms"] * 1e-3) / 1e9 /
                HBM_PEAK_GBS,
                "iteration_hbm_frac": r64["iteration_hbm_frac"]}
        log(f"[bench] fp64: {r64['iters_per_s']:.0f} it/s ({r64['ms_per_step']:.4f} ms), "
            f"dominant {fp64['dominant_kernel']} {fp64['dominant_us']:.1f} us "
            f"({fp64['dominant_frac']:.3f} of 8 TB/s)")

    out = {
        "metric": "CFR iters/s + HBM GB/s at 1e8 nnz",
        "value": rec["iters_per_s"],
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[precision],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {g.name}, {variant}, {mode}, {precision}",
                   "nnz": g.nnz, "n_seq": list(g.n_seq), "terminals": g.tree.n_terminals
                   if g.tree is not None else None, "graph": not args.no_graph,
                   "tiling": rec["tiling"], "tuned": rec["tuned"]},
        "ms_per_step_regions": {"mean": tm["mean_ms"], "sem": tm["sem_ms"],
                                "median": tm["median_ms"], "regions": tm["regions"]},
        "nnz_iters_per_s": g.nnz * rec["iters_per_s"],
        "streamed_gb_per_iter": rec["streamed_gb_per_iter"],
        "iteration_gbs": rec["iteration_gbs"],
        "iteration_hbm_frac": rec["iteration_hbm_frac"],
        "algorithmic_gb_per_iter": rec["algorithmic_gb_per_iter"],
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_us": ms_l * 1e3,
                     "bytes_per_launch": fmt_by, "stream_form": rec["tiling"]["vec"][w],
                     "element_bytes_per_launch": el_by,
                     "element_equiv_gbs": el_by / (ms_l * 1e-3) / 1e9,
                     "basis": "achieved/frac: the bytes the launch's stream form reads and "
                              "writes (quads: one index and four values per quad; row "
                              "pointers; the gathered vector once; the output once) per "
                              "kernel-only HIP-event time; element_equiv_gbs: the element "
                              "stream (index and value per nonzero) over the same time, "
                              "which quads do not read"},
        "cpu_baseline": cpu,
        "oracle_error": err,
        "expl_average": e_gpu["expl"],
        "fp64": fp64,
    }
    if args.config == "cfg3" and not args.no_batch:
        out["batch"] = batch_record(args, torch)
        if not args.no_serve:
            out["serve"] = serve_record(args, torch, [float(args.serve_rate)])
    print(json.dumps(out), flush=True)


def batch_record(args, torch) -> dict:
    """Many games of uneven size solved together (one batch, every launch
    covering all games still iterating) against the same games solved one
    at a time on the same GPU with the same solver and stopping rule, and
    against plain (vanilla) CFR one at a time.  solves/s counts the games
    that reached their target."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import gamegen as gg
    import paper_2605_14277_amd as cfr
    from paper_2605_14277_amd import serve

    n, K, max_it = args.games, args.check_every, args.max_iterations
    variant = args.batch_variant
    precision = "fp32_acc64"
    t0 = time.perf_counter()
    specs = gg.batch_specs(n)
    games = gg.batch_games(specs, workers=args.workers)
    gen_s = time.perf_counter() - t0
    targets = [args.rel_target * gg.payoff_range(g) for g in games]
    nnz = np.array([g.nnz for g in games])
    log(f"[batch] {n} games generated in {gen_s:.1f}s: nnz total {nnz.sum():.3e}, "
        f"median {np.median(nnz):.3e}, max {nnz.max():.3e}")
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=args.workers) as ex:
        prepared = list(ex.map(lambda g: serve.Prepared(g, precision), games))
    prep_s = time.perf_counter() - t0
    units = np.sum([p.units for p in prepared], axis=0)
    b = cfr.Batch([units[0], units[1]], [units[2], units[3]], int(units[4]), max_games=n,
                  precision=precision, mode="alternating", check_every=K,
                  use_graph=not args.no_graph)
    t0 = time.perf_counter()
    ids = [serve.add_prepared(b, p, variant, target=tg, max_iterations=max_it)
           for p, tg in zip(prepared, targets)]
    torch.cuda.synchronize()
    add_s = time.perf_counter() - t0
    for p in prepared:
        p.close()
    log(f"[batch] workspace {b.workspace_bytes / 1e9:.1f} GB; prepared in {prep_s:.1f}s, "
        f"added in {add_s:.1f}s")
    t0 = time.perf_counter()
    tiling = b.tune(reps=args.tune_reps)
    tune_s = time.perf_counter() - t0
    log(f"[batch] tuner chose {tiling} in {tune_s:.1f}s")

    torch.cuda.synchronize()
    finish = {}
    t0 = time.perf_counter()
    while True:
        left = b.run(K)
        now = time.perf_counter() - t0
        for gid in ids:
            if gid not in finish and b.status(gid)["state"] == "done":
                finish[gid] = now
        if left == 0:
            break
    wall = time.perf_counter() - t0
    st = [b.status(gid) for gid in ids]
    iters = np.array([x["iterations"] for x in st])
    reached = int(sum(x["reached_target"] for x in st))
    done_t = np.array([finish[gid] for gid in ids])
    log(f"[batch] batch: {n} games in {wall:.2f}s, {reached} reached the target "
        f"({reached / wall:.2f} solves/s); iterations median {np.median(iters):.0f} "
        f"max {iters.max()}")
    b.close()

    # one game at a time: same games, variant, stopping rule, precision, tiling
    idx = list(range(0, n, max(1, args.baseline_stride)))
    seq_s, seq_reached, same = 0.0, 0, True
    for i in idx:
        el, it, e = solve_alone(cfr, games[i], variant, targets[i], max_it, K, precision, tiling)
        seq_s += el
        seq_reached += int(e <= targets[i])
        same = same and it == iters[i]
    scale = n / len(idx)
    log(f"[batch] one at a time: {len(idx)} games in {seq_s:.2f}s, {seq_reached} reached "
        f"-> {seq_reached * scale / (seq_s * scale):.2f} solves/s (same iteration counts: {same})")
    plain = None
    if args.plain_stride > 0:
        pidx = list(range(0, n, args.plain_stride))
        ps, pr = 0.0, 0
        for i in pidx:
            el, it, e = solve_alone(cfr, games[i], "vanilla", targets[i], max_it, K, precision,
                                    tiling)
            ps += el
            pr += int(e <= targets[i])
        plain = {"games": len(pidx), "seconds": ps, "reached_target": pr,
                 "solves_per_s": pr / ps, "valid": pr == len(pidx), "variant": "vanilla",
                 "max_iterations": max_it}
        log(f"[batch] plain CFR one at a time: {len(pidx)} games in {ps:.2f}s, {pr} reached "
            f"-> {pr / ps:.2f} solves/s")
    batched = reached / wall
    alone = seq_reached / seq_s
    return {"workload": f"{n} games (signals U{{3..32}}, terminals log-uniform 1e2..1e5, depth "
                        f"4..10, U[-1,1] payoffs), {variant}, alternating, {precision}, target "
                        f"{args.rel_target:g} of the payoff range or {max_it} iterations, "
                        f"checks every {K}",
            "games": n, "nnz_total": int(nnz.sum()), "nnz_median": float(np.median(nnz)),
            "nnz_max": int(nnz.max()),
            "solves_per_s": batched, "seconds": wall, "reached_target": reached,
            "valid": reached == n,
            "iterations_median": float(np.median(iters)), "iterations_max": int(iters.max()),
            "finish_p50_s": float(np.percentile(done_t, 50)),
            "finish_p99_s": float(np.percentile(done_t, 99)), "tiling": tiling,
            "one_at_a_time": {"games_timed": len(idx), "seconds_timed": seq_s,
                              "reached_target": seq_reached, "solves_per_s": alone,
                              "valid": seq_reached == len(idx), "same_iterations": bool(same)},
            "speedup_vs_one_at_a_time": batched / alone,
            "plain_cfr_one_at_a_time": plain,
            "speedup_vs_plain_cfr": batched / plain["solves_per_s"] if plain and
            plain["solves_per_s"] > 0 else None,
            "setup_s": {"generate": gen_s, "prepare": prep_s, "add": add_s, "tune": tune_s}}


def serve_record(args, torch, rates) -> dict:
    """Requests arriving as Poisson streams, served with continuous batching
    (games join a batch at check boundaries while others iterate; small games
    in a batch of their own on another stream), against one-at-a-time FIFO
    service of the same requests with the same solver."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import gamegen as gg
    from paper_2605_14277_amd import serve
    import paper_2605_14277_amd as cfr

    K, max_it, precision = args.check_every, args.max_iterations, "fp32_acc64"
    t0 = time.perf_counter()
    pool_games = gg.batch_games(gg.batch_specs(args.pool), workers=args.workers)
    gen_s = time.perf_counter() - t0
    ranges = [gg.payoff_range(g) for g in pool_games]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=args.workers) as ex:
        prepared = list(ex.map(lambda g: serve.Prepared(g, precision), pool_games))
    prep_s = time.perf_counter() - t0
    nnz = np.array([g.nnz for g in pool_games])
    log(f"[serve] pool of {args.pool} games (nnz median {np.median(nnz):.3e}, max "
        f"{nnz.max():.3e}) generated in {gen_s:.1f}s, prepared in {prep_s:.1f}s")
    rng = np.random.Generator(np.random.PCG64(5000))
    n = args.requests
    which = rng.integers(0, args.pool, size=n)
    rel = rng.choice([1e-2, 1e-3], size=n)
    var = rng.choice(["cfr+", "dcfr"], size=n)
    gaps = rng.exponential(1.0, size=n)
    budget = int(args.budget_gb * 1e9)
    tiling = parse_tiling(args.serve_tiling)
    quads = 3 in tiling["vec"]
    # with quads, part of the budget goes to the quad stores (about 0.3 quads
    # per nonzero for the games of this distribution, per product)
    qshare = 0.55 if quads else 1.0
    vb = 4
    # two lanes: games of at most small_nnz nonzeros in a batch of their own
    # (a share of the budget sized by the mix of such games), the rest in
    # the main batch
    small_units = [p.units for p in prepared if p.units[4] <= args.small_nnz]
    small = None
    main_budget = budget
    if args.serve_lanes == 2 and small_units:
        sb = int(budget * args.small_share)
        smix = np.sum(small_units, axis=0) / len(small_units)
        s_seq, s_inf, s_nz = serve.capacities_for_bytes(int(sb * qshare), smix, args.max_games,
                                                        precision)
        small = {"seq_capacity": s_seq, "inf_capacity": s_inf, "nnz_capacity": s_nz,
                 "max_games": args.max_games, "nnz_limit": args.small_nnz,
                 "quad_capacity": int(0.3 * s_nz) if quads else 0}
        main_budget = budget - sb
        log(f"[serve] small-game lane (at most {args.small_nnz:.0e} nonzeros, "
            f"{len(small_units)} of the {args.pool} pool games): {sb / 1e9:.0f} GB -> "
            f"capacity {s_nz:.3e} nonzeros, {args.max_games} slots, a stream of its own")
    mix = np.sum([p.units for p in prepared], axis=0) / args.pool
    seq, inf, nz = serve.capacities_for_bytes(int(main_budget * qshare), mix, args.max_games,
                                              precision)
    qcap = int(0.3 * nz) if quads else 0
    log(f"[serve] device budget {budget / 1e9:.0f} GB; main lane {main_budget / 1e9:.0f} GB -> "
        f"capacity {nz:.3e} nonzeros, {args.max_games} slots"
        + (f", {qcap:.3e} quads per product ({2 * qcap * (4 + 4 * vb) / 1e9:.0f} GB)"
           if quads else "") + f"; product tiling {tiling}")
    if quads:
        with ThreadPoolExecutor(max_workers=args.workers) as ex:
            list(ex.map(lambda p: p.prepare_quads(tiling["perm"]), prepared))
    # one game at a time: each distinct request solved alone once
    service = {}
    t0 = time.perf_counter()
    for k in range(n):
        key = (int(which[k]), str(var[k]), float(rel[k]))
        if key not in service:
            el, it, e = solve_alone(cfr, pool_games[key[0]], key[1], key[2] * ranges[key[0]],
                                    max_it, K, precision, tiling)
            service[key] = (el, it)
    log(f"[serve] {len(service)} distinct requests solved alone in "
        f"{time.perf_counter() - t0:.1f}s")
    svc = np.array([service[(int(which[k]), str(var[k]), float(rel[k]))][0] for k in range(n)])

    per_rate = {}
    for rate in rates:
        arrivals = np.cumsum(gaps / rate)
        reqs = [{"arrival": float(arrivals[k]), "prepared": int(which[k]), "variant": str(var[k]),
                 "target": float(rel[k] * ranges[which[k]]), "max_iterations": max_it}
                for k in range(n)]
        srv = serve.Server(seq, inf, nz, max_games=args.max_games, precision=precision,
                           check_every=K, tiling=tiling, quad_capacity=qcap, small=small,
                           solo=args.solo if small else 0, admit_after=args.admit_after)
        out = srv.serve(reqs, prepared=prepared)
        host = srv.host_stats()
        srv.close()
        done = [o for o in out if o["state"] == "done"]
        lat = np.array([o["latency"] for o in done])
        span = max(o["finished"] for o in out) - float(arrivals[0])
        same = all(out[k]["iterations"] == service[(int(which[k]), str(var[k]),
                                                    float(rel[k]))][1] for k in range(n))
        seq_lat = serve.sequential_latencies(arrivals, svc)
        seq_span = float(np.max(arrivals + seq_lat)) - float(arrivals[0])
        per_rate[str(int(rate))] = {
            "served": {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                       "solves_per_s": len(done) / span,
                       "reached_target": int(sum(o["reached_target"] for o in done)),
                       "rejected": n - len(done),
                       "same_iterations_as_alone": bool(same), "host": host},
            "one_at_a_time": {"p50_s": float(np.percentile(seq_lat, 50)),
                              "p99_s": float(np.percentile(seq_lat, 99)),
                              "solves_per_s": n / seq_span},
        }
        log(f"[serve] {rate:g} req/s: served p50 {np.percentile(lat, 50) * 1e3:.0f} ms, p99 "
            f"{np.percentile(lat, 99) * 1e3:.0f} ms, {len(done) / span:.1f} solves/s; one at a "
            f"time p50 {np.percentile(seq_lat, 50) * 1e3:.0f} ms, p99 "
            f"{np.percentile(seq_lat, 99) * 1e3:.0f} ms, {n / seq_span:.1f} solves/s")
    for p in prepared:
        p.close()
    return {"workload": f"{n} requests per rate, Poisson arrivals, games from a pool of "
                        f"{args.pool} of the batch distribution, CFR+ or DCFR, target 1e-2 or "
                        f"1e-3 of the payoff range or {max_it} iterations, checks every {K}, "
                        f"{args.budget_gb:g} GB device budget, {args.max_games} slots"
                        + (f" per lane; games of at most {args.small_nnz:.0e} nonzeros in a "
                           f"lane of their own ({args.small_share:g} of the budget); the other "
                           f"lane holds {args.solo} game(s) and admits more once a request has "
                           f"waited {args.admit_after:g} s" if small else ""),
            "lanes": 2 if small else 1, "tiling": tiling, "rates": per_rate,
            "pool": {"games": args.pool, "nnz_median": float(np.median(nnz)),
                     "nnz_max": int(nnz.max()), "generate_s": gen_s, "prepare_s": prep_s}}


def bench_batched(args, torch):
    rec = batch_record(args, torch)
    out = {"metric": "batched solves/s to expl 1e-3 of the payoff range",
           "value": rec["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": rec["iterations_max"], "warmup": 0,
           "ms_per_step": rec["seconds"] * 1e3 / max(1, rec["iterations_max"]),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64acc", "data": "synthetic",
           "config": {"workload": rec["workload"], "games": rec["games"],
                      "nnz_total": rec["nnz_total"]},
           "batch": rec}
    print(json.dumps(out), flush=True)


def bench_serving(args, torch):
    rates = [float(r) for r in args.rates.split(",")]
    rec = serve_record(args, torch, rates)
    mid = rec["rates"][str(int(rates[len(rates) // 2]))]
    out = {"metric": "served solves/s and p50/p99 latency to expl 1e-2/1e-3 of the payoff range",
           "value": mid["served"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": args.requests, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64acc", "data": "synthetic",
           "config": {"workload": rec["workload"], "value_rate": rates[len(rates) // 2]},
           "serve": rec}
    print(json.dumps(out), flush=True)


# the size sweep: (terminals, depth, terminal range accepted) of the public
# tree, and the signals per player
SIZE_TREES = ((1e3, 6, 900, 1100), (1e4, 8, 9000, 11000), (1e5, 10, 96000, 106000))
SIZE_SIGNALS = (8, 16, 32)


def bench_sizes(args, torch):
    """Iterations/s against game size: the large game's generator at about
    1e3, 1e4 and 1e5 terminals with 8, 16 and 32 signals (5e4 to 1e8 payoff
    nonzeros), DCFR(1.5, 0, 2) alternating, FP32 values with FP64
    accumulators, autotuned tiling, graph replay; beside each the
    single-threaded FP64 oracle on a bounded sample of the same solve."""
    import gamegen as gg
    import paper_2605_14277_amd as cfr

    variant, mode, precision = "dcfr", "alternating", args.precision or "fp32_acc64"
    vbytes = 8 if precision == "fp64" else 4
    budget = min(args.cpu_budget, 3.0)
    rows = []
    for T, depth, lo, hi in SIZE_TREES:
        for S in SIZE_SIGNALS:
            g = gg.showdown_sized(S, depth, lo, hi, f"sizes-T{T:.0e}-S{S}")
            s = cfr.Solver(g, precision=precision, device=0)
            tiling = s.tune(reps=5)
            s.step(args.warmup, variant, mode)
            torch.cuda.synchronize()
            # about 0.3 s of timed iterations
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.step(20, variant, mode)
            e1.record(s.stream)
            torch.cuda.synchronize()
            k = int(min(5000, max(50, 0.3 / max(e0.elapsed_time(e1) / 20 * 1e-3, 1e-9))))
            e0.record(s.stream)
            s.step(k, variant, mode)
            e1.record(s.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / k
            s.kernel_timing(True)
            s.step(20, variant, mode)
            torch.cuda.synchronize()
            prod = []
            for w in (0, 1):
                n, tot, _ = s.kernel_stats(w)
                rr, cc = g.n_seq[w], g.n_seq[1 - w]
                by = float(g.nnz * (4 + vbytes) + 4 * (rr + 1) + vbytes * (cc + rr))
                prod.append((tot / n, by))
            s.kernel_timing(False)
            slow_ms, slow_by = max(prod)
            s.close()
            n_cpu, el, _ = oracle_sample(g, variant, mode, budget, parallel=False)
            row = {"terminals": g.tree.n_terminals, "S": S, "depth": depth,
                   "nnz": int(g.nnz), "n_seq": [int(v) for v in g.n_seq],
                   "gpu_iters_per_s": 1e3 / ms, "nnz_iters_per_s": g.nnz * 1e3 / ms,
                   "product_us": slow_ms * 1e3,
                   "product_gbs": slow_by / (slow_ms * 1e-3) / 1e9,
                   "cpu_iters_per_s": n_cpu / el, "speedup": (1e3 / ms) / (n_cpu / el),
                   "tiling": tiling}
            rows.append(row)
            log(f"[sizes] T~{T:.0e} S={S:2d}: nnz {g.nnz:.3e}, GPU {row['gpu_iters_per_s']:9.0f} it/s "
                f"({row['nnz_iters_per_s']:.2e} nnz*it/s, slower product {row['product_us']:.1f} us "
                f"= {row['product_gbs']:.0f} GB/s), oracle {row['cpu_iters_per_s']:9.1f} it/s, "
                f"x{row['speedup']:.1f}")
    out = {"metric": "GPU iterations/s over the single-threaded CPU oracle's, by game size",
           "value": rows[-1]["speedup"], "unit": "x", "n_gpus": 1, "steps": None,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64acc" if precision == "fp32_acc64" else precision, "data": "synthetic",
           "config": {"workload": "large-game generator at ~1e3/1e4/1e5 terminals x 8/16/32 "
                                  "signals, dcfr, alternating", "cpu_budget_s": budget,
                      "cpu_cores": 1},
           "sizes": rows}
    print(json.dumps(out), flush=True)




def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="cfg3",
                    choices=["cfg1", "cfg2", "cfg2_d8", "cfg3", "batch", "serve", "sizes"])
    ap.add_argument("--games", type=int, default=256, help="batch: number of games")
    ap.add_argument("--batch-variant", default="pcfr+", help="batch: regret minimiser")
    ap.add_argument("--check-every", type=int, default=10, help="batch: iterations per check")
    ap.add_argument("--max-iterations", type=int, default=2000, help="batch: iteration limit")
    ap.add_argument("--rel-target", type=float, default=1e-3,
                    help="batch: exploitability target as a fraction of the payoff range")
    ap.add_argument("--tune-reps", type=int, default=3, help="batch: autotuner launches each")
    ap.add_argument("--serve-tiling", default="16,16:256,256:2,2:1,1",
                    help="serve: product tiling of the serving loop and of the one-at-a-time "
                         "solves (stream form 2: no per-game quad copy to build at admission)")
    ap.add_argument("--baseline-stride", type=int, default=1,
                    help="batch: solve every k-th game alone for the one-at-a-time rate")
    ap.add_argument("--rates", default="50,200,800", help="serve: arrival rates (req/s)")
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="arrival rate of the serving record in the default line")
    ap.add_argument("--requests", type=int, default=128, help="serve: requests per rate")
    ap.add_argument("--pool", type=int, default=64, help="serve: distinct games")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: device budget")
    ap.add_argument("--serve-lanes", type=int, default=2, choices=[1, 2],
                    help="serve: 2 = games of at most --small-nnz nonzeros in a batch of their "
                         "own on a stream of their own")
    ap.add_argument("--small-nnz", type=float, default=1e7, help="serve: small-game lane limit")
    ap.add_argument("--small-share", type=float, default=0.25,
                    help="serve: share of the device budget for the small-game lane")
    ap.add_argument("--solo", type=int, default=1,
                    help="serve: games the main lane holds before admitting another beside "
                         "them only after --admit-after seconds of waiting (0: always admit)")
    ap.add_argument("--admit-after", type=float, default=0.05,
                    help="serve: the wait that lets a request join a busy main lane")
    ap.add_argument("--max-games", type=int, default=256, help="serve: game slots")
    ap.add_argument("--plain-stride", type=int, default=16,
                    help="batch: also solve every k-th game alone with vanilla CFR (0: skip)")
    ap.add_argument("--workers", type=int, default=16, help="host threads for game generation")
    ap.add_argument("--variant", default=None)
    ap.add_argument("--mode", default=None)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--spmv-order", default="default", choices=["default", "sequential", "parallel"])
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default product tiling instead of running the autotuner")
    ap.add_argument("--tiling", default=None,
                    help="fixed product tiling 'items_Ay,items_ATx:rows_Ay,rows_ATx:vec_Ay,vec_ATx:"
                         "perm_Ay,perm_ATx:xcd_Ay,xcd_ATx' (skips the autotuner)")
    ap.add_argument("--error-iterations", type=int, default=1000,
                    help="iterations at which the GPU result is compared with the all-core "
                         "oracle (the configs' horizon; the solver continues untimed to it)")
    ap.add_argument("--cpu-budget", type=float, default=10.0,
                    help="seconds of single-threaded oracle time for its sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="default line: skip the FP64 record")
    ap.add_argument("--no-batch", action="store_true",
                    help="default line: skip the batch and serving records")
    ap.add_argument("--no-serve", action="store_true", help="default line: skip the serving record")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain device copy of 1.6 GiB (the HBM reference that "
                         "scales the FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        log("bench.py measures one GPU only: the solver runs on a single GPU and "
            "has no multi-GPU path. Run with --gpus 1.")
        sys.exit(2)

    import torch

    if args.copy_probe:
        copy_probe(torch)
        return
    if args.config == "batch":
        bench_batched(args, torch)
        return
    if args.config == "serve":
        bench_serving(args, torch)
        return
    if args.config == "sizes":
        bench_sizes(args, torch)
        return
    bench_large(args, torch)


if __name__ == "__main__":
    main()
