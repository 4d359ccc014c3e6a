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
import re
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


def algorithmic_bytes_per_iteration(g, vbytes: int, abytes: int, predictive: bool,
                                    product_bytes=None) -> float:
    """Bytes one iteration must move at minimum: both payoff streams (index +
    value, or in stream form 3 each quad's index and four values), row
    pointers, each gathered vector once and each product's output once, and
    per sequence: regret and average read-modify-write in the accumulator
    type, the utility read, the behavioural strategy written and read, the
    strategy written, one int32 of treeplex structure (plus the prediction's
    read and write for predictive variants).  product_bytes: the two
    products' bytes per launch as the library counts them for the stream
    form in use (the element-stream formula when None)."""
    n1, n2 = g.n_seq
    if product_bytes is None:
        payoff = 2 * g.nnz * (4 + vbytes) + 4 * (n1 + 1) + 4 * (n2 + 1)
        vectors = 2 * (n1 + n2) * vbytes
        products = payoff + vectors
    else:
        products = sum(product_bytes)
    per_seq = 4 * abytes + 4 * vbytes + 4 + (2 * abytes if predictive else 0)
    return float(products + (n1 + n2) * per_seq)


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


def parse_tiling(text: str) -> dict:
    """'items_Ay,items_ATx:rows_Ay,rows_ATx[:vec_Ay,vec_ATx[:perm_Ay,perm_ATx[:xcd_Ay,xcd_ATx]]]'."""
    parts = text.split(":")
    return {"items": [int(v) for v in parts[0].split(",")],
            "rows": [int(v) for v in parts[1].split(",")],
            "vec": [int(v) for v in parts[2].split(",")] if len(parts) > 2 else [1, 1],
            "perm": [int(v) for v in parts[3].split(",")] if len(parts) > 3 else [0, 0],
            "xcd": [int(v) for v in parts[4].split(",")] if len(parts) > 4 else [1, 1]}


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


def bench_batched(args, torch):
    """Many games of uneven size solved together (one batch, every launch
    covering all games still iterating) against the same games solved one at
    a time on the same GPU with the same stopping rule."""
    import numpy as np

    import gamegen as gg
    import paper_2605_14277_amd as cfr

    n, K, max_it = args.games, args.check_every, args.max_iterations
    variant, precision = args.variant or "pcfr+", args.precision or "fp32_acc64"
    t0 = time.perf_counter()
    specs = gg.batch_specs(n)
    games = [gg.batch_game(sp) for sp in specs]
    gen_s = time.perf_counter() - t0
    targets = [args.rel_target * gg.payoff_range(g) for g in games]
    nnz = np.array([g.nnz for g in games])
    log(f"[bench] {n} games generated in {gen_s:.1f}s: nnz total {nnz.sum():.3e}, "
        f"median {np.median(nnz):.3e}, max {nnz.max():.3e}")
    torch.cuda.set_device(0)
    units = np.sum([cfr.Batch.game_size(g) for g in games], axis=0)
    b = cfr.Batch([units[0], units[1]], [units[2], units[3]], int(units[4]), max_games=n,
                  precision=precision, mode="alternating", check_every=K,
                  use_graph=not args.no_graph)
    t0 = time.perf_counter()
    ids = [b.add(g, variant, target=tg, max_iterations=max_it) for g, tg in zip(games, targets)]
    torch.cuda.synchronize()
    add_s = time.perf_counter() - t0
    log(f"[bench] batch workspace {b.workspace_bytes / 1e9:.1f} GB, games added in {add_s:.1f}s")
    t0 = time.perf_counter()
    tiling = b.tune(reps=args.tune_reps)
    tune_s = time.perf_counter() - t0
    log(f"[bench] tuner chose {tiling} in {tune_s:.1f}s")

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
    log(f"[bench] batch: {n} games in {wall:.2f}s ({n / wall:.2f} solves/s); {reached} reached "
        f"the target, iterations median {np.median(iters):.0f} max {iters.max()}")
    b.close()

    # one game at a time, same games, variant, stopping rule and precision
    idx = list(range(0, n, max(1, args.baseline_stride)))
    seq_s, seq_it, seq_e = 0.0, [], []
    for i in idx:
        el, it, e = solve_alone(cfr, games[i], variant, targets[i], max_it, K, precision, tiling)
        seq_s += el
        seq_it.append(it)
        seq_e.append(e)
    scale = n / len(idx)
    seq_total = seq_s * scale
    same_iters = all(seq_it[j] == iters[i] for j, i in enumerate(idx))
    log(f"[bench] one at a time: {len(idx)} games in {seq_s:.2f}s -> {n / seq_total:.2f} solves/s "
        f"(same iteration counts as in the batch: {same_iters})")
    plain = None
    if args.plain_stride > 0:
        pidx = list(range(0, n, args.plain_stride))
        ps, pr = 0.0, 0
        for i in pidx:
            el, it, e = solve_alone(cfr, games[i], "vanilla", targets[i], max_it, K, "fp32_acc64",
                                    tiling)
            ps += el
            pr += int(e <= targets[i])
        plain = {"games": len(pidx), "seconds": ps, "solves_per_s": len(pidx) / ps,
                 "reached_target": pr, "variant": "vanilla", "max_iterations": max_it}
        log(f"[bench] plain CFR one at a time: {len(pidx)} games in {ps:.2f}s, {pr} reached")

    out = {
        "metric": "batched solves/s to expl 1e-3 of the payoff range",
        "value": n / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": int(iters.max()),
        "warmup": 0,
        "ms_per_step": wall * 1e3 / max(1, int(iters.max())),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_acc64": "f32+f64acc"}[precision],
        "data": "synthetic",
        "config": {"workload": f"batch of {n} games, {variant}, alternating, {precision}, "
                               f"target {args.rel_target:g} of the payoff range or {max_it} "
                               f"iterations, checks every {K}",
                   "games": n, "nnz_total": int(nnz.sum()), "nnz_median": float(np.median(nnz)),
                   "nnz_max": int(nnz.max()), "graph": not args.no_graph},
        "batch": {"seconds": wall, "solves_per_s": n / wall, "reached_target": reached,
                  "iterations_median": float(np.median(iters)), "iterations_max": int(iters.max()),
                  "finish_p50_s": float(np.percentile(done_t, 50)),
                  "finish_p99_s": float(np.percentile(done_t, 99)), "tiling": tiling,
                  "tune_s": tune_s, "add_s": add_s, "generate_s": gen_s},
        "one_at_a_time": {"games_timed": len(idx), "seconds_timed": seq_s,
                          "solves_per_s": n / seq_total, "same_iterations": bool(same_iters)},
        "speedup_vs_one_at_a_time": seq_total / wall,
        "plain_cfr_one_at_a_time": plain,
    }
    print(json.dumps(out), flush=True)


def bench_serving(args, torch):
    """Requests arriving as Poisson streams, served with continuous batching
    (games join the batch at check boundaries while others iterate), against
    one-at-a-time FIFO service of the same requests with the same solver."""
    import numpy as np

    import gamegen as gg
    import paper_2605_14277_amd as cfr
    from paper_2605_14277_amd import serve

    K, max_it, precision = args.check_every, args.max_iterations, args.precision or "fp32_acc64"
    rates = [float(r) for r in args.rates.split(",")]
    t0 = time.perf_counter()
    pool_games = [gg.batch_game(sp) for sp in gg.batch_specs(args.pool)]
    gen_s = time.perf_counter() - t0
    ranges = [gg.payoff_range(g) for g in pool_games]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=16) as ex:
        prepared = list(ex.map(lambda g: serve.Prepared(g, precision), pool_games))
    prep_s = time.perf_counter() - t0
    nnz = np.array([g.nnz for g in pool_games])
    log(f"[bench] pool of {args.pool} games (nnz median {np.median(nnz):.3e}, max {nnz.max():.3e}) "
        f"generated in {gen_s:.1f}s, prepared in {prep_s:.1f}s")
    rng = np.random.Generator(np.random.PCG64(5000))
    n = args.requests
    which = rng.integers(0, args.pool, size=n)
    rel = rng.choice([1e-2, 1e-3], size=n)
    var = rng.choice(["cfr+", "dcfr"], size=n)
    gaps = rng.exponential(1.0, size=n)
    budget = int(args.budget_gb * 1e9)
    mix = np.sum([p.units for p in prepared], axis=0) / args.pool
    tiling = parse_tiling(args.serve_tiling)
    quads = 3 in tiling["vec"]
    # with quads, part of the budget goes to the quad stores (about 0.3 quads
    # per nonzero for the games of this distribution, per product)
    ws_budget = int(budget * (0.55 if quads else 1.0))
    seq, inf, nz = serve.capacities_for_bytes(ws_budget, mix, args.max_games, precision)
    vb = 8 if precision == "fp64" else 4
    qcap = int(0.3 * nz) if quads else 0
    log(f"[bench] device budget {budget / 1e9:.0f} GB -> capacity {nz:.3e} nonzeros, "
        f"{args.max_games} slots" + (f", {qcap:.3e} quads per product "
                                     f"({2 * qcap * (4 + 4 * vb) / 1e9:.0f} GB)" if quads else ""))

    # product tiling of the serving loop and of the one-at-a-time solves
    log(f"[bench] product tiling {tiling}")
    if 3 in tiling["vec"]:
        # quad copies built with the prepared games (host, worker threads)
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=16) as ex:
            list(ex.map(lambda p: p.prepare_quads(tiling["perm"]), prepared))
        log(f"[bench] quad copies of the pool built in {time.perf_counter() - t0:.1f}s")
    # one game at a time: each distinct request solved alone once
    service = {}
    t0 = time.perf_counter()
    for k in range(n):
        key = (int(which[k]), str(var[k]), float(rel[k]))
        if key not in service:
            el, it, e = solve_alone(cfr, pool_games[key[0]], key[1], key[2] * ranges[key[0]], max_it,
                                    K, precision, tiling)
            service[key] = (el, it)
    log(f"[bench] {len(service)} distinct requests solved alone in {time.perf_counter() - t0:.1f}s")
    svc = np.array([service[(int(which[k]), str(var[k]), float(rel[k]))][0] for k in range(n)])

    per_rate = {}
    for rate in rates:
        arrivals = np.cumsum(gaps / rate)
        reqs = [{"arrival": float(arrivals[k]), "prepared": int(which[k]), "variant": str(var[k]),
                 "target": float(rel[k] * ranges[which[k]]), "max_iterations": max_it}
                for k in range(n)]
        srv = serve.Server(seq, inf, nz, max_games=args.max_games, precision=precision,
                           check_every=K, tiling=tiling, quad_capacity=qcap)
        t0 = time.perf_counter()
        out = srv.serve(reqs, prepared=prepared)
        host = srv.batch.host_stats()
        srv.close()
        lat = np.array([o["latency"] for o in out])
        span = max(o["finished"] for o in out) - float(arrivals[0])
        same = all(out[k]["iterations"] == service[(int(which[k]), str(var[k]),
                                                    float(rel[k]))][1] for k in range(n))
        seq_lat = serve.sequential_latencies(arrivals, svc)
        seq_span = float(np.max(arrivals + seq_lat)) - float(arrivals[0])
        per_rate[str(int(rate))] = {
            "served": {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                       "solves_per_s": n / span, "reached_target": int(sum(o["reached_target"]
                                                                           for o in out)),
                       "same_iterations_as_alone": bool(same), "host": host},
            "one_at_a_time": {"p50_s": float(np.percentile(seq_lat, 50)),
                              "p99_s": float(np.percentile(seq_lat, 99)),
                              "solves_per_s": n / seq_span},
        }
        log("[bench]   host " + ", ".join(f"{k} {v['seconds'] * 1e3:.0f} ms/{v['calls']}"
                                        for k, v in host.items()))
        log(f"[bench] {rate:g} req/s: served p50 {np.percentile(lat, 50) * 1e3:.0f} ms, p99 "
            f"{np.percentile(lat, 99) * 1e3:.0f} ms, {n / span:.1f} solves/s; one at a time p50 "
            f"{np.percentile(seq_lat, 50) * 1e3:.0f} ms, p99 {np.percentile(seq_lat, 99) * 1e3:.0f} ms, "
            f"{n / seq_span:.1f} solves/s")
    for p in prepared:
        p.close()
    mid = per_rate[str(int(rates[len(rates) // 2]))]
    out = {
        "metric": "served solves/s and p50/p99 latency to expl 1e-2/1e-3 of the payoff range",
        "value": mid["served"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_acc64": "f32+f64acc"}[precision],
        "data": "synthetic",
        "config": {"workload": f"{n} requests per rate, Poisson arrivals at {args.rates} req/s, "
                               f"games from a pool of {args.pool} of the batch distribution, "
                               f"CFR+ or DCFR, target 1e-2 or 1e-3 of the payoff range or "
                               f"{max_it} iterations, checks every {K}, {args.budget_gb:g} GB "
                               f"device budget, {args.max_games} slots",
                   "value_rate": rates[len(rates) // 2], "tiling": tiling},
        "rates": per_rate,
        "pool": {"games": args.pool, "nnz_median": float(np.median(nnz)),
                 "nnz_max": int(nnz.max()), "generate_s": gen_s, "prepare_s": prep_s},
    }
    print(json.dumps(out), flush=True)


# Game sizes of the size sweep: (terminals, depth, terminal window)
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
            n_cpu, el = cpu_baseline(g, variant, mode, budget)
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
    ap.add_argument("--check-every", type=int, default=10, help="batch: iterations per check")
    ap.add_argument("--max-iterations", type=int, default=2000, help="batch: iteration limit")
    ap.add_argument("--rel-target", type=float, default=1e-3,
                    help="batch: exploitability target as a fraction of the payoff range")
    ap.add_argument("--tune-reps", type=int, default=5, help="batch: autotuner launches each")
    ap.add_argument("--serve-tiling", default="16,16:256,256:2,2:1,1",
                    help="serve: product tiling of the serving loop and of the one-at-a-time "
                         "solves (stream form 2: no per-game quad copy to build at admission)")
    ap.add_argument("--baseline-stride", type=int, default=1,
                    help="batch: solve every k-th game alone for the one-at-a-time rate")
    ap.add_argument("--rates", default="50,200,800", help="serve: arrival rates (req/s)")
    ap.add_argument("--requests", type=int, default=128, help="serve: requests per rate")
    ap.add_argument("--pool", type=int, default=64, help="serve: distinct games")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: device budget")
    ap.add_argument("--max-games", type=int, default=256, help="serve: game slots")
    ap.add_argument("--plain-stride", type=int, default=16,
                    help="batch: also solve every k-th game alone with vanilla CFR (0: skip)")
    ap.add_argument("--variant", default=None)
    ap.add_argument("--mode", default=None)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--spmv-order", default="default", choices=["default", "sequential", "parallel"])
    ap.add_argument("--sweep", action="store_true",
                    help="time both products under every tiling (stderr table, 'sweep' field)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default product tiling instead of running the autotuner")
    ap.add_argument("--tiling", default=None,
                    help="fixed product tiling 'items_Ay,items_ATx:rows_Ay,rows_ATx:vec_Ay,vec_ATx:"
                         "perm_Ay,perm_ATx:xcd_Ay,xcd_ATx' (skips the autotuner)")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    sweep = None
    if args.sweep:
        sweep = []
        s.step(3, variant, mode)
        for perm in (0, 1):
            for vec in (0, 1, 2, 3):
                for items in ((8, 16) if vec == 3 else (4, 8, 16)):
                    for rows in (64, 128, 256):
                        s.tiling = {"items": [items, items], "rows": [rows, rows],
                                    "vec": [vec, vec], "perm": [perm, perm]}
                        s.kernel_timing(True)
                        s.step(20, variant, mode)
                        us = []
                        for k in (0, 1):
                            n, tot, _ = s.kernel_stats(k)
                            us.append(tot / n * 1e3)
                        s.kernel_timing(False)
                        sweep.append({"perm": perm, "vec": vec, "items": items, "rows": rows,
                                      "csr_us": us[0], "csc_us": us[1]})
                        log(f"[sweep] perm {perm} vec {vec} items {items:2d} rows {rows:3d}: "
                            f"A y {us[0]:7.1f} us, A^T x {us[1]:7.1f} us")
    tune_s = None
    if args.tiling:
        s.tiling = parse_tiling(args.tiling)
    elif not args.no_tune:
        t0 = time.perf_counter()
        s.tune(reps=10)
        tune_s = time.perf_counter() - t0
    tiling = s.tiling
    log(f"[bench] product tiling {tiling}" + (f" (autotuner, {tune_s:.1f}s)" if tune_s else ""))

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
    product_bytes = [st[3] for st in stats]
    stats.sort(reverse=True)
    tot, kname, nl, by_format = stats[0]
    avg_ms = tot / nl
    digest = kernel_source_digest()
    traffic = measured_traffic(kname, digest, tiling)
    e = s.exploitability("average")

    vbytes = 8 if precision == "fp64" else 4
    abytes = 4 if precision == "fp32" else 8
    # algorithmic bytes: each nonzero's index and value (the element stream),
    # the row pointers, the gathered vector once and the output once, for
    # every stream form; the bytes the launch's own format moves (fewer with
    # quads) are reported beside them
    alg = algorithmic_bytes_per_iteration(g, vbytes, abytes, variant in ("pcfr+", "pcfr"))
    alg_format = algorithmic_bytes_per_iteration(g, vbytes, abytes, variant in ("pcfr+", "pcfr"),
                                                 product_bytes)
    w = 0 if kname == "spmv_csr" else 1
    n_rows, n_cols = g.n_seq[w], g.n_seq[1 - w]
    by = float(g.nnz * (4 + vbytes) + 4 * (n_rows + 1) + vbytes * (n_cols + n_rows))
    achieved = by / (avg_ms * 1e-3) / 1e9
    format_gbs = by_format / (avg_ms * 1e-3) / 1e9
    log(f"[bench] {kname}: {nl} launches, {avg_ms * 1e3:.1f} us avg, {achieved:.0f} GB/s "
        f"algorithmic ({format_gbs:.0f} GB/s of its own format's bytes); expl after "
        f"{s.iteration} it = {e['expl']:.4g}")

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
                   if g.tree is not None else None, "graph": not args.no_graph,
                   "tiling": tiling, "tuned": tune_s is not None},
        "nnz_iters_per_s": g.nnz * its,
        "algorithmic_gb_per_iter": alg / 1e9,
        "iteration_gbs": alg / (ms_per_step * 1e-3) / 1e9,
        "iteration_hbm_frac": alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "format_gb_per_iter": alg_format / 1e9,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_us": avg_ms * 1e3,
                     "bytes_per_launch": by, "stream_form": tiling["vec"][w],
                     "format_bytes_per_launch": by_format, "format_gbs": format_gbs,
                     "format_frac": format_gbs / HBM_PEAK_GBS,
                     "basis": "achieved/frac: element-stream bytes (index + value per nonzero, "
                              "row pointers, gathered vector, output) per kernel-only HIP-event "
                              "time; format_*: the bytes of the stream form the launch reads "
                              "(quads move fewer, so frac can pass 1 while format_frac < 1)"},
        "cpu_baseline": cpu,
        "expl_average": e["expl"],
    }
    if sweep is not None:
        out["sweep"] = sweep
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
