#!/usr/bin/env python3
"""Benchmark: KKT refactor + solve + FGMRES refinement units per second on the
70,000-bus-shaped synthetic grid (N = 665,000, 5,285,000 nonzeros), with p50/p99 latency,
the roofline position of the dominant kernel and the CPU-oracle baseline.

One step (unit) = kkt_refactor(K_t) followed by kkt_refine(b_t) (triangular solve plus FGMRES
refinement, as Algorithm 1 pairs every solve with refinement) that ends with a backward error
<= 1e-10, by default as one kkt_refactor_refine call (same results bit for bit), for t cycling through the 50-system sequence.  All values and
right-hand sides are resident in HBM before the timed region starts; analysis (host, once
per pattern) is timed separately.  One GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KKT refactor+solve/s at berr<=1e-10 (70k-bus-shaped); p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=250)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=2, help="workload index: 0 grid200, 1 grid25k, 2 grid70k")
    ap.add_argument("--cpu-sample", type=int, default=8, help="oracle units timed for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--approx-sweeps", type=int, default=0, metavar="K",
                    help="precondition the FGMRES steps with K Jacobi sweeps per triangle instead of exact solves")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default=None,
                    help="factor storage and refactorization precision (refinement stays FP64); default "
                         "fp64 for the grid workloads, fp32 for the batched one")
    ap.add_argument("--solve-mode", choices=("fixed", "ticket", "levels"), default="fixed",
                    help="triangular solves: persistent launch with fixed item order (default), with "
                         "ticket order, or one launch per level")
    ap.add_argument("--path", choices=("fused", "separate"), default="fused",
                    help="grid: kkt_refactor_refine (forward substitution beside the refactorization, "
                         "default) or kkt_refactor followed by kkt_refine; the results are the same bit for bit")
    ap.add_argument("--workload", choices=("grid", "batch", "serve"), default="grid",
                    help="grid: one grid's refactor+solve sequence (--config); batch: 64 systems of 8 "
                         "patterns (1k-10k buses) refactored together; serve: Poisson request streams "
                         "over 500/2k/10k/25k-bus patterns")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000",
                    help="serve: mean arrival rates (requests/s)")
    ap.add_argument("--requests", type=int, default=200, help="serve: requests per rate")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain MIB-MiB device copy (counter scaling reference) and exit")
    return ap.parse_args()


def coprime_stride(T):
    """A stride near 0.35 T that is coprime to T: the timed order t_i = i * stride mod T
    visits every system once per T units and spreads any prefix over the whole sequence
    (the D range widens along it)."""
    import math
    st = max(1, int(round(0.35 * T)))
    while math.gcd(st, T) != 1:
        st += 1
    return st


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count(), model


def nearest_rank(xs, p):
    s = sorted(xs)
    k = max(1, int(-(-p * len(s) // 100)))
    return s[k - 1]


def unit_bytes(n, nnz_a, nnz_lu, k, fb=8):
    """Compulsory HBM bytes of one unit with k FGMRES iterations (int32 indices, FP64
    values, factor values of fb bytes): the refactorization reads A's values and map and
    writes every factor value once, each solve reads the factor once, each residual/product
    reads A once, and Arnoldi step j reads and writes j+2 basis-length vectors."""
    b_ref = 12 * nnz_a + (fb + 4) * nnz_lu + 16 * n
    b_solve = (fb + 4) * nnz_lu + 48 * n
    b_spmv = 12 * nnz_a + 28 * n
    b_orth = sum(32 * (j + 2) * n + 8 * n for j in range(1, k + 1))
    return b_ref + (k + 2) * b_spmv + (k + 1) * b_solve + b_orth + 16 * n


def copy_calibration(mib):
    """Runs a plain device-to-device copy of MIB MiB five times: the reference against which
    the HBM byte counters (FETCH_SIZE, WRITE_SIZE) of the path's kernels are scaled."""
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = mib * (1 << 20) // 8
    x = torch.rand(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "copies": 5, "check": bool(torch.equal(x, y))}))


def kernel_source_digest():
    """SHA-256 of the kernel source, which ties a stored counter reading to the kernels it
    was taken from."""
    import hashlib
    path = os.path.join(ROOT, "paper_2302_08656_amd", "csrc", "kkt_kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch of KERNEL from the stored counter summary (FETCH_SIZE + WRITE_SIZE,
    scaled by the same counters on a plain copy), or None when there is no reading for this
    kernel or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "kkt_grid70k_hbm_counters.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
            if rec.get("kernel") == kernel and rec.get("source_sha256") == kernel_source_digest():
                return rec["bytes_per_launch"]
    return None


def bench_batch(args):
    """64 independent systems: 8 patterns (bus counts log-uniform in 1k-10k), 8 value sets
    each, one handle per system.  A step = one batched refactorization of all 64 handles
    (kkt_batch_refactor, graph replay) + the refinement of each to berr <= 1e-10.  Each
    pattern's schedule is autotuned once.  Baselines on the same 64 systems: the plain FP64
    path (one handle per pattern, refactor + refine one system after the other) and the
    same precision without batching."""
    import numpy as np
    import torch

    import kktgen
    import paper_2302_08656_amd as K

    prec = args.precision or "fp32"
    fp = K.FP32 if prec == "fp32" else K.FP64
    specs = kktgen.batch_specs()
    seqs = [kktgen.make_sequence(s) for s in specs]
    T = specs[0].steps
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    vals = [[torch.from_numpy(q.values(t)).to(dev) for t in range(T)] for q in seqs]
    rhs = [[torch.from_numpy(q.rhs(t)).to(dev) for t in range(T)] for q in seqs]
    t0 = time.perf_counter()
    tunings, tune_ms = [], []
    handles = []
    for p, q in enumerate(seqs):
        sk = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), factor_precision=fp).bind()
        choice, ms = sk.autotune(vals[p][0], reps=3)
        tunings.append(choice)
        tune_ms.append(ms)
        sk.close()
        for j in range(T):
            h = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), factor_precision=fp)
            h.set_tuning(**choice)
            handles.append((p, j, h.bind()))
    t_setup = time.perf_counter() - t0
    batch = K.KKTBatch([h for _, _, h in handles])
    xs = [torch.empty_like(rhs[p][0]) for p, _, _ in handles]

    def step(i):
        sel = [(p, (j + i) % T) for p, j, _ in handles]
        batch.refactor([vals[p][t] for p, t in sel])
        _, infos = batch.refine([rhs[p][t] for p, t in sel], xs)
        return infos

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    lat, iters, fails = [], [], 0
    t_start = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        infos = step(args.warmup + i)
        lat.append((time.perf_counter() - a) * 1e3)
        for inf in infos:
            iters.append(inf.iters)
            fails += int(inf.status != K.OK or not (inf.berr <= 1e-10))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    nsys = len(handles)
    value = (args.steps * nsys - fails) / elapsed
    # refactorization alone, batched: one graph replay for all 64
    torch.cuda.synchronize()
    a = time.perf_counter()
    for i in range(args.steps):
        sel = [(p, (j + i) % T) for p, j, _ in handles]
        batch.refactor([vals[p][t] for p, t in sel])
    torch.cuda.synchronize()
    batch_refactor_ms = (time.perf_counter() - a) * 1e3 / args.steps
    batch.close()

    def one_by_one(fp_, tuned):
        solvers = []
        for p, q in enumerate(seqs):
            sk = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), factor_precision=fp_)
            if tuned:
                sk.set_tuning(**tunings[p])
            solvers.append(sk.bind())
        x1 = [torch.empty_like(rhs[p][0]) for p in range(len(seqs))]
        for p, sk in enumerate(solvers):           # warm-up (graph recording)
            sk.refactor(vals[p][0])
            sk.refine(rhs[p][0], x1[p])
        torch.cuda.synchronize()
        n_ok, its = 0, []
        refac_ms = 0.0
        a = time.perf_counter()
        for i in range(args.steps):
            for p, j, _ in handles:
                t = (j + i) % T
                solvers[p].refactor(vals[p][t])
                _, inf = solvers[p].refine(rhs[p][t], x1[p])
                its.append(inf[0].iters)
                n_ok += int(inf[0].status == K.OK and inf[0].berr <= 1e-10)
        torch.cuda.synchronize()
        el = time.perf_counter() - a
        a = time.perf_counter()
        for p, j, _ in handles:
            solvers[p].refactor(vals[p][j])
        torch.cuda.synchronize()
        refac_ms = (time.perf_counter() - a) * 1e3
        for sk in solvers:
            sk.close()
        return {"value": round(n_ok / el, 3), "fgmres_iters_mean": round(float(np.mean(its)), 3),
                "refactor_ms_for_64": round(refac_ms, 3)}

    plain = one_by_one(K.FP64, False)
    same = one_by_one(fp, True)
    for _, _, h in handles:
        h.close()
    out = {
        "metric": "batched KKT refactor+solve/s at berr<=1e-10 (64 systems, 8 patterns, 1k-10k buses); p50/p99 step latency",
        "value": round(value, 3), "unit": "systems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64" if fp == K.FP32 else "f64", "data": "synthetic",
        "config": {"workload": "batch: " + ", ".join(f"{s.buses}-bus (N={q.n})" for s, q in zip(specs, seqs)) +
                               f"; {T} value sets each, 64 handles, one batched refactorization + 64 refinements per step",
                   "precision": ("FP32 factors, FP64 refinement" if fp == K.FP32 else "FP64"),
                   "tunings": tunings, "autotune_ms": [round(m, 4) for m in tune_ms],
                   "setup_s": round(t_setup, 2)},
        "p50_ms": round(nearest_rank(lat, 50), 4), "p99_ms": round(nearest_rank(lat, 99), 4),
        "failures": fails, "fgmres_iters_mean": round(float(np.mean(iters)), 3),
        "batched_refactor_ms_for_64": round(batch_refactor_ms, 3),
        "plain_fp64_one_by_one": plain,
        "same_precision_one_by_one": same,
    }
    print(json.dumps(out))


def bench_serve(args):
    """Serving: for each mean rate, a Poisson trace of requests (pattern drawn from 500/2k/
    10k/25k buses with probabilities 0.4/0.3/0.2/0.1, a value set, 1-4 right-hand sides)
    is submitted at its arrival times to the serving engine (FP32 factors, FP64 refinement,
    4 workers); latency = submit to completion.  The plain FP64 path is the same trace
    served by one worker with FP64 factors (one request after the other, as a caller of
    kkt_refactor/kkt_refine would)."""
    import numpy as np
    import torch

    import kktgen
    import paper_2302_08656_amd as K

    prec = args.precision or "fp32"
    fp = K.FP32 if prec == "fp32" else K.FP64
    specs = kktgen.serve_specs()
    seqs = [kktgen.make_sequence(s) for s in specs]
    T = specs[0].steps
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    vals = [[torch.from_numpy(q.values(t)).to(dev) for t in range(T)] for q in seqs]
    rates = [float(r) for r in args.rates.split(",")]
    nreq = args.requests
    # right-hand sides and outputs, one slot per request index (reused across rates)
    traces = {r: kktgen.serve_trace(r, nreq, T, seed_k=i) for i, r in enumerate(rates)}

    def run(rate, fp_, inflight, trace):
        sv = K.KKTServer(hbm_budget=32 << 30, max_inflight=inflight, max_nrhs=4)
        pids = [sv.add_pattern(q.n, q.rowptr, q.colind, q.values(0), factor_precision=fp_) for q in seqs]
        # warm-up: one request per pattern (replica, graph), not timed
        for p, q in enumerate(seqs):
            b = torch.from_numpy(q.rhs(0)).to(dev)
            sv.wait(sv.submit(pids[p], vals[p][0], b, torch.empty_like(b)))
        bs = []
        for k, (_, p, t, r) in enumerate(trace):
            q = seqs[p]
            b = torch.from_numpy(np.ascontiguousarray(q.rhs(t, nrhs=r))).to(dev)
            bs.append((b, torch.empty_like(b)))
        torch.cuda.synchronize()
        tickets = []
        t0 = time.perf_counter()
        for k, (arr, p, t, r) in enumerate(trace):
            d = t0 + arr - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets.append(sv.submit(pids[p], vals[p][t], bs[k][0], bs[k][1]))
        lat, its, fails = [], [], 0
        for tk in tickets:
            rc, info, tm = sv.wait(tk)
            lat.append(tm["latency_ms"])
            its += [i.iters for i in info]
            fails += int(rc != K.OK or any(not (i.berr <= 1e-10) for i in info))
        el = time.perf_counter() - t0
        st = sv.stats()
        sv.close()
        return {"rate": rate, "throughput": round((len(trace) - fails) / el, 2),
                "p50_ms": round(nearest_rank(lat, 50), 3), "p99_ms": round(nearest_rank(lat, 99), 3),
                "failures": fails, "fgmres_iters_mean": round(float(np.mean(its)), 3),
                "replicas": st["replicas"], "peak_gib": round(st["peak_bytes"] / 2**30, 3)}

    rows, plain, fp64_4 = [], [], []
    for r in rates:
        rows.append(run(r, fp, 4, traces[r]))
        print(f"[bench] serve rate {r}: {rows[-1]}", file=sys.stderr, flush=True)
        if fp != K.FP64:
            fp64_4.append(run(r, K.FP64, 4, traces[r]))
            print(f"[bench] serve fp64 rate {r}: {fp64_4[-1]}", file=sys.stderr, flush=True)
        plain.append(run(r, K.FP64, 1, traces[r]))
        print(f"[bench] plain fp64 rate {r}: {plain[-1]}", file=sys.stderr, flush=True)
    best = max(rows, key=lambda x: x["throughput"])
    out = {
        "metric": "served KKT refactor+solve requests/s at berr<=1e-10 (Poisson, 500-25k buses, 1-4 rhs); p50/p99 latency",
        "value": best["throughput"], "unit": "requests/s", "n_gpus": 1, "steps": nreq, "warmup": len(seqs),
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64" if fp == K.FP32 else "f64", "data": "synthetic",
        "config": {"workload": "serve: " + ", ".join(f"{s.buses}-bus (N={q.n})" for s, q in zip(specs, seqs)) +
                               f" with probabilities {list(kktgen.SERVE_PROBS)}; {nreq} requests per rate; "
                               "4 workers, 32 GiB budget",
                   "precision": "FP32 factors, FP64 refinement" if fp == K.FP32 else "FP64"},
        "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"],
        "per_rate": rows, "fp64_four_workers": fp64_4, "plain_fp64_one_worker": plain,
    }
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described but not built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import numpy as np
    import torch

    import kktgen
    import paper_2302_08656_amd as K

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    args.precision = args.precision or "fp64"
    spec = kktgen.config(args.config)
    t0 = time.perf_counter()
    q = kktgen.make_sequence(spec)
    T = q.steps
    vals = [q.values(t) for t in range(T)]
    rhs = [q.rhs(t) for t in range(T)]
    t_gen = time.perf_counter() - t0
    print(f"[bench] generated {spec.name}: N={q.n} nnz={q.nnz} steps={T} in {t_gen:.1f}s", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    fp32 = args.precision == "fp32"
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, vals[0], approx_sweeps=args.approx_sweeps,
                     factor_precision=K.FP32 if fp32 else K.FP64,
                     persistent_solve={"fixed": 1, "ticket": 2, "levels": 0}[args.solve_mode])
    t_analyze = time.perf_counter() - t0
    st = sk.stats
    print(f"[bench] analyze {t_analyze:.2f}s nnz_lu={st['nnz_lu']} levels={st['levels_f']} "
          f"gpu_levels={st['gpu_levels_f']}/{st['gpu_levels_l']}/{st['gpu_levels_u']}", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sk.bind(0)
    dvals = [torch.from_numpy(v).to(dev) for v in vals]
    drhs = [torch.from_numpy(b).to(dev) for b in rhs]
    x = torch.empty(q.n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def unit(t):
        if args.path == "fused":
            return sk.refactor_refine(dvals[t], drhs[t], x)[1]
        sk.refactor(dvals[t])
        _, info = sk.refine(drhs[t], x)
        return info[0]

    stride = coprime_stride(T)
    order = [(i * stride) % T for i in range(max(args.steps, args.warmup, 1))]
    for i in range(args.warmup):
        unit(order[i])
    torch.cuda.synchronize()
    lat, iters, fails, berrs, perts = [], [], 0, [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t = order[i]
        a = time.perf_counter()
        inf = unit(t)
        lat.append((time.perf_counter() - a) * 1e3)
        iters.append(inf.iters)
        berrs.append(inf.berr)
        perts.append(inf.perturbed_pivots)
        if inf.status != K.OK or not (inf.berr <= 1e-10):
            fails += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ok_units = args.steps - fails
    value = ok_units / elapsed

    # per-kernel-class launch timing with HIP events on the library's stream (torch's
    # current stream), over a second pass of the same units in the same order
    nprof = min(args.steps, T)
    sk.profile(True)
    solves = 0
    for i in range(nprof):
        solves += 1 + unit(order[i]).iters
    prof = sk.profile_read()
    sk.profile(False)
    sym = sk.export_symbolic()
    cols = np.repeat(np.arange(q.n), np.diff(sym["colptr"]))
    nnz_l = int(np.count_nonzero(sym["rowidx"] > cols))
    nnz_u = st["nnz_lu"] - q.n - nnz_l
    # algorithmic bytes per unit of work of each kernel class, from the compulsory-traffic
    # definitions (int32 indices, FP64 values, FP32 factor values with --precision fp32): a
    # refactorization class writes each factor entry of the columns it factors once and reads
    # its structure once (fb + 4 bytes per entry); solves read each factor entry and its
    # column index once plus the vectors;
    # the value update reads A's values and map and writes the factor; the row-ordered copy
    # of the factor is this design's own layout conversion and is reported apart
    # (layout_copy_bytes), not priced into any class
    fb = 4 if fp32 else 8
    ent = fb + 4
    per_unit = {
        "refactor_large": ent * st["nnz_lu_wide"] * nprof,
        "refactor_medium": ent * st["nnz_lu_medium"] * nprof,
        "refactor_w256": ent * st["nnz_lu_w256"] * nprof,
        "refactor_small": ent * (st["nnz_lu"] - st["nnz_lu_wide"] - st["nnz_lu_medium"] - st["nnz_lu_w256"]) * nprof,
        "lsolve": (ent * nnz_l + 48 * q.n) * solves,
        "usolve": (ent * (nnz_u + q.n) + 48 * q.n) * solves,
        "update": (12 * q.nnz + ent * st["nnz_lu"] + 40 * q.n) * nprof,
    }
    tname = "float" if fp32 else "double"
    kernel_of = {"refactor_large": f"k_refactor_wide<WideCfg<{tname}, 512, 2, 256, 32, 4> >",
                 "refactor_medium": f"k_refactor_wide<WideCfg<{tname}, 256, 4, 128, 16, 2> >",
                 "refactor_w256": f"k_refactor_wide<WideCfg<{tname}, 256, 2, 128, 32, 4> >",
                 "refactor_small": "k_refactor_small",
                 "lsolve": "k_lsolve_persistent", "usolve": "k_usolve_persistent", "to_csr": "k_to_csr",
                 "update": "k_set_call..k_max_parts", "residual": "k_residual/k_spmv", "krylov": "krylov"}
    ranked = sorted((v[1], k) for k, v in prof.items())
    dom = ranked[-1][1]
    launches, ms = prof[dom]
    if per_unit.get(dom) and launches:
        ach = per_unit[dom] / (ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(ach, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 6), "traffic": stored_traffic(kernel_of[dom]),
                    "kernel": kernel_of[dom], "launches": launches, "avg_launch_us": round(ms / launches * 1e3, 3),
                    "bytes_per_launch": per_unit[dom] // launches,
                    "bytes_rule": f"{ent} B per factor entry of the columns the launches factor",
                    "layout_copy_bytes_per_unit": (4 + 2 * fb) * st["nnz_lu"]}
    else:
        roofline = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                    "traffic": None, "kernel": kernel_of.get(dom, dom)}
    b_unit = sum(unit_bytes(q.n, q.nnz, st["nnz_lu"], k, fb) for k in iters) / len(iters)
    whole = {"bytes_per_unit": int(b_unit), "achieved": round(b_unit * value / 1e9, 3), "unit": "GB/s",
             "frac": round(b_unit * value / 1e9 / HBM_PEAK_GBS, 6)}
    breakdown = {k: {"launches_per_unit": round(v[0] / nprof, 2), "ms_per_unit": round(v[1] / nprof, 4)}
                 for k, v in prof.items()}
    nproc, cpu_model = host_info()
    timed = sorted(set(order[:args.steps]))

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "units/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{spec.name}: {spec.buses}-bus-shaped KKT sequence, N={q.n}, "
                               f"nnz={q.nnz}, {T} systems, 1 rhs each",
                   "precision": ("FP32 factors (refactorization and the factor reads of the solves), "
                                 "FP64 residuals and FGMRES" if fp32 else "FP64 throughout"),
                   "nnz_lu": st["nnz_lu"], "pivot_tau": sk.opts["pivot_tau"],
                   "offdiag_pivots": int(np.count_nonzero(sym["P"] != sym["Q"])),
                   "timed_order": f"system (i * {stride}) mod {T} for unit i = 0..{args.steps - 1}",
                   "timed_systems": (f"all {T}" if len(timed) == T else timed),
                   "refinement_preconditioner": (f"{args.approx_sweeps} Jacobi sweeps per triangle"
                                                 if args.approx_sweeps else "exact triangular solves"),
                   "solve_mode": args.solve_mode, "path": args.path},
        "p50_ms": round(nearest_rank(lat, 50), 4), "p99_ms": round(nearest_rank(lat, 99), 4),
        "failures": fails, "fgmres_iters_mean": round(float(np.mean(iters)), 3),
        "berr_max": float(np.max(berrs)),
        "perturbed_pivots_per_unit": round(float(np.mean(perts)), 2),
        "workspace_bytes": sk.workspace_bytes(1),
        "analyze_s": round(t_analyze, 3),
        "analyze_amortized_ms_per_unit": round(t_analyze / T * 1e3, 3),
        "roofline": roofline,
        "whole_unit_bytes": whole,
        "kernel_breakdown": breakdown,
    }
    sk.close()
    del dvals, drhs, x
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        so = oracle.Symbolic(q.n, q.rowptr, q.colind, vals[0])
        t_oa = time.perf_counter() - t0
        sample = order[:max(1, min(args.cpu_sample, args.steps))]
        t0 = time.perf_counter()
        for t in sample:
            lu, r, c, _, _ = so.refactor(vals[t])
            so.fgmres(vals[t], lu, r, c, rhs[t])
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(len(sample) / t_cpu, 4), "unit": "units/s", "cores": 1,
                               "kind": "oracle", "nproc": nproc, "cpu_model": cpu_model,
                               "sample": f"the first {len(sample)} timed units (systems {sample}) of the same "
                                         f"order, single-threaded C oracle; oracle analyze {t_oa:.1f}s"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
