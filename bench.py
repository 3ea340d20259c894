#!/usr/bin/env python3
"""Benchmark of the LADMM mapping solve on one MI355X.

A step is one full solve (data projection, `iters` LADMM iterations, output
transpose) of the 3-D diffusion-relaxation workload: a 128 x 128 x 64 grid
(1,048,576 voxels), P = 60 measurements (6 b-values x 10 echo times),
Q = 1600 spectral nodes (40 x 40 grid of diffusivity x T2), float32
iteration, 300 iterations, lambda = 1e-2, rank from the 0.005 % rule.
Inputs are seeded synthetic data resident in device memory before the
timed region. The dictionary factorisation (SVD) is done once per context
and reported separately as setup_ms.

Prints one JSON line (see the field list at the end of main()).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LADMM voxel-iterations/s at fixed error vs FP64 oracle; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "c2": "3-D diffusion-relaxation 128x128x64, P=60, Q=1600 (40x40), fp32, 300 iters",
    "c3": "3-D T1-T2 fingerprinting-like 96x96x32, P=1000, Q=1024 (32x32), bf16x3, 300 iters",
    "c1": "2-D diffusion-relaxation 32x32, P=30, Q=100 (10x10), fp64, 500 iters",
    "c4": "64 uneven 2-D slices (sides 48..256), P in {30,60}, Q in {100,400,1600}, one batch, "
          "200 iters",
    "c3x": "3-D T1-T2 fingerprinting-like 96x96x32, P=1000, Q=1024 (32x32) at the exact rank "
           "r=min(P,Q)=1000 (unapproximated K), bf16x3 GEMM path, 300 iters",
    "c5": "served stream: Poisson arrivals, N log-uniform 1e3..1e6 (2-D up to 65,536, else "
          "nz=32), Q in {100 fp64 500 it, 400 fp32 300 it, 1024 bf16x3 300 it, "
          "1600 fp32 300 it}",
}
DTYPE_NAME = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3 (f32 state)"}
# workloads that run a recipe at another rank: name -> (recipe, rank)
RECIPE = {"c3x": ("c3", -1)}
MFMA_PEAK_TFS = {"bf16x3": 2500.0, "fp32": 157.3}    # dense MI355X matrix peaks


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_label(name, default_prec, prec):
    """The workload's description, naming the precision actually run."""
    label = WORKLOADS[name]
    return label if prec == default_prec else label.replace(default_prec, prec)


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * p / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def alg_bytes_per_voxel_iter(Q, r, wbytes):
    """Bytes one fused iteration must move per voxel: read z^k and write
    z^{k+1} (Q values each), read w, y, a.h and write w, y (r values each)."""
    return (2 * Q + 5 * r) * wbytes


def sampled_parity(mp, prob, prec, kernel, workload):
    """Full-size solve for the stored number of iterations (4), compared at
    sampled voxels with oracle values written by tests/golden/make_fullsize_golden.py
    (the norm of z at the voxel and its projection on a fixed seeded Gaussian
    vector). Both relative differences are lower bounds of the voxel's
    relative error; the element-wise check is tests/test_gpu_fullsize.py."""
    import numpy as np
    import torch
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{workload}.json")
    if not os.path.exists(path) or list(prob.grid) != json.load(open(path))["grid"]:
        return None
    with open(path) as fh:
        gold = json.load(fh)
    dt = torch.float64 if prec == "fp64" else torch.float32
    M = torch.tensor(prob.m, dtype=dt, device="cuda")
    F = mp.solve_torch(M, prob.lam, prob.beta, gold["iters"], precision=prec, kernel=kernel,
                       rank=gold["rank"], xi_p=gold["xi_p"])
    torch.cuda.synchronize()
    g = np.random.Generator(np.random.PCG64(gold["projection_seed"])).standard_normal(prob.Q)
    nx, ny, _ = prob.grid
    e_norm = e_proj = 0.0
    for smp in gold["samples"]:
        x, y, z = smp["voxel"]
        zr = F[x + nx * (y + ny * z)].double().cpu().numpy()
        e_norm = max(e_norm, abs(np.linalg.norm(zr) - smp["norm"]) / smp["norm"])
        e_proj = max(e_proj, abs(zr @ g - smp["proj"]) / (smp["norm"] * np.linalg.norm(g)))
    del M, F
    return {"kind": "norm and seeded projection of z at sampled voxels vs stored oracle values",
            "max_rel_err_norm": e_norm, "max_rel_err_proj": e_proj,
            "samples": len(gold["samples"]), "iters": gold["iters"],
            "tol": {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3}[prec]}


def iters300_parity(name, prec, kernel, F=None):
    """z after the configured iteration count (300; 500 for c1) against the
    stored FP64 oracle results of tests/golden/make_iters300_golden.py: the full
    Q-vectors at the sampled voxels and the spectral sum of z at every voxel. For
    c3 and c1 the stored problem is the benchmark's own (full size), so the timed
    map F is checked; for c2 it is the same recipe on a 128 x 128 x 8 grid (256
    bricks of the timed 16 x 8 x 4 launch shape), solved here in the same
    precision."""
    import numpy as np
    import torch

    from paper_2401_12890_amd import _ffi, synth
    case = {"c2": ("c2crop", 300), "c3": ("c3", 300), "c1": ("c1", 500)}.get(name)
    path = os.path.join(ROOT, "tests", "golden", f"iters{case[1]}_{case[0]}.npz") if case else None
    if not path or not os.path.exists(path):
        return None
    g = np.load(path)
    grid = tuple(int(v) for v in g["grid"])
    prob = synth.generate(str(g["recipe"]), grid=grid)
    own = F is not None and tuple(F.shape) == (prob.N, prob.Q)
    if not own:
        with _ffi.Mapper(prob.K, prob.grid) as mp:
            M = torch.tensor(prob.m, dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")
            F = mp.solve_torch(M, prob.lam, prob.beta, int(g["iters"]), precision=prec, kernel=kernel)
            torch.cuda.synchronize()
            del M
    idx = torch.as_tensor(g["index"], device=F.device)
    z_s = F[idx].double().cpu().numpy()
    zsum = F.double().sum(dim=1).cpu().numpy()
    e_s = float(np.linalg.norm(z_s - g["z"]) / np.linalg.norm(g["z"]))
    e_sum = float(np.linalg.norm(zsum - g["z_sum_q"]) / np.linalg.norm(g["z_sum_q"]))
    return {"kind": f"z^{int(g['iters'])} at sampled voxels (full Q-vectors) and every voxel's spectral "
                    "sum vs stored FP64 oracle values",
            "map": "the timed map" if own else f"same recipe on {'x'.join(map(str, grid))}",
            "samples": int(len(g["index"])), "iters": int(g["iters"]),
            "rel_err_sampled": e_s, "rel_err_spectral_sums": e_sum,
            "tol": {"fp32": 1e-5, "bf16x3": 1e-3, "fp64": 1e-10}[prec]}


def kernel_source_digest(source="kernels_fused.hip"):
    """sha256 of a kernel source file: counter-derived traffic is only reported
    while it matches the source the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "paper_2401_12890_amd", "csrc", source)
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(workload, kernel_id, precision):
    """HBM bytes per launch of the loop's kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, KiB per dispatch, scaled by the
    calibration factor measured on a copy kernel of known size), or None when
    there is none for this workload, kernel family (2 fused, 4 chunk split) and
    precision, or its kernel source has changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_id", 2) != kernel_id or rec.get("precision") != precision:
        return None
    if rec.get("kernel_source_sha256") != kernel_source_digest(rec.get("kernel_source_file", "kernels_fused.hip")):
        return None
    kib = rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] + \
        rec["write_kib_per_dispatch"] * rec["write_scale"]
    return kib * 1024.0


def cpu_baseline(name, seconds_hint=20.0, rank=0):
    """The FP64 oracle, untuned, on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    from paper_2401_12890_amd import synth
    grid = {"c2": (64, 64, 8), "c3": (48, 48, 8), "c1": (32, 32, 1)}[name]
    if rank == -1:
        grid = (24, 24, 8)
    prob = synth.generate(name, grid=grid)
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 1, rank=rank)
    t1 = time.perf_counter()
    one = t1 - t0
    # iterations beyond the first, quadrupled until they take 2 s (a small
    # problem's few iterations are lost in the setup's timing noise)
    n_it = 6
    while True:
        t0 = time.perf_counter()
        oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 1 + n_it, rank=rank)
        t1 = time.perf_counter()
        loop = (t1 - t0) - one
        if loop >= 2.0 or n_it >= 16384:
            break
        n_it *= 4
    per_iter = max(loop, 1e-9) / n_it
    N = prob.N
    return {"value": N / per_iter, "unit": "voxel-iterations/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{name} generator on a {grid[0]}x{grid[1]}x{grid[2]} grid ({N} voxels, "
                      f"Q={prob.Q}{', exact rank' if rank == -1 else ''}), {n_it} float64 "
                      f"iterations after one, NumPy "
                      f"{np.__version__}, {platform.processor() or platform.machine()}"}


def cpu_baseline_batch(sub):
    """The FP64 oracle, untuned, on a few slices of the batched workload."""
    import oracle
    t0 = time.perf_counter()
    for p in sub:
        oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 1)
    one = time.perf_counter() - t0
    t0 = time.perf_counter()
    for p in sub:
        oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 4)
    four = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": sum(p.N for p in sub) * 3 / max(four - one, 1e-9),
            "unit": "voxel-iterations/s", "cores": int(cores), "kind": "oracle",
            "sample": f"the first {len(sub)} slices ({sum(p.N for p in sub)} voxels), 3 float64 "
                      f"iterations after one"}


def batch200_parity(Fs, probs, prec):
    """The timed batch's own maps of the stored slices (tests/golden/batch200_c4.npz,
    written by tests/golden/make_batch200_golden.py from the generator and the
    oracle only: per Q the smallest and the largest slice at the configured 200
    iterations) against the stored FP64 values: the full Q-vectors at the sampled
    voxels and every voxel's spectral sum; the worst slice is reported."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "batch200_c4.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    if int(g["iters"]) != probs[0].iters or int(g["nslices"]) != len(probs):
        return None

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    import torch
    e_s, e_sum = 0.0, 0.0
    for k in (int(v) for v in g["slices"]):
        F = Fs[k]
        idx = torch.as_tensor(g[f"s{k}_index"], device=F.device)
        e_s = max(e_s, rel(F[idx].double().cpu().numpy(), g[f"s{k}_z"]))
        e_sum = max(e_sum, rel(F.double().sum(dim=1).cpu().numpy(), g[f"s{k}_z_sum_q"]))
    return {"kind": "the timed batch's maps of stored slices vs stored FP64 oracle values (z^200 at "
                    "sampled voxels, every voxel's spectral sum; worst slice)",
            "slices": [int(v) for v in g["slices"]], "iters": int(g["iters"]),
            "rel_err_sampled": e_s, "rel_err_spectral_sums": e_sum,
            "tol": {"fp32": 1e-5, "bf16x3": 1e-3}[prec]}


def bench_batch(args):
    """Batched uneven slices: one batch solve (all slices, shared launches,
    autotuned bricks) per step, in bf16x3 and in float32, against the same
    slices solved one after another in float32."""
    import numpy as np
    import torch

    from paper_2401_12890_amd import _ffi, synth
    log("generating 64 slices")
    probs = synth.generate_batch(iters=args.iters)
    iters = probs[0].iters
    Ntot = sum(p.N for p in probs)
    Ms = [torch.tensor(p.m, dtype=torch.float32, device="cuda") for p in probs]
    Fs = [torch.empty((p.N, p.Q), dtype=torch.float32, device="cuda") for p in probs]
    bm = _ffi.BatchMapper([p.K for p in probs], [p.grid for p in probs])
    lams, betas = [p.lam for p in probs], [p.beta for p in probs]
    torch.cuda.synchronize()
    out = {}
    for prec in ("bf16x3", "fp32"):
        bm.solve_torch(Ms, lams, betas, iters, Fs=Fs, precision=prec, autotune=True)  # tune + warm
        torch.cuda.synchronize()
        tuned = bm.stats()["classes"]
        lat, loop = [], []
        for k in range(args.steps):
            ts = time.perf_counter()
            bm.solve_torch(Ms, lams, betas, iters, Fs=Fs, precision=prec)
            lat.append((time.perf_counter() - ts) * 1e3)
            loop.append(bm.stats()["iterate_ms"])
            log(f"{prec} batch step {k}: {lat[-1]:.1f} ms (loop {loop[-1]:.1f} ms)")
        torch.cuda.synchronize()
        par = None if args.no_parity else batch200_parity(Fs, probs, prec)
        out[prec] = dict(ms=sum(lat) / len(lat), loop_ms=sum(loop) / len(loop), lat=lat,
                         classes=tuned, ranks=None, parity=par)
    # the same slices one after another (float32, default bricks)
    seq_ms = 0.0
    ranks = []
    mps = [_ffi.Mapper(p.K, p.grid) for p in probs]
    for mp, p, M, F in zip(mps, probs, Ms, Fs):               # warm
        mp.solve_torch(M, p.lam, p.beta, iters, F=F, precision="fp32")
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for mp, p, M, F in zip(mps, probs, Ms, Fs):
        mp.solve_torch(M, p.lam, p.beta, iters, F=F, precision="fp32")
        ranks.append(mp.stats()["rank"])
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - ts) * 1e3
    for mp in mps:
        mp.close()
    bm.close()
    alg = sum((2 * p.Q + 5 * r) * 4 * p.N for p, r in zip(probs, ranks))
    per_launch_ms = out["bf16x3"]["loop_ms"] / iters
    achieved = alg / (per_launch_ms / 1e3) / 1e9
    value = Ntot * iters / (out["bf16x3"]["ms"] / 1e3)
    cpu = None if args.no_cpu_baseline else cpu_baseline_batch(probs[:2])
    line = {
        "metric": METRIC, "value": value, "unit": "voxel-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": out["bf16x3"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3 (f32 state)", "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": WORKLOADS["c4"], "slices": len(probs), "voxels": Ntot,
                   "iters": iters, "classes_bf16x3": out["bf16x3"]["classes"],
                   "classes_fp32": out["fp32"]["classes"]},
        "p50_ms": percentile(out["bf16x3"]["lat"], 50), "p99_ms": percentile(out["bf16x3"]["lat"], 99),
        "batched_fp32_voxel_iter_per_s": Ntot * iters / (out["fp32"]["ms"] / 1e3),
        "sequential_fp32_voxel_iter_per_s": Ntot * iters / (seq_ms / 1e3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "shared fused launches (bf16x3)", "avg_launch_ms": per_launch_ms,
                     "alg_bytes_per_launch": alg},
        "cpu_baseline": cpu,
        "parity": None if args.no_parity else {"bf16x3": out["bf16x3"]["parity"], "fp32": out["fp32"]["parity"]},
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_serve(probs):
    """The FP64 oracle, untuned, on one small job of each dictionary class of
    the served stream (cropped to at most 48 x 48 voxels)."""
    import oracle
    from paper_2401_12890_amd import synth
    sub = []
    for sp in probs:
        g = (min(sp["grid"][0], 48), min(sp["grid"][1], 48), 1)
        sub.append(synth.serving_problem(dict(sp, grid=g), single=False))
    t0 = time.perf_counter()
    for p in sub:
        oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 1)
    one = time.perf_counter() - t0
    t0 = time.perf_counter()
    for p in sub:
        oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 4)
    four = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": sum(p.N for p in sub) * 3 / max(four - one, 1e-9),
            "unit": "voxel-iterations/s", "cores": int(cores), "kind": "oracle",
            "sample": f"one job per dictionary class cropped to <= 48x48 "
                      f"({sum(p.N for p in sub)} voxels, Q={[p.Q for p in sub]}), 3 float64 "
                      f"iterations after one"}


def bench_serve(args):
    """Served stream: jobs are submitted at their Poisson arrival times to a
    server that admits them first in, first out under a device-memory budget
    and advances all running jobs in shared fused launches (continuous
    batching over four streams). Reported: throughput over the makespan,
    p50 / p99 arrival-to-completion latency, the offered load, and the same
    stream served one job at a time (service times measured on the same
    server, queueing replayed for the same arrivals)."""
    import numpy as np
    import torch

    from paper_2401_12890_amd import _ffi, synth
    prec_of = {"c1": "fp64", "c2": "fp32", "c3": "bf16x3"}
    specs = synth.serving_stream(njobs=args.jobs, rate=args.rate)
    log(f"generating {len(specs)} served jobs")
    jobs, Ks = [], {}
    for k, sp in enumerate(specs):
        prec = prec_of[sp["recipe"]]
        p = synth.serving_problem(sp, single=prec != "fp64")
        dt = torch.float64 if prec == "fp64" else torch.float32
        M = torch.from_numpy(np.ascontiguousarray(p.m)).to(device="cuda", dtype=dt)
        F = torch.empty((p.N, p.Q), dtype=dt, device="cuda")
        Ks.setdefault(sp["Q"], p.K)
        jobs.append(dict(spec=sp, prec=prec, iters=p.iters, lam=p.lam, beta=p.beta, M=M, F=F,
                         grid=p.grid, N=p.N, P=p.P, Q=p.Q))
        if k % 10 == 9:
            log(f"  {k + 1} jobs generated")
    torch.cuda.synchronize()
    budget = args.budget_gb * 1e9

    def server():
        sv = _ffi.Server(budget, args.streams)
        dicts = {Q: sv.add_dictionary(K) for Q, K in Ks.items()}
        seen = set()
        for j in jobs:                    # warm every class: kernels and device constants
            key = (j["Q"], j["grid"][2] == 1)
            if key in seen:
                continue
            seen.add(key)
            g = (16, 16, 1) if key[1] else (8, 8, 4)
            sv.submit(dicts[j["Q"]], g, j["M"][:256], j["lam"], j["beta"], 2, ready=True,
                      precision=j["prec"])
        sv.drain()
        return sv, dicts

    def submit(sv, dicts, j):
        return sv.submit(dicts[j["Q"]], j["grid"], j["M"], j["lam"], j["beta"], j["iters"],
                         F=j["F"], ready=True, precision=j["prec"])

    # ---- continuous batching at the arrival times
    sv, dicts = server()
    n = len(jobs)
    ids, sub_wall = [None] * n, [0.0] * n
    log(f"serving {n} jobs at {args.rate} jobs/s")
    t0 = time.perf_counter()
    nxt = 0
    while True:
        now = time.perf_counter() - t0
        while nxt < n and specs[nxt]["t"] <= now:
            ids[nxt] = submit(sv, dicts, jobs[nxt])
            sub_wall[nxt] = time.perf_counter() - t0
            nxt += 1
        pending = sv.pump(args.horizon)
        if nxt == n and pending == 0:
            break
        if pending == 0 and nxt < n:
            time.sleep(max(0.0, specs[nxt]["t"] - (time.perf_counter() - t0)))
    sv.drain()
    wall = time.perf_counter() - t0
    infos = [sv.poll(i) for i in ids]
    stats = sv.stats()
    off = infos[0]["submit_ms"] - sub_wall[0] * 1e3      # server clock - loop clock
    arrive = [off + sp["t"] * 1e3 for sp in specs]
    lat = [inf["done_ms"] - a for inf, a in zip(infos, arrive)]
    makespan_ms = max(inf["done_ms"] for inf in infos) - arrive[0]
    vox_it = sum(j["N"] * j["iters"] for j in jobs)
    value = vox_it / (makespan_ms / 1e3)
    ranks = [inf["rank"] for inf in infos]
    alg = sum(alg_bytes_per_voxel_iter(j["Q"], r, 8 if j["prec"] == "fp64" else 4) * j["N"] *
              j["iters"] for j, r in zip(jobs, ranks))
    log(f"continuous batching: makespan {makespan_ms:.0f} ms, p50 {percentile(lat, 50):.0f} ms, "
        f"p99 {percentile(lat, 99):.0f} ms, {stats['launches']} launches")

    # ---- parity: served maps equal the same jobs solved alone (smallest job per class)
    parity = None
    if not args.no_parity:
        smallest = {}
        for k, j in enumerate(jobs):
            key = (j["Q"], j["prec"])
            if key not in smallest or j["N"] < jobs[smallest[key]]["N"]:
                smallest[key] = k
        same = []
        for k in smallest.values():
            j = jobs[k]
            Fserved = sv.result(ids[k])
            with _ffi.Mapper(Ks[j["Q"]], j["grid"]) as mp:
                Fsolo = mp.solve_torch(j["M"], j["lam"], j["beta"], j["iters"],
                                       precision=j["prec"], kernel="fused")
                torch.cuda.synchronize()
            same.append(bool(torch.equal(Fserved, Fsolo)))
            del Fsolo
        parity = {"kind": "served map bitwise equal to the same job solved alone (fused kernel)",
                  "jobs": [dict(N=jobs[k]["N"], Q=jobs[k]["Q"], precision=jobs[k]["prec"])
                           for k in smallest.values()], "equal": same}
    sv.close()

    # ---- one job at a time on the same kind of server: service times
    sv, dicts = server()
    service = []
    for j in jobs:
        i = submit(sv, dicts, j)
        sv.drain()
        inf = sv.poll(i)
        service.append(inf["done_ms"] - inf["submit_ms"])
    sv.close()
    end, seq_lat = -1e30, []
    for a, sms in zip(arrive, service):
        end = max(a, end) + sms
        seq_lat.append(end - a)
    seq_makespan = end - arrive[0]
    rho = args.rate * (sum(service) / n) / 1e3
    log(f"one at a time: mean service {sum(service) / n:.1f} ms, offered load {rho:.2f}, "
        f"p50 {percentile(seq_lat, 50):.0f} ms, p99 {percentile(seq_lat, 99):.0f} ms")
    cpu = None
    if not args.no_cpu_baseline:
        firsts = {}
        for sp in specs:
            firsts.setdefault(sp["Q"], sp)
        cpu = cpu_baseline_serve(list(firsts.values()))
    achieved = alg / (makespan_ms / 1e3) / 1e9
    by_class = {}
    for j, l_cb, l_seq in zip(jobs, lat, seq_lat):
        c = by_class.setdefault(f"Q={j['Q']} {j['prec']}", dict(jobs=0, cb=[], seq=[], voxels=0))
        c["jobs"] += 1
        c["voxels"] += j["N"]
        c["cb"].append(l_cb)
        c["seq"].append(l_seq)
    classes = {k: dict(jobs=v["jobs"], voxels=v["voxels"], p50_ms=percentile(v["cb"], 50),
                       max_ms=max(v["cb"]), one_at_a_time_p50_ms=percentile(v["seq"], 50),
                       one_at_a_time_max_ms=max(v["seq"]))
               for k, v in sorted(by_class.items())}
    line = {
        "metric": METRIC, "value": value, "unit": "voxel-iterations/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": makespan_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "mixed (f64, f32, bf16x3)",
        "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": WORKLOADS["c5"], "jobs": n, "rate_jobs_per_s": args.rate,
                   "voxels": sum(j["N"] for j in jobs), "budget_bytes": budget,
                   "streams": stats["streams"], "horizon_ms": args.horizon,
                   "classes": stats["classes"]},
        "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
        "offered_load": rho, "mean_service_ms": sum(service) / n,
        "one_at_a_time": {"p50_ms": percentile(seq_lat, 50), "p99_ms": percentile(seq_lat, 99),
                          "voxel_iter_per_s": vox_it / (seq_makespan / 1e3)},
        "server": {"launches": stats["launches"], "peak_bytes": stats["peak_bytes"],
                   "wall_s": wall},
        "latency_by_class": classes,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "shared fused launches, all classes (aggregate over the makespan)",
                     "alg_bytes": alg},
        "cpu_baseline": cpu, "parity": parity,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None)
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "unfused", "split"])
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--grid", type=int, nargs=3, default=None,
                    help="solve the workload's recipe on another grid (nx ny nz)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-monitor", action="store_true",
                    help="skip the monitored solve that measures the monitoring cost")
    ap.add_argument("--jobs", type=int, default=None, help="served stream: number of jobs")
    ap.add_argument("--rate", type=float, default=20.0, help="served stream: arrivals per s")
    ap.add_argument("--streams", type=int, default=4, help="served stream: HIP streams")
    ap.add_argument("--horizon", type=float, default=4.0, help="served stream: ms per pump")
    ap.add_argument("--budget-gb", type=float, default=96.0, help="served stream: state budget")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU path is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2401_12890_amd import _ffi, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "c4":
        return bench_batch(args)
    if args.workload == "c5":
        return bench_serve(args)
    log("generating workload", args.workload)
    recipe, rank = RECIPE.get(args.workload, (args.workload, 0))
    prob = synth.generate(recipe, iters=args.iters, grid=args.grid)
    prec = args.precision or prob.precision
    iters = prob.iters
    dt = torch.float64 if prec == "fp64" else torch.float32
    wbytes = 8 if prec == "fp64" else 4
    M = torch.tensor(prob.m, dtype=dt, device="cuda")
    F = torch.empty((prob.N, prob.Q), dtype=dt, device="cuda")
    mp = _ffi.Mapper(prob.K, prob.grid)
    setup_ms = mp.stats()["setup_ms"]
    stream = torch.cuda.current_stream()
    kw = dict(precision=prec, kernel=args.kernel, rank=rank)
    log("warmup", args.warmup)
    for _ in range(args.warmup):
        mp.solve_torch(M, prob.lam, prob.beta, iters, F=F, stream=stream, **kw)
    torch.cuda.synchronize()
    lat, loop_ms, gemm = [], [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        ts = time.perf_counter()
        mp.solve_torch(M, prob.lam, prob.beta, iters, F=F, stream=stream, **kw)
        lat.append((time.perf_counter() - ts) * 1e3)
        sk = mp.stats()
        loop_ms.append(sk["iterate_ms"])
        gemm.append((sk["gemm_ms"], sk["gemm_flops"]))
        log(f"step {k}: {lat[-1]:.2f} ms (loop {loop_ms[-1]:.2f} ms)")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    st = mp.stats()
    r = st["rank"]
    ms_per_step = max(wall * 1e3, ev_ms) / args.steps
    value = prob.N * iters / (ms_per_step / 1e3)

    # dominant kernel: the per-iteration kernel(s) of the loop, timed by the
    # library's HIP events on this stream (no monitoring in the timed loop)
    per_launch_ms = (sum(loop_ms) / len(loop_ms)) / iters
    alg = alg_bytes_per_voxel_iter(prob.Q, r, wbytes) * prob.N
    achieved = alg / (per_launch_ms / 1e3) / 1e9
    kern_name = {1: "k_update+k_projw (unfused)", 2: "k_fused",
                 3: "hipBLASLt GEMM (GEMM path)" if st.get("gemm_library") else "k_gemm_tn (GEMM path)",
                 4: "k_split (chunk split)"}[st["kernel"]]
    if st["kernel"] == 3:
        # dominant kernel: the GEMM (two launches per iteration, equal flops), timed by the
        # library's HIP events around each launch. Algorithmic flops: the two contractions
        # at the unpadded rank, 2 x 2 r Q per voxel, times 3 bf16 products for bf16x3.
        g_ms = sum(x[0] for x in gemm) / len(gemm)
        n_launch = 2 * iters
        split = 3 if prec == "bf16x3" else 1
        alg_flops = 2.0 * r * prob.Q * prob.N * split          # per launch
        per_gemm_ms = g_ms / n_launch
        achieved_t = alg_flops / (per_gemm_ms / 1e3) / 1e12
        peak = MFMA_PEAK_TFS[prec]
        roofline = {"bound": "mfma", "achieved": round(achieved_t, 1), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved_t / peak, 4), "traffic": None,
                    "kernel": kern_name, "avg_launch_ms": round(per_gemm_ms, 5),
                    "alg_flops_per_launch": alg_flops,
                    "issued_flops_per_launch": sum(x[1] for x in gemm) / len(gemm) / n_launch,
                    "gemm_share_of_loop": round(g_ms / (sum(loop_ms) / len(loop_ms)), 4)}
    else:
        traffic = measured_traffic(args.workload, st["kernel"], prec)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": kern_name, "avg_launch_ms": round(per_launch_ms, 5),
                    "alg_bytes_per_launch": alg}
        if 2 * prob.N * prob.Q * wbytes < (64 << 20):
            roofline["note"] = ("the state arrays fit in the caches: the run is latency-bound and "
                                "the fraction of the HBM peak does not bound it")

    # monitoring cost: one more solve with the float64 reductions every 10 iterations
    monitor = None
    if not args.no_monitor:
        mp.solve_torch(M, prob.lam, prob.beta, iters, F=F, stream=stream, check_every=10, **kw)
        torch.cuda.synchronize()
        sm = mp.stats()
        plain = sum(loop_ms) / len(loop_ms)
        monitor = {"check_every": 10, "checks": len(sm["hist_iter"]),
                   "loop_ms": sm["iterate_ms"], "plain_loop_ms": plain,
                   "overhead": sm["iterate_ms"] / plain - 1.0,
                   "objective_last": sm["hist_objective"][-1] if sm["hist_objective"] else None}
        log(f"monitored loop {sm['iterate_ms']:.2f} ms against {plain:.2f} ms")

    parity = None
    if not args.no_parity and args.grid is None and args.iters is None:
        log("parity vs stored oracle values")
        parity = {"fullsize_iters4": sampled_parity(mp, prob, prec, args.kernel, args.workload)}
        if rank == 0:                    # stored long runs exist at the rank rule's rank
            parity["iters300" if recipe != "c1" else "iters500"] = iters300_parity(recipe, prec, args.kernel, F)
    mp.close()
    del M, F
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(recipe, rank=rank)

    out = {
        "metric": METRIC, "value": value, "unit": "voxel-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE_NAME[prec], "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": workload_label(args.workload, prob.precision, prec) if args.grid is None
                   else f"{args.workload} recipe on a {'x'.join(map(str, prob.grid))} grid",
                   "grid": list(prob.grid), "P": prob.P,
                   "Q": prob.Q, "rank": r, "iters": iters, "lambda": prob.lam,
                   "beta": prob.beta, "precision": prec, "kernel": kern_name},
        "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
        "loop_voxel_iter_per_s": prob.N * iters / (sum(loop_ms) / len(loop_ms) / 1e3),
        "setup_ms": setup_ms, "project_ms": st["project_ms"], "output_ms": st["output_ms"],
        "roofline": roofline, "cpu_baseline": cpu, "parity": parity, "monitor": monitor,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
