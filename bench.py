#!/usr/bin/env python3
"""Benchmark of the MVGD hot path on one MI355X: assemble + apply on a synthetic cloud.

Workload (default): flat torus (cos t, sin t, cos p, sin p) in R^4 plus noise 1e-4, N = 1,000,000
points, K = 32, f = cos(2t) cos(3p) (Delta f = -13 f), FP32-mixed; the same cloud is also run in
FP64 on the same GPU. A step is one mvgd_assemble (neighbour search, fits, stencil, ELL write) plus
one mvgd_apply of f, with the points already resident in HBM.

Prints ONE JSON line (rank 0, N = 1):
  value        rows/s of the FP32-mixed path = N / (wall time per step)
  roofline     the dominant work, the assembly (neighbour-search kernel + fit kernel, launched
               back to back): algorithmic bytes per assembly (point read + ELL write) / its
               average duration from HIP events recorded by the library on the launch stream,
               against 8 TB/s; traffic from committed rocprofv3 counter summaries of the two
               kernels when they match the current kernel sources, else null
  cpu_baseline the FP64 oracle (brute-force kNN + QR, OpenMP over rows) on a bounded sample of rows
               of the same cloud, on the host cores
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    """Hash of the sources the assembly kernel is compiled from (its body and device helpers)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1603_04100_amd", "csrc")
    for name in ("assemble.hpp", "common.hpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str, precision: str, n_rows: int):
    """HBM bytes per launch of the assembly kernel from a committed counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"assemble_{workload}_{precision}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("n_rows") != n_rows:
        return None
    return rec.get("hbm_bytes_per_launch")


def make_workload(name: str):
    from paper_1603_04100_amd import clouds
    return clouds.config(name)


def run_gpu(mv, torch, P, f, k, steps, warmup, flags, offsets=None):
    """Steps back to back. The event timings of a step are read (and its handle freed) after the
    next step has been enqueued: by then the assembly call of the next step has waited for the
    stream, so reading them costs no extra synchronisation."""
    tk, prev = [], None
    for it in range(warmup + steps):
        if it == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        L = mv.mvgd_assemble(P, k, flags=flags, cloud_offsets=offsets)
        y = mv.mvgd_apply(L, f)
        if prev is not None:
            if prev[1]:
                tk.append(mv.mvgd_timing(prev[0]))
            mv.mvgd_free(prev[0])
        prev = (L, it >= warmup)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tk.append(mv.mvgd_timing(prev[0]))
    mv.mvgd_free(prev[0])
    return wall / steps, tk, y


def run_unbatched(mv, torch, P, f, k, offsets, flags):
    """The same clouds assembled and applied one call per cloud (context for batching)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(len(offsets) - 1):
        a, b = offsets[c], offsets[c + 1]
        L = mv.mvgd_assemble(P[a:b], k, flags=flags)
        mv.mvgd_apply(L, f[a:b].contiguous())
        mv.mvgd_free(L)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(oracle, pts64, k, target_s: float, max_rows: int):
    n = pts64.shape[0]
    rng = np.random.default_rng(123)
    probe = rng.choice(n, min(512, n), replace=False)
    t = time.perf_counter()
    oracle.rows(pts64, k, rows=probe)
    per_row = (time.perf_counter() - t) / probe.shape[0]
    m = int(min(max_rows, n, max(64, target_s / max(per_row, 1e-9))))
    rows = rng.choice(n, m, replace=False)
    t = time.perf_counter()
    cols, vals = oracle.rows(pts64, k, rows=rows)
    dt = time.perf_counter() - t
    return rows, cols, vals, m / dt, dt, m


def bench_serving(args):
    """Serving stream: Poisson arrivals of random spheres / ellipsoids / tori, each request an
    assemble plus 8 applies; continuous batching (FP32-mixed) against one request at a time
    (FP64). Prints one JSON line with p50/p99 latency and throughput of both."""
    import torch
    from paper_1603_04100_amd import serve
    reqs = serve.make_requests(duration_s=args.serve_seconds, rate_hz=args.serve_rate, seed=5)
    print(f"[bench] serving: {len(reqs)} requests over {args.serve_seconds} s at "
          f"{args.serve_rate}/s, {sum(r.points.shape[0] for r in reqs)} points",
          file=sys.stderr, flush=True)
    # warm-up: buffers sized for the largest request (and a few-request batch), the library's
    # kernels loaded, the device allocators' pools grown
    n_max = max(r.points.shape[0] for r in reqs)
    warm = serve.make_requests(duration_s=0.05, rate_hz=200, seed=99, max_requests=4)
    big = max(reqs, key=lambda r: r.points.shape[0])
    warm[-1] = serve.Request(-1, warm[-1].arrival, big.points, big.rhs, big.k)
    srv = serve.Server(precision="fp32", n_streams=4, max_batch=16)
    srv.reserve(4 * n_max)
    # every worker serves the largest request at once (the library's pool grown for four
    # concurrent assemblies of it), then a small mixed batch
    srv.run([serve.Request(-2 - i, 0.0, big.points, big.rhs, big.k) for i in range(4)],
            batching=False)
    srv.run(warm)
    base_srv = serve.Server(precision="fp64", n_streams=1, max_batch=1)
    base_srv.reserve(n_max)
    base_srv.run(warm, batching=False)
    mixed = srv.run(reqs).summary()
    print(f"[bench] batched fp32: {mixed}", file=sys.stderr, flush=True)
    base = base_srv.run(reqs, batching=False).summary()
    print(f"[bench] one-at-a-time fp64: {base}", file=sys.stderr, flush=True)
    out = {"metric": "serving p99 latency (assemble + 8 applies per request)",
           "value": mixed["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": mixed["requests"],
           "warmup": 4, "ms_per_step": mixed["mean_ms"], "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 storage/f64 solves",
           "data": "synthetic",
           "config": {"workload": "serving", "rate_hz": args.serve_rate,
                      "duration_s": args.serve_seconds, "k": 24, "n_apply": 8,
                      "sizes": "log-uniform [5e3, 5e5]", "noise": 1e-3},
           "batched_fp32": mixed, "one_at_a_time_fp64": base,
           "kernel_source_hash": kernel_source_hash()}
    print(json.dumps(out))


def bench_solve(args):
    """-Delta U = 2x on a randomly sampled unit sphere (Sec. 4.2), one pinned value: assemble,
    then BiCGSTAB on the device (FP32-mixed matrix and FP64 matrix); damped Jacobi on the plain
    least-squares rows for contrast. Prints one JSON line."""
    import torch
    from paper_1603_04100_amd import clouds, mvgd as mv
    n, k = args.solve_points, 20
    cl = clouds.sphere(n, 5, k)
    print(f"[bench] sphere solve: N={n} K={k}", file=sys.stderr, flush=True)
    res = {}
    for prec, dt, rtol in (("fp32", torch.float32, 1e-6), ("fp64", torch.float64, 1e-9)):
        P = torch.tensor(cl.points, dtype=dt, device="cuda:0")
        b = 2.0 * cl.points[:, 0]
        b[0] = cl.points[0, 0]
        bt = torch.tensor(b, dtype=dt, device="cuda:0")
        L = mv.mvgd_assemble(P, k)
        mv.mvgd_solve(L, bt, rtol=rtol, max_iter=20, pin_first=True)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = mv.mvgd_solve(L, bt, rtol=rtol, max_iter=20000, pin_first=True,
                                check_every=50)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        err = float((x.double().cpu() - torch.tensor(cl.points[:, 0])).abs().max())
        # per BiCGSTAB iteration: two ELL products ((K+1)(4 + s_v) B per row each, plus the
        # gathered x in double) and ~14 double vector reads/writes per row
        s_v = 4 if prec == "fp32" else 8
        bytes_it = n * (2 * ((k + 1) * (4 + s_v) + 8) + 14 * 8)
        it_s = dt_s / max(info["iterations"], 1)
        res[prec] = {"iterations": info["iterations"], "converged": info["converged"],
                     "rel_residual": info["rel_residual"], "solve_s": dt_s,
                     "ms_per_iteration": it_s * 1e3,
                     "algorithmic_GBps_per_iteration": bytes_it / it_s / 1e9,
                     "max_abs_err_vs_x": err}
        print(f"[bench] {prec}: {res[prec]}", file=sys.stderr, flush=True)
        mv.mvgd_free(L)
    P = torch.tensor(cl.points, device="cuda:0")
    for name, flags in (("mvgd", 0), ("ls", mv.MVGD_FLAG_LS)):
        L = mv.mvgd_assemble(P, k, flags=flags)
        x, info = mv.mvgd_solve(L, torch.tensor(2.0 * cl.points[:, 0], device="cuda:0"),
                                method="jacobi", max_iter=500, rtol=1e-8, pin_first=True,
                                check_every=100)
        res[f"jacobi_500_{name}"] = info
        mv.mvgd_free(L)
    out = {"metric": "BiCGSTAB solve of -Delta U = 2x on the sphere (assembled MVGD matrix)",
           "value": res["fp32"]["solve_s"], "unit": "s", "n_gpus": 1,
           "steps": res["fp32"]["iterations"], "warmup": 1,
           "ms_per_step": res["fp32"]["ms_per_iteration"], "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 matrix/f64 vectors",
           "data": "synthetic", "config": {"workload": "sphere_poisson", "n_points": n, "k": k,
                                           "rtol_fp32": 1e-6, "rtol_fp64": 1e-9},
           "results": res, "kernel_source_hash": kernel_source_hash()}
    print(json.dumps(out))


def bench_neumann(args):
    """Open surface with the Neumann condition (Sec. 3.1): upper unit hemisphere, N interior points
    plus ~sqrt(pi N) equispaced points on the boundary circle, K = 20. A step is one
    mvgd_assemble_neumann (search on the whole cloud, boundary frames, ghost points, assembly on
    the augmented cloud, folding), timed by wall clock around each call (the call itself waits
    for the stream); the plain assembly of the same cloud is timed alongside. Then
    (sigma - Delta) U = (sigma + 6) z^2 - 2, sigma = 1, with dU/dn = 0 (solution z^2) by BiCGSTAB on
    the device. Prints one JSON line."""
    import torch
    from paper_1603_04100_amd import clouds, mvgd as mv
    n, k, kb = args.solve_points, 20, 6
    cl = clouds.hemisphere(n, 8, k)
    m = cl.meta["boundary"]
    dev = "cuda:0"
    print(f"[bench] hemisphere Neumann: N={cl.n_points} K={k} boundary {int(m.sum())}",
          file=sys.stderr, flush=True)
    res = {}
    bmask = torch.tensor(m, device=dev)
    for prec, dt, rtol in (("fp32", torch.float32, 1e-6), ("fp64", torch.float64, 1e-9)):
        P = torch.tensor(cl.points, dtype=dt, device=dev)
        for _ in range(max(1, args.warmup)):
            L, ni, gx, gs = mv.mvgd_assemble_neumann(P, bmask, k, kb)
            mv.mvgd_free(L)
            mv.mvgd_free(mv.mvgd_assemble(P, k))
        torch.cuda.synchronize()
        tn, tp = [], []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            L, ni, gx, gs = mv.mvgd_assemble_neumann(P, bmask, k, kb)
            torch.cuda.synchronize()
            tn.append(time.perf_counter() - t0)
            if _ < args.steps - 1:
                mv.mvgd_free(L)
            t0 = time.perf_counter()
            Lp = mv.mvgd_assemble(P, k)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t0)
            mv.mvgd_free(Lp)
        ng = int(gs.shape[0])
        z = cl.points[~m, 2]
        b = torch.tensor(np.concatenate([7.0 * z ** 2 - 2.0, np.zeros(ng)]), dtype=dt, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = mv.mvgd_solve(L, b, sigma=1.0, rtol=rtol, max_iter=40000, check_every=50)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        err = float((x[:ni].double().cpu() - torch.tensor(z ** 2)).abs().max())
        mv.mvgd_free(L)
        med_n, med_p = float(np.median(tn)), float(np.median(tp))
        res[prec] = {"assemble_neumann_ms": med_n * 1e3, "assemble_plain_ms": med_p * 1e3,
                     "rows_per_s": ni / med_n, "n_interior": ni, "n_ghost": ng,
                     "solve": info, "solve_s": ts, "max_abs_err_vs_z2": err}
        print(f"[bench] {prec}: {res[prec]}", file=sys.stderr, flush=True)
    out = {"metric": "MVGD rows/s with the Neumann condition by reflection (open surface)",
           "value": res["fp32"]["rows_per_s"], "unit": "rows/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["fp32"]["assemble_neumann_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 storage/f64 solves",
           "data": "synthetic", "config": {"workload": "hemisphere_neumann",
                                           "n_points": cl.n_points, "k": k, "k_boundary": kb,
                                           "sigma": 1.0},
           "results": res, "kernel_source_hash": kernel_source_hash()}
    print(json.dumps(out))


def bench_eigs(args):
    """Eigenvalues of -L on a random unit sphere (Sec. 4): the 16 with the smallest real parts by
    the device's Chebyshev-filtered subspace iteration, FP32-mixed and FP64 matrices; errors
    against l (l + 1) as the paper's E_l^inf (l = 1, 2, 3). Prints one JSON line."""
    import torch
    from paper_1603_04100_amd import clouds, mvgd as mv
    n, k = args.eig_points, 20
    cl = clouds.sphere(n, 5, k)
    print(f"[bench] sphere eigenvalues: N={n} K={k}", file=sys.stderr, flush=True)
    exact = np.concatenate([np.full(2 * l + 1, l * (l + 1.0)) for l in range(4)])
    res = {}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        P = torch.tensor(cl.points, dtype=dt, device="cuda:0")
        L = mv.mvgd_assemble(P, k)
        mv.mvgd_eigs(L, 4, max_iter=2)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, info = mv.mvgd_eigs(L, 16, tol=1e-10)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        lr = np.sort(lam.real)
        einf = {f"E{l}_inf": float(np.max(np.abs(lr[l * l:(l + 1) ** 2] - l * (l + 1.0)))
                                    / (l * (l + 1.0))) for l in (1, 2, 3)}
        res[prec] = {"seconds": dt_s, "lambda": [float(x) for x in lr], "max_imag":
                     float(np.abs(lam.imag).max()), **einf, **info}
        print(f"[bench] {prec}: {dt_s:.3f} s, {info}, {einf}", file=sys.stderr, flush=True)
        mv.mvgd_free(L)
    out = {"metric": "seconds for the 16 smallest eigenvalues of -L on the sphere",
           "value": res["fp32"]["seconds"], "unit": "s", "n_gpus": 1,
           "steps": res["fp32"]["iterations"], "warmup": 1,
           "ms_per_step": 1e3 * res["fp32"]["seconds"] / max(res["fp32"]["iterations"], 1),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 matrix/f64 vectors", "data": "synthetic",
           "config": {"workload": "sphere_eigs", "n_points": n, "k": k, "nev": 16, "tol": 1e-10},
           "results": res, "kernel_source_hash": kernel_source_hash()}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="flat_torus4_1m")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the LS / MLS variant timings and row statistics")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--solve-points", type=int, default=1_000_000)
    ap.add_argument("--eig-points", type=int, default=200_000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device copy per step (counter scaling reference)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is described in DESIGN.md and not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1603_04100_amd import mvgd as mv

    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "sphere_poisson":
        return bench_solve(args)
    if args.workload == "hemisphere_neumann":
        return bench_neumann(args)
    if args.workload == "sphere_eigs":
        return bench_eigs(args)
    cl = make_workload(args.workload)
    n, k = cl.n_points, cl.k
    batched = cl.offsets.shape[0] > 2
    offsets = [int(v) for v in cl.offsets] if batched else None
    nrhs = cl.f.shape[1] if batched else 1
    dev = "cuda:0"
    pts32 = cl.points.astype(np.float32)
    P32 = torch.tensor(pts32, device=dev)
    f32 = torch.tensor(np.ascontiguousarray(cl.f[:, :nrhs].astype(np.float32)), device=dev)
    if nrhs == 1:
        f32 = f32.reshape(-1)
    print(f"[bench] {args.workload}: N={n} K={k} n={cl.n_ambient}; warmup {args.warmup}, "
          f"steps {args.steps}", file=sys.stderr, flush=True)
    if args.copy_probe:
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
    flags = mv.MVGD_FLAG_TIME
    # ---------------- FP32-mixed (headline) ----------------
    t32, tk32, y32 = run_gpu(mv, torch, P32, f32, k, args.steps, args.warmup, flags, offsets)
    unbatched = run_unbatched(mv, torch, P32, f32, k, offsets, 0) if batched else None
    if args.copy_probe:
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
    asm32 = float(np.mean([t["assemble_ms"] for t in tk32]))
    bin32 = float(np.mean([t["bin_ms"] for t in tk32]))
    app32 = float(np.mean([t["apply_ms"] for t in tk32]))
    print(f"[bench] fp32-mixed: {t32 * 1e3:.3f} ms/step (bin {bin32:.3f}, assemble kernel "
          f"{asm32:.3f}, apply {app32:.3f} ms)", file=sys.stderr, flush=True)
    # ---------------- FP64 on the same GPU ----------------
    fp64 = None
    if not args.no_fp64 and not batched:
        P64 = torch.tensor(cl.points, device=dev)
        f64 = torch.tensor(cl.f[:, 0], device=dev)
        st64 = max(3, args.steps // 2)
        t64, tk64, y64 = run_gpu(mv, torch, P64, f64, k, st64, min(args.warmup, 2), flags)
        asm64 = float(np.mean([t["assemble_ms"] for t in tk64]))
        fp64 = {"value": n / t64, "ms_per_step": t64 * 1e3, "steps": st64,
                "assemble_kernel_ms": asm64,
                "bin_ms": float(np.mean([t["bin_ms"] for t in tk64])),
                "apply_ms": float(np.mean([t["apply_ms"] for t in tk64]))}
        print(f"[bench] fp64: {t64 * 1e3:.3f} ms/step (assemble kernel {asm64:.3f} ms)",
              file=sys.stderr, flush=True)
        del P64, f64

    # ---------------- discretisation variants and their row sign statistics ----------------
    variants = None
    if not args.no_variants:
        variants = {}
        for name, vf in (("mvgd", 0), ("ls", mv.MVGD_FLAG_LS), ("mvgd_mls", mv.MVGD_FLAG_MLS),
                         ("ls_mls", mv.MVGD_FLAG_LS | mv.MVGD_FLAG_MLS)):
            tv, tkv, _ = run_gpu(mv, torch, P32, f32, k, 3, 1, flags | vf, offsets)
            L = mv.mvgd_assemble(P32, k, flags=vf, cloud_offsets=offsets)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rs = mv.mvgd_row_stats(L)
            t_rs = time.perf_counter() - t0
            mv.mvgd_free(L)
            variants[name] = {"ms_per_step": tv * 1e3,
                              "assemble_kernel_ms": float(np.mean([t["assemble_ms"] for t in tkv])),
                              "m_row_fraction": rs["n_m_rows"] / rs["n_rows"],
                              "mean_neg_ratio": rs["mean_ratio"], "max_neg_ratio": rs["max_ratio"],
                              "diag_negative_fraction": rs["n_diag_negative"] / rs["n_rows"],
                              "row_stats_call_ms": t_rs * 1e3}
            print(f"[bench] variant {name}: {tv * 1e3:.3f} ms/step, M-rows "
                  f"{rs['n_m_rows']}/{rs['n_rows']}, mean neg ratio {rs['mean_ratio']:.4f}",
                  file=sys.stderr, flush=True)

    # ---------------- accuracy against the FP64 oracle + CPU baseline ----------------
    acc, cpu = {}, None
    y32n = y32.cpu().numpy().astype(np.float64).reshape(n, -1)[:, 0]
    acc["max_abs_lf_minus_exact_fp32"] = float(np.abs(y32n - cl.lap_f[:, 0]).max())
    acc["rms_lf_minus_exact_fp32"] = float(np.sqrt(((y32n - cl.lap_f[:, 0]) ** 2).mean()))
    if not args.no_cpu_baseline:
        import oracle
        # the sampled cloud: the whole cloud, or the largest cloud of a batch
        c = int(np.argmax(np.diff(cl.offsets))) if batched else 0
        a, b = int(cl.offsets[c]), int(cl.offsets[c + 1])
        pts_o = pts32[a:b].astype(np.float64)  # the FP32-mixed run's exact input
        rows, ocols, ovals, rps, dt, m = cpu_baseline(oracle, pts_o, k, args.cpu_seconds, 200_000)
        cpu = {"value": rps, "unit": "rows/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": f"{m} random rows of a {b - a}-point cloud of the workload (FP64 oracle: "
                         f"brute-force kNN over all {b - a} points + Householder QR per row), "
                         f"{dt:.1f} s wall"}
        # row parity of the GPU matrix on the sampled rows and L.f error vs the FP64 oracle
        L = mv.mvgd_assemble(P32, k, cloud_offsets=offsets)
        rp, col, val = mv.mvgd_csr(L)
        col = col.cpu().numpy().reshape(n, k + 1)[a:b][rows]
        val = val.cpu().numpy().astype(np.float64).reshape(n, k + 1)[a:b][rows]
        mv.mvgd_free(L)
        ref = (ovals * cl.f[a:b][ocols, 0]).sum(1)
        y32n = y32n[a:b]
        acc["sampled_rows"] = int(m)
        acc["knn_sparsity_identical"] = bool((col == ocols).all())
        acc["max_row_rel_err_fp32"] = float((np.abs(val - ovals).max(1) / np.abs(ovals).max(1)).max())
        acc["lf_rel_err_vs_fp64_oracle_fp32"] = float(np.abs(y32n[rows] - ref).max() / np.abs(ref).max())

    # ---------------- roofline of the dominant kernel ----------------
    s_p, s_v = 4, 4
    bytes_per_row = cl.n_ambient * s_p + (k + 1) * (4 + s_v)
    metric = ("MVGD rows/s at N=1M (FP32-mixed vs FP64), L·f rel err vs FP64 oracle; p99 ms"
              if not batched else
              "MVGD rows/s, batched assembly of many clouds in one launch + apply of 4 RHS")
    achieved = bytes_per_row * n / (asm32 * 1e-3) / 1e9
    from paper_1603_04100_amd import autotune
    tun = autotune.lookup(cl.n_ambient, k, "fp32", n // (cl.offsets.shape[0] - 1))
    search = "search_persistent_kernel" if tun.get("launch", 1) == 2 else "search_kernel"
    smode = {1: 0, 2: 1}.get(tun.get("search", 0), 2)  # default and 3: the tile search
    kernel_name = (f"{search}<float,{cl.n_ambient},{smode}> + "
                   f"fit_kernel<float,{cl.n_ambient},2>")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": counter_traffic(args.workload, "fp32", n),
            "kernel": kernel_name, "kernel_ms": round(asm32, 4),
            "search_ms": round(float(np.mean([t["search_ms"] for t in tk32])), 4),
            "fit_ms": round(float(np.mean([t["fit_ms"] for t in tk32])), 4),
            "algorithmic_bytes_per_row": bytes_per_row}
    dev_step = np.array([t["bin_ms"] + t["assemble_ms"] + t["apply_ms"] for t in tk32])
    out = {
        "metric": metric,
        "value": n / t32, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t32 * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 storage/f64 solves",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_points": n, "k": k, "n_ambient": cl.n_ambient,
                   "precision": "fp32-mixed", "nrhs": nrhs, "step": "assemble+apply",
                   "n_clouds": int(cl.offsets.shape[0] - 1)},
        "unbatched_ms": None if unbatched is None else unbatched * 1e3,
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64": fp64,
        "variants_fp32": variants,
        "kernels_ms": {"bin": bin32, "assemble": asm32, "apply": app32},
        "device_step_ms": {"p50": float(np.percentile(dev_step, 50)),
                           "p99": float(np.percentile(dev_step, 99))},
        "accuracy": acc,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
