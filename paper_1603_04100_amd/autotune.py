"""Autotuner for the neighbour-search tunables of mvgd_assemble.

The tunables change only performance, never results (the neighbour search is exact):

* cell_alpha       grid cell edge relative to the estimated K-th neighbour distance
* radius_mu        initial search radius relative to the same estimate
* cells_per_point  cell-table budget per point (finer grids cost a larger table)
* launch           1 = one workgroup per 64-point group, 2 = persistent per-XCD work queues
* search           1 = the group's queries stream their common cell box, 2 = every query walks
                   its own box, 3 = as 1 with the distances from the matrix cores

``tune`` times the assembly kernel (HIP events recorded by the library on its stream) over a
grid of settings on a given workload and returns the fastest. ``main`` tunes the named
workloads and merges the winners into ``tuning.json`` next to this file, keyed by ambient
dimension, K, precision and log2 of the points per cloud; ``lookup`` (used by mvgd_assemble when
no tuning is passed) returns the entry of the nearest size for the same (n, K, precision).
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(_HERE, "tuning.json")

GRID = {
    "cell_alpha": (0.45, 0.6, 0.8, 1.0),
    "radius_mu": (1.4, 1.7, 2.0),
    "cells_per_point": (4.0, 8.0, 16.0),
    "launch": (1, 2),
    "search": (1, 2, 3),
}

_table = None


def _key(n_ambient: int, k: int, precision: str, d_manifold: int = 2) -> str:
    return f"n{n_ambient}_k{k}_{precision}" if d_manifold == 2 else \
        f"n{n_ambient}_d{d_manifold}_k{k}_{precision}"


def _load() -> dict:
    global _table
    if _table is None:
        try:
            with open(TABLE) as f:
                _table = json.load(f)
        except (OSError, ValueError):
            _table = {}
    return _table


def lookup(n_ambient: int, k: int, precision: str, points_per_cloud: int,
           d_manifold: int = 2) -> dict:
    """Tuned settings for this shape (nearest log2 size), or {} for the library defaults."""
    entries = _load().get(_key(n_ambient, k, precision, d_manifold), {})
    if not entries:
        return {}
    b = math.log2(max(points_per_cloud, 1))
    best = min(entries, key=lambda s: abs(float(s) - b))
    return dict(entries[best]["settings"])


def tune(points, k: int, cloud_offsets=None, reps: int = 3, grid: dict | None = None,
         verbose: bool = False, d_manifold: int = 2):
    """Time the assembly kernel over the settings grid; return (best settings, all results)."""
    import torch
    from . import mvgd as mv

    grid = grid or GRID
    names = list(grid)
    results = []
    for combo in itertools.product(*(grid[n] for n in names)):
        settings = dict(zip(names, combo))
        times = []
        for r in range(reps + 1):
            L = mv.mvgd_assemble(points, k, cloud_offsets=cloud_offsets, tuning=settings,
                                 flags=mv.MVGD_FLAG_TIME, d_manifold=d_manifold)
            t = mv.mvgd_timing(L)
            mv.mvgd_free(L)
            if r > 0:  # first run warms the allocator pool
                times.append(t["bin_ms"] + t["assemble_ms"])
        ms = sorted(times)[len(times) // 2]
        results.append((ms, settings))
        if verbose:
            print(f"  {settings} -> {ms:.3f} ms", flush=True)
    torch.cuda.synchronize()
    results.sort(key=lambda x: x[0])
    return results[0][1], results


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workloads", nargs="+",
                    default=["flat_torus4_1m", "torus_200k", "sphere_2k", "ellipsoids_256",
                             "circle_100k"])
    ap.add_argument("--precisions", nargs="+", default=["fp32", "fp64"])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()

    import numpy as np
    import torch
    from . import clouds

    table = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            table = json.load(f)
    for name in args.workloads:
        cl = clouds.config(name)
        offs = None if cl.offsets.shape[0] == 2 else [int(v) for v in cl.offsets]
        per_cloud = cl.n_points // (cl.offsets.shape[0] - 1)
        for prec in args.precisions:
            dt = torch.float32 if prec == "fp32" else torch.float64
            P = torch.tensor(cl.points.astype(np.float32 if prec == "fp32" else np.float64),
                             device="cuda:0")
            d = cl.meta.get("d", 2)
            best, res = tune(P, cl.k, cloud_offsets=offs, reps=args.reps, d_manifold=d)
            default_ms = next(ms for ms, s in res if s == {"cell_alpha": 0.6, "radius_mu": 1.7,
                                                           "cells_per_point": 8.0, "launch": 1,
                                                           "search": 1})
            print(f"[autotune] {name} {prec}: best {res[0][0]:.3f} ms {best} "
                  f"(defaults {default_ms:.3f} ms)", flush=True)
            key = _key(cl.n_ambient, cl.k, prec, d)
            table.setdefault(key, {})[f"{math.log2(per_cloud):.2f}"] = {
                "settings": best, "ms": res[0][0], "default_ms": default_ms, "workload": name,
                "points_per_cloud": per_cloud}
            del P
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"[autotune] wrote {args.out}")


if __name__ == "__main__":
    main()
