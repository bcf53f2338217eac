"""Serving loop: assemble + apply requests arriving over time, with continuous batching.

Each request is one point cloud (host memory) with R right-hand sides; the answer is L f for each
of them. The loop runs on one host thread and drives the C ABI on several HIP streams:

* admission: a request is admitted when its estimated device footprint fits in the HBM budget
  that is still free (matrices of requests in flight stay resident until their applies finish);
* continuous batching: whenever a stream slot is free, every admitted request that is waiting
  (up to ``max_batch``) is uploaded and assembled together in ONE batched mvgd_assemble call
  (one launch over all their clouds) and their right-hand sides are applied in ONE mvgd_apply
  with nrhs = R; requests that arrive meanwhile wait for the next free slot, so their work
  overlaps with the batches already on the device;
* completion: a HIP event per batch; results are copied back and latency is measured from
  arrival to the moment the host sees the event complete.

``one_at_a_time`` is the plain baseline: the same requests, one stream, no batching, FP64.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import mvgd as mv


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    points: np.ndarray      # [N, n] float64 (host)
    rhs: np.ndarray         # [N, R] float64 (host)
    k: int
    result: np.ndarray | None = None
    done: float | None = None
    batch: int = -1


def footprint_bytes(n_points: int, n_ambient: int, k: int, nrhs: int, vsize: int) -> int:
    """Device bytes a request holds while in flight: points, sliced ELL (columns + values),
    permutation, assembly scratch (sorted points, keys, slots, inverse permutation, cell table),
    right-hand sides, results and the apply staging buffer."""
    ell = n_points * (k + 1) * (4 + vsize)
    scratch = n_points * (4 * vsize + 16 + 8 * 4)
    vectors = 3 * n_points * nrhs * vsize
    return n_ambient * n_points * vsize + ell + 4 * n_points + scratch + vectors


@dataclass
class Stats:
    latencies_ms: list = field(default_factory=list)
    batches: int = 0
    batch_sizes: list = field(default_factory=list)
    rows: int = 0
    wall_s: float = 0.0
    admission_waits: int = 0

    def summary(self) -> dict:
        lat = np.array(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {"requests": len(self.latencies_ms), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "max_ms": float(lat.max()), "batches": self.batches,
                "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
                "rows": self.rows, "wall_s": self.wall_s,
                "req_per_s": len(self.latencies_ms) / max(self.wall_s, 1e-9),
                "rows_per_s": self.rows / max(self.wall_s, 1e-9),
                "admission_waits": self.admission_waits}


class Server:
    def __init__(self, precision: str = "fp32", n_streams: int = 4, max_batch: int = 16,
                 hbm_budget_bytes: int = 64 << 30, device: str = "cuda:0"):
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.vsize = 4 if precision == "fp32" else 8
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.max_batch = max_batch
        self.budget = hbm_budget_bytes

    def _launch(self, batch, stream):
        """Upload, assemble (batched) and apply one batch on `stream`; returns the in-flight
        record."""
        offs = np.concatenate([[0], np.cumsum([r.points.shape[0] for r in batch])]).astype(np.int64)
        pts = np.concatenate([r.points for r in batch]).astype(
            np.float32 if self.precision == "fp32" else np.float64)
        rhs = np.concatenate([r.rhs for r in batch]).astype(pts.dtype)
        with torch.cuda.stream(stream):
            P = torch.from_numpy(pts).pin_memory().to(self.device, non_blocking=True)
            X = torch.from_numpy(np.ascontiguousarray(rhs)).pin_memory().to(self.device,
                                                                          non_blocking=True)
            L = mv.mvgd_assemble(P, batch[0].k, cloud_offsets=list(offs), stream=stream)
            Y = mv.mvgd_apply(L, X, stream=stream)
            Yh = torch.empty(Y.shape, dtype=Y.dtype, pin_memory=True)
            Yh.copy_(Y, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return {"batch": batch, "L": L, "keep": (P, X, Y), "Yh": Yh, "ev": ev, "offs": offs,
                "stream": stream, "bytes": sum(self._fp(r) for r in batch)}

    def _fp(self, r: Request) -> int:
        return footprint_bytes(r.points.shape[0], r.points.shape[1], r.k, r.rhs.shape[1],
                               self.vsize)

    def run(self, requests: list[Request], batching: bool = True) -> Stats:
        """Serve requests (sorted by arrival) in real time; returns latency statistics."""
        st = Stats()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        inflight = []
        free = list(self.streams)
        used = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # completions
            for rec in list(inflight):
                if rec["ev"].query():
                    tdone = time.perf_counter() - t0
                    Yh = rec["Yh"].numpy()
                    for j, r in enumerate(rec["batch"]):
                        r.result = Yh[rec["offs"][j]:rec["offs"][j + 1]].astype(np.float64)
                        r.done = tdone
                        st.latencies_ms.append((tdone - r.arrival) * 1e3)
                        st.rows += r.points.shape[0]
                    mv.mvgd_free(rec["L"])
                    used -= rec["bytes"]
                    free.append(rec["stream"])
                    inflight.remove(rec)
            # admission + launch into free slots
            while free and waiting:
                batch, need = [], 0
                limit = self.max_batch if batching else 1
                while waiting and len(batch) < limit:
                    r = waiting[0]
                    b = self._fp(r)
                    if used + need + b > self.budget and (batch or inflight):
                        st.admission_waits += 1
                        break
                    batch.append(waiting.popleft())
                    need += b
                if not batch:
                    break
                rec = self._launch(batch, free.pop())
                for r in batch:
                    r.batch = st.batches
                used += rec["bytes"]
                inflight.append(rec)
                st.batches += 1
                st.batch_sizes.append(len(batch))
            if not (pending and pending[0].arrival <= time.perf_counter() - t0):
                if inflight and not free:
                    time.sleep(0.0002)
                elif not waiting and pending and not inflight:
                    time.sleep(max(0.0, min(0.001, pending[0].arrival - (time.perf_counter() - t0))))
        st.wall_s = time.perf_counter() - t0
        return st


def one_at_a_time(requests: list[Request], precision: str = "fp64") -> Stats:
    """Baseline: one stream, one request at a time, no batching (FP64 by default)."""
    return Server(precision=precision, n_streams=1, max_batch=1).run(requests, batching=False)


def make_requests(duration_s: float = 3.0, rate_hz: float = 200.0, seed: int = 5, k: int = 24,
                  n_min: int = 5000, n_max: int = 500_000, n_apply: int = 8,
                  max_requests: int | None = None) -> list[Request]:
    from . import clouds
    out = []
    for d in clouds.serving_stream(duration_s=duration_s, rate_hz=rate_hz, seed=seed, k=k,
                                   n_min=n_min, n_max=n_max, n_apply=n_apply,
                                   max_requests=max_requests):
        out.append(Request(d["id"], d["arrival"], d["points"], d["rhs"], d["k"]))
    return out
