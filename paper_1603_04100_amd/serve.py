"""Serving loop: assemble + apply requests arriving over time, with continuous batching.

Each request is one point cloud (host memory) with R right-hand sides; the answer is L f for each
of them. A dispatcher (the calling thread) admits and batches requests; one worker thread per HIP
stream serves the batches:

* admission: a request is admitted when its estimated device footprint fits in the HBM budget
  that is still free (a batch's matrix and vectors stay resident until its results are back);
* continuous batching: whenever a worker is idle, every admitted request that is waiting (up to
  ``max_batch``) goes to it as one batch: ONE batched mvgd_assemble call (one launch over all
  their clouds) and ONE mvgd_apply with nrhs = R. Requests that arrive meanwhile wait for the next
  idle worker, so their work overlaps with the batches already on the device;
* workers: each owns a stream, page-locked staging buffers and device buffers that grow on demand
  and are reused, so a batch costs one host copy per request into staging (with the cast to the
  serving precision), one upload, the two library calls and one download. The library calls and
  the copies release the interpreter lock, and a worker blocked in the assembly's single
  synchronisation does not hold up the dispatcher or the other workers;
* completion: a HIP event per batch; latency runs from arrival until the worker has seen the event
  complete and copied the results out.

``one_at_a_time`` is the plain baseline: the same requests, one worker, no batching, FP64.
"""
from __future__ import annotations

import collections
import gc
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import mvgd as mv


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    points: np.ndarray      # [N, n] (host; cast to the serving precision when staged)
    rhs: np.ndarray         # [N, R]
    k: int
    result: np.ndarray | None = None
    done: float | None = None
    dispatched: float | None = None
    batch: int = -1


def footprint_bytes(n_points: int, n_ambient: int, k: int, nrhs: int, vsize: int) -> int:
    """Device bytes a request holds while in flight: points, sliced ELL (columns + values),
    permutation, assembly scratch (sorted points, keys, slots, inverse permutation, cell table),
    right-hand sides, results and the apply staging buffer."""
    ell = n_points * (k + 1) * (4 + vsize)
    scratch = n_points * (4 * vsize + 16 + 8 * 4)
    vectors = 3 * n_points * nrhs * vsize
    return n_ambient * n_points * vsize + ell + 4 * n_points + scratch + vectors


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else 0.0


@dataclass
class Stats:
    latencies_ms: list = field(default_factory=list)
    queue_ms: list = field(default_factory=list)     # arrival -> handed to a worker
    service_ms: list = field(default_factory=list)   # handed to a worker -> results on the host
    batches: int = 0
    batch_sizes: list = field(default_factory=list)
    rows: int = 0
    wall_s: float = 0.0
    admission_waits: int = 0

    def summary(self) -> dict:
        lat = self.latencies_ms or [0.0]
        return {"requests": len(self.latencies_ms), "p50_ms": _pct(lat, 50),
                "p99_ms": _pct(lat, 99), "mean_ms": float(np.mean(lat)),
                "max_ms": float(np.max(lat)),
                "queue_p50_ms": _pct(self.queue_ms, 50), "queue_p99_ms": _pct(self.queue_ms, 99),
                "service_p50_ms": _pct(self.service_ms, 50),
                "service_p99_ms": _pct(self.service_ms, 99), "batches": self.batches,
                "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
                "rows": self.rows, "wall_s": self.wall_s,
                "req_per_s": len(self.latencies_ms) / max(self.wall_s, 1e-9),
                "rows_per_s": self.rows / max(self.wall_s, 1e-9),
                "admission_waits": self.admission_waits}


def _grow(buf: dict, name: str, numel: int, pinned: bool, dtype, device, stream) -> torch.Tensor:
    """Buffer `name` of at least `numel` elements (page-locked host or device memory), grown by
    at least 25% when it is too small. Only called between batches of its worker."""
    t = buf.get(name)
    if t is None or t.numel() < numel:
        cap = max(numel, int(1.25 * (t.numel() if t is not None else 0)), 1 << 16)
        if pinned:
            t = torch.empty(cap, dtype=dtype, pin_memory=True)
        else:
            with torch.cuda.stream(stream):
                t = torch.empty(cap, dtype=dtype, device=device)
        buf[name] = t
    return t


class _Worker(threading.Thread):
    """Serves one batch at a time on its own stream, with reusable staging and device buffers."""

    def __init__(self, server: "Server", idx: int):
        super().__init__(name=f"mvgd-serve-{idx}", daemon=True)
        self.server = server
        self.stream = server.streams[idx]
        self.buf = server.buffers[idx]  # kept by the server across runs
        self.inbox: queue.Queue = queue.Queue()
        self.ev = torch.cuda.Event()

    def _buffer(self, name: str, numel: int, pinned: bool) -> torch.Tensor:
        return _grow(self.buf, name, numel, pinned, self.server.dtype, self.server.device,
                     self.stream)

    def run(self):
        torch.cuda.set_device(self.server.device)
        while True:
            item = self.inbox.get()
            if item is None:
                return
            t0, batch = item
            try:
                self._serve(batch)
            except BaseException as e:  # reported by the dispatcher
                self.server._errors.append(e)
            self.server._done.put((self, batch))

    def _serve(self, batch):
        srv = self.server
        na, nrhs = batch[0].points.shape[1], batch[0].rhs.shape[1]
        sizes = [r.points.shape[0] for r in batch]
        offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        n = int(offs[-1])
        hp = self._buffer("hp", n * na, True)
        hr = self._buffer("hr", n * nrhs, True)
        ho = self._buffer("ho", n * nrhs, True)
        hp_np, hr_np, ho_np = hp.numpy(), hr.numpy(), ho.numpy()
        for j, r in enumerate(batch):  # copy + cast into page-locked staging
            a, b = int(offs[j]), int(offs[j + 1])
            hp_np[a * na:b * na].reshape(b - a, na)[...] = r.points
            hr_np[a * nrhs:b * nrhs].reshape(b - a, nrhs)[...] = r.rhs
        dp = self._buffer("dp", n * na, False)
        dr = self._buffer("dr", n * nrhs, False)
        do = self._buffer("do", n * nrhs, False)
        with torch.cuda.stream(self.stream):
            dp[:n * na].copy_(hp[:n * na], non_blocking=True)
            dr[:n * nrhs].copy_(hr[:n * nrhs], non_blocking=True)
            L = mv.mvgd_assemble(dp[:n * na].view(n, na), batch[0].k,
                                 cloud_offsets=[int(v) for v in offs], stream=self.stream)
            try:
                mv.mvgd_apply(L, dr[:n * nrhs].view(n, nrhs), y=do[:n * nrhs].view(n, nrhs),
                              stream=self.stream)
                ho[:n * nrhs].copy_(do[:n * nrhs], non_blocking=True)
                self.ev.record(self.stream)
                self.ev.synchronize()
            finally:
                mv.mvgd_free(L)
        out = ho_np[:n * nrhs].reshape(n, nrhs)
        tdone = time.perf_counter() - srv._t0
        for j, r in enumerate(batch):
            r.result = out[offs[j]:offs[j + 1]].astype(np.float64)
            r.done = tdone


class Server:
    def __init__(self, precision: str = "fp32", n_streams: int = 4, max_batch: int = 16,
                 hbm_budget_bytes: int = 64 << 30, device: str = "cuda:0"):
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.vsize = 4 if precision == "fp32" else 8
        self.device = device
        self.max_batch = max_batch
        self.budget = hbm_budget_bytes
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.buffers = [{} for _ in range(n_streams)]
        self._done: queue.Queue = queue.Queue()
        self._errors: list = []
        self._t0 = 0.0

    def reserve(self, n_points: int, n_ambient: int = 3, nrhs: int = 8):
        """Pre-size every worker's staging and device buffers for batches of n_points points."""
        for buf, stream in zip(self.buffers, self.streams):
            for name, numel in (("hp", n_points * n_ambient), ("hr", n_points * nrhs),
                                ("ho", n_points * nrhs)):
                _grow(buf, name, numel, True, self.dtype, self.device, stream)
                _grow(buf, "d" + name[1], numel, False, self.dtype, self.device, stream)
        torch.cuda.synchronize()

    def _fp(self, r: Request) -> int:
        return footprint_bytes(r.points.shape[0], r.points.shape[1], r.k, r.rhs.shape[1],
                               self.vsize)

    def run(self, requests: list[Request], batching: bool = True) -> Stats:
        """Serve requests (sorted by arrival) in real time; returns latency statistics. The
        interpreter's cyclic garbage collector is paused meanwhile (a full collection stops every
        thread, the dispatcher included)."""
        workers = [_Worker(self, i) for i in range(len(self.streams))]
        for w in workers:
            w.start()
        gc_was_on = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, batching, workers)
        finally:
            for w in workers:
                w.inbox.put(None)
            for w in workers:
                w.join()
            if gc_was_on:
                gc.enable()

    def _run(self, requests, batching, workers) -> Stats:
        st = Stats()
        self._errors = []
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        idle = list(workers)
        busy = 0
        used = 0
        torch.cuda.synchronize()
        self._t0 = t0 = time.perf_counter()
        while pending or waiting or busy:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # completions
            while True:
                try:
                    w, batch = self._done.get_nowait()
                except queue.Empty:
                    break
                busy -= 1
                idle.append(w)
                for r in batch:
                    used -= self._fp(r)
                    st.latencies_ms.append((r.done - r.arrival) * 1e3 if r.done is not None
                                           else float("nan"))
                    st.queue_ms.append((r.dispatched - r.arrival) * 1e3)
                    st.service_ms.append(((r.done or r.dispatched) - r.dispatched) * 1e3)
                    st.rows += r.points.shape[0]
            if self._errors:
                while busy:
                    self._done.get()
                    busy -= 1
                raise self._errors[0]
            # admission + dispatch to idle workers
            while idle and waiting:
                batch, need = [], 0
                limit = self.max_batch if batching else 1
                while waiting and len(batch) < limit:
                    b = self._fp(waiting[0])
                    if used + need + b > self.budget and (batch or busy):
                        st.admission_waits += 1
                        break
                    batch.append(waiting.popleft())
                    need += b
                if not batch:
                    break
                tdisp = time.perf_counter() - t0
                for r in batch:
                    r.batch = st.batches
                    r.dispatched = tdisp
                used += need
                busy += 1
                idle.pop().inbox.put((tdisp, batch))
                st.batches += 1
                st.batch_sizes.append(len(batch))
            # wait for a completion or the next arrival (requests still waiting here are held
            # back by admission or by busy workers: only a completion can release them)
            now = time.perf_counter() - t0
            timeout = 0.002
            if pending:
                timeout = max(0.0, min(timeout, pending[0].arrival - now))
            if busy and timeout > 0:
                try:
                    self._done.put(self._done.get(timeout=timeout))  # handled at the loop top
                except queue.Empty:
                    pass
            elif timeout > 0:
                time.sleep(timeout)
        st.wall_s = time.perf_counter() - t0
        return st


def one_at_a_time(requests: list[Request], precision: str = "fp64") -> Stats:
    """Baseline: one worker, one request at a time, no batching (FP64 by default)."""
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
