"""Serving loop: a resident index answering a stream of query requests.

Requests (one query trajectory each, with its own d) arrive over time. The
scheduler admits waiting requests while the estimated result-buffer bytes of
everything in flight fit a fixed pool (the paper's point that concurrent
users compete for GPU memory, and that result memory must be reserved ahead
of the kernel, Sec. 3 and Sec. 5), groups the admitted requests into one
query batch (continuous batching: requests that arrive while others run join
the next batch), and keeps `streams` batches in flight on separate HIP
streams so their work overlaps on the device. Each request records its
arrival, admission and completion times.

Result bytes are estimated as in the paper's performance model (Sec. 8):
the hit fraction alpha is tracked per temporal epoch (50 epochs over the
database's time extent), and a query segment's expected hits are alpha of
its epoch times its number of candidate entries (computed on the host from
the bin table). Alpha is updated from every completed batch, and a waiting
request is estimated again each time a batch is formed. The device memory
each executor's query handle holds (its buffers grow and are kept) counts
against the pool too: a batch is admitted on an executor when the other
executors' holdings (or their in-flight estimates, if larger) plus the
larger of this executor's holding and the batch's estimate fit. A batch whose
estimate is too small still completes: the library re-runs the pair kernel
with a larger buffer. The library's native scheduler (tds_server_*, the
NativeServer binding) follows the same policy; this one keeps it in Python
for host tests with the oracle standing in for the GPU.
"""
from __future__ import annotations

import collections
import gc
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import api

HIT_BYTES = 24
FIELDS = ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1")


@dataclass
class Request:
    rid: int
    seg: object                 # x0..t1 host arrays
    d: np.ndarray               # per-segment threshold
    arrival: float = 0.0        # seconds after the start of the run
    t_admit: float = -1.0
    t_done: float = -1.0
    est_bytes: float = 0.0
    n_eval: int = 0
    n_overlap: int = 0
    hits: Optional[api.Hits] = None   # caller indices within this request

    @property
    def n(self) -> int:
        return int(np.asarray(self.seg.t0).shape[0])

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class AlphaModel:
    """Hit fraction per temporal epoch (exponential moving average)."""

    def __init__(self, t_first: float, t_last: float, epochs: int = 50, prior: float = 1e-4,
                 smoothing: float = 0.5):
        self.t0, self.t1, self.epochs = t_first, t_last, epochs
        self.alpha = np.full(epochs, prior)
        self.smoothing = smoothing

    def epoch(self, t0) -> np.ndarray:
        span = max(self.t1 - self.t0, 1e-300)
        e = np.floor((np.asarray(t0) - self.t0) / span * self.epochs)
        return np.clip(e, 0, self.epochs - 1).astype(np.int64)

    def expected_hits(self, t0, n_eval) -> float:
        return float(np.sum(self.alpha[self.epoch(t0)] * n_eval))

    def update(self, t0, n_eval, hits_per_seg):
        ep = self.epoch(t0)
        ev = np.bincount(ep, weights=n_eval, minlength=self.epochs)
        hv = np.bincount(ep, weights=hits_per_seg, minlength=self.epochs)
        seen = ev > 0
        a = np.where(seen, hv / np.maximum(ev, 1), self.alpha)
        self.alpha = np.where(seen, self.smoothing * self.alpha + (1 - self.smoothing) * a, self.alpha)


class GpuExecutor:
    """Runs one query batch on its own query handle and HIP stream."""

    def __init__(self, index: api.Index, opts: Dict):
        import torch
        self.qh = api.Query(index)
        self.stream = torch.cuda.Stream()
        self.opts = dict(opts)

    def __call__(self, seg, d, capacity: int):
        self.qh.batch(seg, d, capacity=capacity, stream=self.stream, **self.opts)
        h = self.qh.fetch(out="host")
        return h, self.qh.stats()

    def device_bytes(self) -> int:
        """Device memory the executor's query handle holds (kept between batches)."""
        return self.qh.device_bytes()

    def close(self):
        self.qh.close()


def _concat(reqs: Sequence[Request]):
    class Seg:
        pass

    s = Seg()
    for f in FIELDS:
        setattr(s, f, np.concatenate([np.asarray(getattr(r.seg, f)) for r in reqs]))
    d = np.concatenate([np.broadcast_to(r.d, (r.n,)) for r in reqs]).astype(np.float64)
    return s, d


class Server:
    """Admission + continuous batching over `streams` in-flight batches."""

    def __init__(self, index: api.Index, pool_bytes: float = 64e6, streams: int = 2,
                 max_batch_segments: int = 1 << 20, k_safety: float = 4.0,
                 opts: Optional[Dict] = None, executor_factory: Optional[Callable] = None,
                 alpha: Optional[AlphaModel] = None):
        info = index.info() if index is not None else {"t_first": 0.0, "t_last": 1.0}
        self.bins = index.bins() if index is not None else None
        self.pool_bytes = float(pool_bytes)
        self.streams = int(streams)
        self.max_batch_segments = int(max_batch_segments)
        self.k_safety = float(k_safety)
        self.alpha = alpha or AlphaModel(info["t_first"], info["t_last"])
        opts = dict(opts or dict(mode="fp32_refine", tiling="range"))
        factory = executor_factory or (lambda: GpuExecutor(index, opts))
        self.executors = [factory() for _ in range(self.streams)]
        self.lock = threading.Lock()
        self.in_flight_bytes = 0.0
        # device bytes each executor's handle holds after its last batch
        # (buffers grow and are kept); counted against the pool with the
        # estimates of the batches in flight
        self.reserved = [0.0] * self.streams
        self.in_flight = [0.0] * self.streams
        self.batches: List[Dict] = []

    # -------------------------------------------------------------- planning
    def plan(self, r: Request):
        """Candidate counts per segment and the request's estimated result bytes."""
        if self.bins is not None:
            f, l = api.plan_ranges(self.bins, r.seg.t0, r.seg.t1)
            r._n_eval_seg = np.maximum(l - f + 1, 0).astype(np.float64)
        else:
            r._n_eval_seg = np.zeros(r.n)
        r.n_eval = int(r._n_eval_seg.sum())
        self.estimate(r)

    def estimate(self, r: Request):
        """Estimated result bytes of a planned request under the current alpha."""
        r.est_bytes = HIT_BYTES * self.k_safety * max(1.0, self.alpha.expected_hits(r.seg.t0, r._n_eval_seg))

    # -------------------------------------------------------------- running
    def warmup(self, requests: Sequence[Request], reserve_segments: int = 0) -> None:
        """Run the requests once on every executor, untimed and unrecorded.

        Grows each query handle's device buffers to the sizes these requests
        need, so that a measured run does not pay first-use allocations
        (a buffer that grows is freed with hipFree, which waits for the whole
        device, the other executors' batches included). With
        reserve_segments, one more batch repeats the requests' segments up to
        that many, so batches of up to that size find their buffers grown.
        Last, the requests are served four times over through the admission
        loop at staggered arrivals, so that the worker threads' first calls
        into the runtime also happen here: a first measured run otherwise
        showed fetches of 6-7 ms on small batches that later runs in the same
        process did not.
        The hit-rate estimates learnt here are kept; the batch log is not.
        """
        for k, ex in enumerate(self.executors):
            for r in requests:
                self.plan(r)
                cap = int(r.est_bytes / HIT_BYTES) + 1024
                ex(r.seg, np.broadcast_to(r.d, (r.n,)).astype(np.float64), cap)
            # one batch of all of them with the whole pool as capacity: the
            # device buffers reach the sizes the largest admitted batch needs
            if requests:
                seg, d = _concat(list(requests))
                ex(seg, d, int(self.pool_bytes / HIT_BYTES) + 1024)
                n = len(d)
                if reserve_segments > n:
                    reps = -(-int(reserve_segments) // n)
                    big = type(seg)()
                    for f in FIELDS:
                        setattr(big, f, np.tile(getattr(seg, f), reps)[:reserve_segments])
                    ex(big, np.tile(d, reps)[:reserve_segments], int(self.pool_bytes / HIT_BYTES) + 1024)
            if hasattr(ex, "device_bytes"):
                self.reserved[k] = float(ex.device_bytes())
        if requests:
            replay = [Request(rid=k, seg=r.seg, d=r.d, arrival=2e-4 * k)
                      for k, r in enumerate(list(requests) * 4)]
            self.run(replay)
        self.batches.clear()

    def run(self, requests: Sequence[Request], time_scale: float = 1.0) -> Dict:
        """Serve requests at their arrival times (seconds x time_scale).

        The objects alive at the start are moved out of the garbage
        collector's generations for the run (gc.freeze), so its collections
        only walk what the run itself allocates.
        """
        gc.collect()
        gc.freeze()
        try:
            return self._run(requests, time_scale)
        finally:
            gc.unfreeze()

    def _run(self, requests: Sequence[Request], time_scale: float) -> Dict:
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            self.plan(r)
        pending: collections.deque = collections.deque()
        free_exec: "queue.Queue[int]" = queue.Queue()
        for i in range(self.streams):
            free_exec.put(i)
        done_evt = threading.Event()
        n_done = [0]
        threads: List[threading.Thread] = []
        start = time.perf_counter()
        now = lambda: time.perf_counter() - start  # noqa: E731
        errors: List[BaseException] = []

        def work(ei: int, batch: List[Request], cap_bytes: float):
            try:
                seg, d = _concat(batch)
                cap = int(cap_bytes / HIT_BYTES) + 1024
                t_launch = now()
                h, st = self.executors[ei](seg, d, cap)
                t_end = now()
                off = np.cumsum([0] + [r.n for r in batch])
                hq = np.asarray(h.query)
                order = np.argsort(hq, kind="stable")
                hq_sorted = hq[order]
                hits_seg = np.bincount(hq, minlength=off[-1]).astype(np.float64)
                for k, r in enumerate(batch):
                    a, b = np.searchsorted(hq_sorted, [off[k], off[k + 1]])
                    sel = order[a:b]
                    r.hits = api.Hits(hq[sel] - off[k], np.asarray(h.entry)[sel], np.asarray(h.traj)[sel],
                                      np.asarray(h.ta)[sel], np.asarray(h.tb)[sel])
                    r.t_done = t_end
                dev = getattr(self.executors[ei], "device_bytes", None)
                with self.lock:
                    t0_all = np.concatenate([np.asarray(r.seg.t0) for r in batch])
                    ev_all = np.concatenate([r._n_eval_seg for r in batch])
                    self.alpha.update(t0_all, ev_all, hits_seg)
                    self.in_flight_bytes -= cap_bytes
                    self.in_flight[ei] = 0.0
                    if dev is not None:
                        self.reserved[ei] = float(dev())
                    self.batches.append(dict(n_req=len(batch), n_seg=int(off[-1]), hits=len(hq),
                                             t_launch=t_launch, t_end=t_end, retries=st["retries"],
                                             ms_pair=st.get("ms_pair", 0.0)))
                    n_done[0] += len(batch)
                    if n_done[0] == len(reqs):
                        done_evt.set()
            except BaseException as exc:  # surfaced by run()
                errors.append(exc)
                done_evt.set()
            finally:
                free_exec.put(ei)

        i = 0
        while n_done[0] < len(reqs) and not errors:
            t = now()
            while i < len(reqs) and reqs[i].arrival * time_scale <= t:
                pending.append(reqs[i])
                i += 1
            launched = False
            if pending:
                try:
                    ei = free_exec.get_nowait()
                except queue.Empty:
                    ei = None
                if ei is not None:
                    batch, nseg, nbytes = [], 0, 0.0
                    with self.lock:
                        # the other executors hold their buffers, or more
                        # while a batch of theirs is in flight; this one
                        # needs the larger of its buffers and the estimate
                        others = sum(max(self.reserved[x], self.in_flight[x])
                                     for x in range(self.streams) if x != ei)
                        while pending:
                            r = pending[0]
                            # waiting requests are re-estimated with the alpha
                            # the batches completed so far have updated
                            self.estimate(r)
                            need = max(self.reserved[ei], nbytes + r.est_bytes)
                            fits = (others + need <= self.pool_bytes
                                    or not batch and self.in_flight_bytes == 0)
                            if not fits or (batch and nseg + r.n > self.max_batch_segments):
                                break
                            pending.popleft()
                            batch.append(r)
                            nseg += r.n
                            nbytes += r.est_bytes
                        if batch:
                            self.in_flight_bytes += nbytes
                            self.in_flight[ei] = nbytes
                    if batch:
                        ta = now()
                        for r in batch:
                            r.t_admit = ta
                        th = threading.Thread(target=work, args=(ei, batch, nbytes), daemon=True)
                        th.start()
                        threads.append(th)
                        launched = True
                    else:
                        free_exec.put(ei)
            if not launched:
                nxt = reqs[i].arrival * time_scale - now() if i < len(reqs) else 1e-3
                time.sleep(min(max(nxt, 0.0), 2e-4) if pending or i < len(reqs) else 1e-3)
        for th in threads:
            th.join()
        if errors:
            raise errors[0]
        wall = now()
        lat = np.array([r.latency for r in reqs])
        wait = np.array([r.t_admit - r.arrival for r in reqs])
        service = np.array([r.t_done - r.t_admit for r in reqs])
        return dict(n_requests=len(reqs), wall_s=wall, p50_ms=float(np.percentile(lat, 50) * 1e3),
                    p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                    p99_wait_ms=float(np.percentile(wait, 99) * 1e3),
                    p99_service_ms=float(np.percentile(service, 99) * 1e3),
                    n_batches=len(self.batches),
                    mean_batch_requests=float(np.mean([b["n_req"] for b in self.batches])),
                    retries=int(sum(b["retries"] for b in self.batches)))

    def close(self):
        for e in self.executors:
            if hasattr(e, "close"):
                e.close()


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process with `rate` requests per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
