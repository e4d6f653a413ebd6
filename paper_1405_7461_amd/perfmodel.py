"""Response-time model of the search (Sec. 8), measured on the device it runs on.

The paper predicts a query's response time from a GPU component and a CPU
component. GPU component (Sec. 8.1): a batch with i interactions over c
candidate entries takes

    T(i, c) = T1(alpha i, c) + T2(beta i, c) + T3(gamma i, c) - 2 Theta(i, c)

where T1, T2 and T3 are the times of batches whose interactions are all
hits, all temporal misses, and all temporal hits but spatial misses, Theta
the time of a batch with no work (each of the three terms contains it), alpha
the hit fraction (estimated per temporal epoch by sampling), beta the
temporal-miss fraction (exact, from the candidate ranges and the sorted time
arrays) and gamma = 1 - alpha - beta. T1..T3 and Theta are read off
benchmark curves (time against interactions, one curve per candidate count
c) by linear interpolation in i along the two curves that bracket c, then
linearly in c. CPU component (Sec. 8.2): a fitted curve a + b q^e for the
host work that scales with the query segments (the transfer of the
host inputs) and sigma / bandwidth for returning sigma result bytes.

Differences from the paper's setting: one call here is one persistent
launch over all tiles of the batch (the paper's sum over kernel invocations
of size s becomes one term with c = i / q, q the segments with candidates),
and the benchmark curves are measured with device-resident inputs and
outputs, so Theta holds the fixed per-call cost (launches, counter readback,
synchronisation) and the CPU component only what host memory adds.

``calibrate`` runs the four synthetic benchmarks on the GPU;
``estimate_alpha`` follows the paper's sampling of alpha per epoch;
``PerfModel.predict`` evaluates the model for a batch of query segments
without running it.
"""
from __future__ import annotations

import json
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import api

HIT_BYTES_HOST = 40          # one tds_hit record in host memory
QUERY_BYTES_HOST = 9 * 8     # eight coordinates and d per query segment


# ------------------------------------------------------------ interpolation

def _along(xs: np.ndarray, ys: np.ndarray, x: float) -> float:
    """Piecewise-linear value of one benchmark curve at x; beyond its ends the
    outermost segment is extended."""
    n = xs.shape[0]
    if n == 1:
        return float(ys[0])
    j = int(np.clip(np.searchsorted(xs, x, side="right") - 1, 0, n - 2))
    w = (x - xs[j]) / (xs[j + 1] - xs[j])
    return float(ys[j] * (1.0 - w) + ys[j + 1] * w)


def lookup(curves: Dict[float, Tuple[np.ndarray, np.ndarray]], i: float, c: float) -> float:
    """Time at (i interactions, c candidates): the bracketing c curves read at
    i, blended linearly in c; c outside the measured range takes the
    nearest curve."""
    keys = np.array(sorted(curves), dtype=np.float64)
    if c <= keys[0]:
        return _along(*curves[float(keys[0])], i)
    if c >= keys[-1]:
        return _along(*curves[float(keys[-1])], i)
    j = int(np.searchsorted(keys, c, side="right") - 1)
    lo, hi = float(keys[j]), float(keys[j + 1])
    w = (c - lo) / (hi - lo)
    return (1.0 - w) * _along(*curves[lo], i) + w * _along(*curves[hi], i)


# ------------------------------------------------------------------- model

@dataclass
class CpuFit:
    a: float = 0.0        # ms
    b: float = 0.0        # ms
    e: float = 1.0
    d2h_bytes_per_ms: float = 2.0e7

    def ms(self, q: float, sigma_bytes: float, host_inputs: bool, host_output: bool) -> float:
        t = (self.a + self.b * max(q, 1.0) ** self.e) if host_inputs else 0.0
        return max(t, 0.0) + (sigma_bytes / self.d2h_bytes_per_ms if host_output else 0.0)


@dataclass
class PerfModel:
    tables: Dict[str, Dict[float, Tuple[np.ndarray, np.ndarray]]]
    cpu: CpuFit = field(default_factory=CpuFit)
    alpha: Optional[np.ndarray] = None       # per epoch
    t_first: float = 0.0
    t_last: float = 1.0
    tile_ms: float = 0.0                     # cost of one more tile in the launch
    sort_ms: Tuple[float, float] = (0.0, 0.0)  # a + b q: the t_start sort of Periodic and greedy

    # Sec. 8.1
    def gpu_ms(self, alpha: float, beta: float, i: float, c: float) -> float:
        gamma = max(0.0, 1.0 - alpha - beta)
        return (lookup(self.tables["hit"], alpha * i, c) + lookup(self.tables["tmiss"], beta * i, c)
                + lookup(self.tables["smiss"], gamma * i, c) - 2.0 * lookup(self.tables["noop"], i, c))

    def epoch_of(self, t0) -> np.ndarray:
        n = len(self.alpha)
        span = max(self.t_last - self.t_first, 1e-300)
        e = np.floor((np.asarray(t0, dtype=np.float64) - self.t_first) / span * n)
        return np.clip(e, 0, n - 1).astype(np.int64)

    def predict(self, index: "api.Index", q, tiling="range", batch_size: int = 128,
                host_inputs=False, host_output=False) -> Dict:
        """Predicted response time (ms) of one call for query segments q."""
        w = workload_terms(index, q, tiling, batch_size)
        if self.alpha is None:
            raise ValueError("estimate alpha first (estimate_alpha)")
        a_seg = self.alpha[self.epoch_of(np.asarray(q.t0))]
        hits = float(np.sum(a_seg * w["seg_interactions"]))
        i = w["interactions"]
        alpha = hits / i if i else 0.0
        beta = 1.0 - w["n_overlap"] / i if i else 0.0
        c = i / max(w["q_active"], 1)
        g = self.gpu_ms(alpha, beta, i, c) if i else lookup(self.tables["noop"], 0.0, 1.0)
        # the benchmark batches are one tile each; every further tile of the
        # launch costs tile_ms (the counterpart of the paper's per-invocation
        # overhead summed over batches)
        g += self.tile_ms * max(w["n_tiles"] - 1, 0)
        # Periodic and the greedy tilings also sort their segments by t_start
        if tiling != "range":
            g += max(0.0, self.sort_ms[0] + self.sort_ms[1] * w["q_active"])
        cpu = self.cpu.ms(len(q.t0), hits * HIT_BYTES_HOST, host_inputs, host_output)
        return dict(ms=g + cpu, gpu_ms=g, cpu_ms=cpu, alpha=alpha, beta=beta, gamma=1 - alpha - beta,
                    interactions=i, c=c, expected_hits=hits, n_tiles=w["n_tiles"])

    def to_json(self) -> str:
        t = {k: {str(c): [list(map(float, x)), list(map(float, y))] for c, (x, y) in v.items()}
             for k, v in self.tables.items()}
        return json.dumps(dict(tables=t, cpu=self.cpu.__dict__,
                               alpha=None if self.alpha is None else list(map(float, self.alpha)),
                               t_first=self.t_first, t_last=self.t_last, tile_ms=self.tile_ms,
                               sort_ms=list(self.sort_ms)))

    @staticmethod
    def from_json(s: str) -> "PerfModel":
        d = json.loads(s)
        t = {k: {float(c): (np.array(x), np.array(y)) for c, (x, y) in v.items()}
             for k, v in d["tables"].items()}
        return PerfModel(t, CpuFit(**d["cpu"]), None if d["alpha"] is None else np.array(d["alpha"]),
                         d["t_first"], d["t_last"], d.get("tile_ms", 0.0),
                         tuple(d.get("sort_ms", (0.0, 0.0))))


# ------------------------------------------------- interactions and beta

def workload_terms(index: "api.Index", q, tiling="range", batch_size: int = 128) -> Dict:
    """Interactions, exactly overlapping pairs and per-segment interactions of
    a batch, on the host from the index's bins (no kernel runs).

    range tiling: each segment meets its own candidate range. Periodic:
    consecutive runs of batch_size segments with candidates, in (t_start,
    caller index) order as the device walks them, meet the candidate range of
    their temporal extent (smallest t_start to largest t_end, Sec. 4).
    """
    t0 = np.asarray(q.t0, dtype=np.float64)
    t1 = np.asarray(q.t1, dtype=np.float64)
    bins = index.bins()
    first, last = api.plan_ranges(bins, t0, t1)
    size = np.where(last >= first, last - first + 1, 0).astype(np.float64)
    active = size > 0
    if tiling == "periodic":
        order = np.argsort(t0, kind="stable")
        order = order[active[order]]
        seg_int = np.zeros_like(size)
        starts = np.arange(0, order.size, batch_size)
        if starts.size:
            lo_t = t0[order[starts]]
            hi_t = np.maximum.reduceat(t1[order], starts)
            gf, gl = api.plan_ranges(bins, lo_t, hi_t)
            for k, s in enumerate(starts):
                seg_int[order[s:s + batch_size]] = gl[k] - gf[k] + 1
        interactions = float(seg_int.sum())
        n_tiles = -(-order.size // batch_size)
    else:
        seg_int = size
        interactions = float(size.sum())
        n_tiles = int(np.unique(np.stack([first[active], last[active]]), axis=1).shape[1]) if active.any() else 0
    st0, st1 = index.sorted_times()
    n_ovl = float((np.searchsorted(st0, t1, side="left") - np.searchsorted(st1, t0, side="right")).sum())
    return dict(interactions=interactions, n_overlap=n_ovl, seg_interactions=seg_int,
                q_active=int(active.sum()), n_tiles=int(n_tiles))


# ------------------------------------------------------------- benchmarks

class _Seg:
    pass


def _segments(x0, y0, z0, t0, x1, y1, z1, t1, d):
    s = _Seg()
    c = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    s.x0, s.y0, s.z0, s.t0, s.x1, s.y1, s.z1, s.t1 = map(c, (x0, y0, z0, t0, x1, y1, z1, t1))
    s.d = c(d)
    s.traj = np.arange(len(s.t0), dtype=np.int64)
    return s


def _entries(kind: str, c: int, rng) -> "_Seg":
    """c entries in one temporal bin. "near": spans [0, 1] within 0.1 of the
    origin; "split": spans alternate between [0, 0.5] and [0.95, 1.0] (a query
    over (0.6, 0.9) overlaps the bin but none of them), spread over a box of
    side 1000 as the temporal misses of a real candidate range are (the
    binary32 filter tests space only, so temporal misses next to the query
    would all go to the refine, which real ones rarely do)."""
    p = rng.uniform(-0.05, 0.05, size=(c, 3))
    if kind == "split":
        p = rng.uniform(-500.0, 500.0, size=(c, 3))
    v = rng.uniform(-0.05, 0.05, size=(c, 3))
    if kind == "near":
        t0, t1 = np.zeros(c), np.ones(c)
    else:
        early = np.arange(c) % 2 == 0
        t0 = np.where(early, 0.0, 0.95)
        t1 = np.where(early, 0.5, 1.0)
    return _segments(p[:, 0], p[:, 1], p[:, 2], t0, p[:, 0] + v[:, 0], p[:, 1] + v[:, 1],
                     p[:, 2] + v[:, 2], t1, np.zeros(c))


def _queries(kind: str, q: int, rng) -> "_Seg":
    """q query segments of one benchmark kind (all pairs of one class)."""
    p = rng.uniform(-0.05, 0.05, size=(q, 3))
    if kind == "hit":        # overlap [0, 1], within 0.3 of every entry, d = 1
        t0, t1, off, d = 0.0, 1.0, 0.0, 1.0
    elif kind == "tmiss":    # (0.6, 0.9): inside the bin, outside every entry's span
        t0, t1, off, d = 0.6, 0.9, 0.0, 1.0
    elif kind == "smiss":    # overlap in time, 1000 away in space
        t0, t1, off, d = 0.0, 1.0, 1000.0, 1.0
    else:                    # noop: after the index's time extent, no candidates
        t0, t1, off, d = 10.0, 11.0, 0.0, 1.0
    x = p[:, 0] + off
    return _segments(x, p[:, 1], p[:, 2], np.full(q, t0), x, p[:, 1], p[:, 2], np.full(q, t1),
                     np.full(q, d))


def _to_device(s):
    import torch
    out = _Seg()
    for f in ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1", "d"):
        setattr(out, f, torch.as_tensor(getattr(s, f), device="cuda"))
    out.traj = s.traj
    return out


def _time_call(qh, qs, opts, reps, out="device"):
    import torch
    stream = torch.cuda.current_stream()
    ts = []
    hits = 0
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qh.batch(qs, qs.d, stream=stream, **opts)
        h = qh.fetch(out=out)
        torch.cuda.synchronize()
        if r:
            ts.append((time.perf_counter() - t0) * 1e3)
        hits = len(h)
    return float(np.median(ts)), hits


def calibrate(qs: Sequence[int] = (256, 2048, 16384, 131072),
              cs: Sequence[int] = (256, 1024, 4096, 16384, 65536),
              reps: int = 5, max_hits: int = 1 << 22, opts: Optional[Dict] = None,
              seed: int = 0, log=None) -> PerfModel:
    """Measure T1 (all hits), T2 (all temporal misses), T3 (all spatial
    misses) and Theta (no candidates) over a grid of query counts q and
    candidate counts c, and fit the CPU component. Hit benchmarks with more
    than max_hits results are skipped (their curve extends linearly)."""
    import torch
    opts = dict(opts or dict(mode="fp32_refine", tiling="range", block_size=256))
    rng = np.random.default_rng(seed)
    tables: Dict[str, Dict[float, Tuple[list, list]]] = {k: {} for k in ("hit", "tmiss", "smiss", "noop")}
    for c in cs:
        for ent_kind, kinds in (("near", ("hit", "smiss", "noop")), ("split", ("tmiss",))):
            ix = api.build_index(_entries(ent_kind, c, rng), 1)
            qh = api.Query(ix)
            try:
                for kind in kinds:
                    xs, ys = [], []
                    for q in qs:
                        if kind == "hit" and q * c > max_hits:
                            continue
                        dq = _to_device(_queries(kind, q, rng))
                        ms, hits = _time_call(qh, dq, opts, reps)
                        want = q * c if kind == "hit" else 0
                        if hits != want:
                            raise RuntimeError(f"benchmark {kind} q={q} c={c}: {hits} hits, expected {want}")
                        xs.append(float(q * c))
                        ys.append(ms)
                        if log:
                            log(f"calibrate {kind:5s} c={c:6d} q={q:6d}: {ms:.4f} ms")
                    tables[kind][float(c)] = (np.array(xs), np.array(ys))
            finally:
                qh.close()
                ix.close()
    # CPU component: host inputs and host output against the device-resident call
    ix = api.build_index(_entries("near", cs[0], rng), 1)
    qh = api.Query(ix)
    try:
        qv, dt = [], []
        for q in list(qs) + [4 * qs[-1]]:
            hq = _queries("noop", q, rng)
            ms_host, _ = _time_call(qh, hq, opts, reps, out="host")
            ms_dev, _ = _time_call(qh, _to_device(hq), opts, reps)
            qv.append(float(q))
            dt.append(max(ms_host - ms_dev, 1e-4))
        a, b, e = _fit_power(np.array(qv), np.array(dt))
    finally:
        qh.close()
        ix.close()
    bw = _d2h_bandwidth()
    tile_ms = _tile_cost(opts, rng, reps)
    sort_ms = _sort_cost(opts, rng, reps)
    out = {k: {c: (np.array(x), np.array(y)) for c, (x, y) in v.items()} for k, v in tables.items()}
    return PerfModel(out, CpuFit(a, b, e, bw), tile_ms=tile_ms, sort_ms=sort_ms)


def _sort_cost(opts: Dict, rng, reps: int, qs: Sequence[int] = (16384, 131072),
               m: int = 1024) -> Tuple[float, float]:
    """Extra preparation of the tilings that sort by t_start: query segments
    spread over m t_start bins (entries one per unit of time, far from every
    query: no hits), the preparation stage's event time under Periodic minus
    that under range tiling, as a + b q through the two query counts."""
    import torch
    k = np.arange(m, dtype=np.float64)
    far = 1000.0 + 10.0 * k
    z = np.zeros(m)
    ix = api.build_index(_segments(far, z, z, k, far, z, z, k + 1.0, np.ones(m)), m)
    qh = api.Query(ix)
    stream = torch.cuda.current_stream()
    try:
        diff = []
        for q in qs:
            t0 = rng.uniform(0.0, m - 1.0, size=q)
            p = rng.uniform(-0.05, 0.05, size=(q, 3))
            dq = _to_device(_segments(p[:, 0], p[:, 1], p[:, 2], t0, p[:, 0], p[:, 1], p[:, 2], t0 + 0.5,
                                      np.ones(q)))
            prep = {}
            for tiling in ("range", "periodic"):
                ts = []
                for r in range(reps + 1):
                    qh.batch(dq, dq.d, stream=stream, timing=True, **dict(opts, tiling=tiling, batch_size=128))
                    qh.fetch(out="device")
                    if r:
                        ts.append(qh.stats()["ms_prep"])
                prep[tiling] = float(np.median(ts))
            diff.append(prep["periodic"] - prep["range"])
        b = (diff[1] - diff[0]) / (qs[1] - qs[0])
        return (diff[0] - b * qs[0], b)
    finally:
        qh.close()
        ix.close()


def _tile_cost(opts: Dict, rng, reps: int, q: int = 131072, c: int = 1024) -> float:
    """Cost of one more tile: spatial-miss batches whose segments share one
    range, cut into q / s Periodic tiles, against the same batch in the
    fewest Periodic tiles (the same preparation, sort included)."""
    ix = api.build_index(_entries("near", c, rng), 1)
    qh = api.Query(ix)
    try:
        dq = _to_device(_queries("smiss", q, rng))
        s_max = 65536
        base, _ = _time_call(qh, dq, dict(opts, tiling="periodic", batch_size=s_max), reps)
        xs, ys = [], []
        for s in (16, 64, 256, 1024):
            ms, _ = _time_call(qh, dq, dict(opts, tiling="periodic", batch_size=s), reps)
            xs.append(float(-(-q // s) - -(-q // s_max)))
            ys.append(ms - base)
        xs, ys = np.array(xs), np.array(ys)
        return max(float(np.dot(xs, ys) / np.dot(xs, xs)), 0.0)  # slope through the origin
    finally:
        qh.close()
        ix.close()


def _fit_power(q: np.ndarray, t: np.ndarray) -> Tuple[float, float, float]:
    """Least squares a + b q^e over a grid of exponents (e in [0.2, 1.5])."""
    best = None
    for e in np.linspace(0.2, 1.5, 131):
        A = np.column_stack([np.ones_like(q), q ** e])
        coef, res, *_ = np.linalg.lstsq(A, t, rcond=None)
        r = float(np.sum((A @ coef - t) ** 2))
        if best is None or r < best[0]:
            best = (r, float(coef[0]), float(coef[1]), float(e))
    return best[1], best[2], best[3]


def _d2h_bandwidth(nbytes: int = 64 << 20) -> float:
    """Device-to-host copy rate into pinned memory, bytes per ms."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 3 * nbytes / ((time.perf_counter() - t0) * 1e3)


# ------------------------------------------------------------------ alpha

def estimate_alpha(model: PerfModel, index: "api.Index", rep_queries, num_epochs: int = 50,
                   s: int = 256, tol: float = 0.05, max_rounds: int = 8, seed: int = 0,
                   opts: Optional[Dict] = None) -> Dict:
    """Sec. 8.1's alpha per temporal epoch: for each epoch, batches of s
    consecutive (in t_start order) query segments of a representative query
    set that start in the epoch are run and their hit fraction recorded;
    rounds of samples are added until the hits the estimates predict for the
    whole representative set are within tol of its true hit count."""
    opts = dict(opts or dict(mode="fp32_refine", tiling="range"))
    info = index.info()
    model.t_first, model.t_last = info["t_first"], info["t_last"]
    model.alpha = np.zeros(num_epochs)
    rng = np.random.default_rng(seed)
    t0 = np.asarray(rep_queries.t0)
    order = np.argsort(t0, kind="stable")
    ep_sorted = model.epoch_of(t0[order])
    w = workload_terms(index, rep_queries)
    qh = api.Query(index)
    try:
        qh.batch(rep_queries, rep_queries.d, **opts)
        true_hits = len(qh.fetch())
        hits_e = np.zeros(num_epochs)
        ints_e = np.zeros(num_epochs)
        err = np.inf
        rounds = 0
        for rounds in range(1, max_rounds + 1):
            for e in range(num_epochs):
                pos = np.nonzero(ep_sorted == e)[0]
                if pos.size == 0:
                    continue
                start = int(rng.integers(0, max(pos.size - s, 0) + 1))
                sel = order[pos[start:start + s]]
                sub = _subset(rep_queries, sel)
                qh.batch(sub, sub.d, **opts)
                hits_e[e] += len(qh.fetch())
                ints_e[e] += qh.stats()["n_eval"]
            model.alpha = np.where(ints_e > 0, hits_e / np.maximum(ints_e, 1), 0.0)
            pred = float(np.sum(model.alpha[model.epoch_of(t0)] * w["seg_interactions"]))
            err = abs(pred - true_hits) / max(true_hits, 1)
            if err <= tol:
                break
    finally:
        qh.close()
    return dict(rounds=rounds, rel_error=err, true_hits=true_hits)


def _subset(s, idx):
    out = _Seg()
    for f in ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1", "d"):
        out.__dict__[f] = np.ascontiguousarray(np.asarray(getattr(s, f))[idx])
    out.traj = np.asarray(getattr(s, "traj", np.arange(len(s.t0))))[idx]
    return out
