"""Seeded generators for the five workload shapes (C1-C5) of the search.

Every array is float64 (coordinates, times, thresholds) or int64 (ids).
Segments of one trajectory are emitted in order; a database is the
concatenation of its trajectories, so the input order is (trajectory,
segment). Nothing here is sorted by time: sorting is the index's job.

Seeds: ``seed_for(k, stream)`` = 14057461 + 100*k + stream, with stream 0
for the database, 1 for the queries and 2 for arrivals / threshold draws.

Workload recipes (the paper measured on its own datasets, which are not
available; these synthetic stand-ins take the paper's shapes, Sec. 7.1 and
Table 1, and the searches S1-S10):

* C1 - 200 trajectories x 100 unit-time segments, t in [0,100], start
  U[0,100]^3, steps U[-1,1] per axis; 10 query trajectories from the same
  generator; d = 2.0; 100 bins.
* C2 - 2,500 x 400 (1M segments, the Galaxy/S1-S2 shape), start U[0,1000]^3,
  Gaussian steps sigma = 1 per axis per unit time; 100 query trajectories
  (40,000 segments); d in {1, 5, 25}; 1,000 bins.
* C3 - 10,000 x 500 (5M segments) on circular orbits in a Plummer sphere
  (scale radius 1, radii resampled above 10), GM = 0.01, vertices at
  t = 0..500 with N(0, 1e-4^2) jitter per axis; 200 query trajectories;
  d in {0.001, 0.01}; 500 bins.
* C4 - the C2 database shape with exponential step lengths (mean 1) in
  uniform directions; 256 query trajectories of log-uniform length in
  [10, 2000] segments of duration 1/8 starting on a 1/64 grid, steps of
  exponential length (mean 1/8); each query trajectory draws its own d
  from {1, 5, 25}.
* C5 - 25,000 x 400 (10M segments) Gaussian walk (the C2 generator);
  requests of log-uniform length in [10, 5000] segments of duration 1/16
  starting on a 1/128 grid, Gaussian steps with variance 1/16 per axis
  (Brownian scaling of the database walk); d log-uniform in [0.5, 50].

Query trajectories are new trajectories from the database's generator, not
members of the database, so no segment is compared with itself.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

BASE_SEED = 14057461


def seed_for(k: int, stream: int) -> int:
    return BASE_SEED + 100 * int(k) + int(stream)


def rng_for(k: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(k, stream)))


FIELDS = ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1")


@dataclass
class Segments:
    """Structure-of-arrays line segments (start point, end point, ids).

    ``d`` is the per-segment distance threshold of a query set (None for a
    database).
    """

    x0: np.ndarray
    y0: np.ndarray
    z0: np.ndarray
    t0: np.ndarray
    x1: np.ndarray
    y1: np.ndarray
    z1: np.ndarray
    t1: np.ndarray
    traj: np.ndarray
    seg: np.ndarray
    d: Optional[np.ndarray] = None
    meta: Dict = field(default_factory=dict)

    def __len__(self) -> int:
        return int(self.t0.shape[0])

    def arrays(self) -> List[np.ndarray]:
        return [getattr(self, f) for f in FIELDS]

    def subset(self, idx) -> "Segments":
        idx = np.asarray(idx)
        return Segments(
            *[np.ascontiguousarray(a[idx]) for a in self.arrays()],
            traj=np.ascontiguousarray(self.traj[idx]),
            seg=np.ascontiguousarray(self.seg[idx]),
            d=None if self.d is None else np.ascontiguousarray(self.d[idx]),
            meta=dict(self.meta),
        )

    def with_d(self, d) -> "Segments":
        out = self.subset(np.arange(len(self)))
        out.d = np.broadcast_to(np.asarray(d, dtype=np.float64), (len(self),)).copy()
        return out


def concat(parts: Sequence[Segments]) -> Segments:
    has_d = all(p.d is not None for p in parts)
    return Segments(
        *[np.concatenate([getattr(p, f) for p in parts]) for f in FIELDS],
        traj=np.concatenate([p.traj for p in parts]),
        seg=np.concatenate([p.seg for p in parts]),
        d=np.concatenate([p.d for p in parts]) if has_d else None,
    )


def from_polylines(verts: np.ndarray, times: np.ndarray, traj_ids=None) -> Segments:
    """Cut (ntraj, L+1, 3) vertices with (ntraj, L+1) times into segments."""
    ntraj, nv, _ = verts.shape
    L = nv - 1
    p0 = verts[:, :-1, :].reshape(-1, 3)
    p1 = verts[:, 1:, :].reshape(-1, 3)
    t0 = times[:, :-1].reshape(-1)
    t1 = times[:, 1:].reshape(-1)
    if traj_ids is None:
        traj_ids = np.arange(ntraj, dtype=np.int64)
    traj = np.repeat(np.asarray(traj_ids, dtype=np.int64), L)
    seg = np.tile(np.arange(L, dtype=np.int64), ntraj)
    c = np.ascontiguousarray
    return Segments(c(p0[:, 0]), c(p0[:, 1]), c(p0[:, 2]), c(t0),
                    c(p1[:, 0]), c(p1[:, 1]), c(p1[:, 2]), c(t1),
                    traj=traj, seg=seg)


def from_ragged(polys: Sequence[np.ndarray], times: Sequence[np.ndarray], traj_ids=None) -> Segments:
    """Like from_polylines for trajectories of different lengths."""
    parts = []
    for i, (v, t) in enumerate(zip(polys, times)):
        tid = i if traj_ids is None else traj_ids[i]
        parts.append(from_polylines(v[None], t[None], [tid]))
    return concat(parts)


# ---------------------------------------------------------------- walkers

def _uniform_dirs(rng, shape):
    v = rng.standard_normal(size=shape + (3,))
    n = np.sqrt((v * v).sum(-1, keepdims=True))
    n[n == 0] = 1.0
    return v / n


def _walk(start: np.ndarray, steps: np.ndarray) -> np.ndarray:
    """start (ntraj,3), steps (ntraj,L,3) -> vertices (ntraj,L+1,3)."""
    out = np.empty((start.shape[0], steps.shape[1] + 1, 3))
    out[:, 0] = start
    np.cumsum(steps, axis=1, out=out[:, 1:])
    out[:, 1:] += start[:, None, :]
    return out


def uniform_walk(rng, ntraj, L, box, step):
    start = rng.uniform(0.0, box, size=(ntraj, 3))
    steps = rng.uniform(-step, step, size=(ntraj, L, 3))
    times = np.broadcast_to(np.arange(L + 1, dtype=np.float64), (ntraj, L + 1))
    return from_polylines(_walk(start, steps), times)


def gaussian_walk(rng, ntraj, L, box, sigma):
    start = rng.uniform(0.0, box, size=(ntraj, 3))
    steps = rng.normal(0.0, sigma, size=(ntraj, L, 3))
    times = np.broadcast_to(np.arange(L + 1, dtype=np.float64), (ntraj, L + 1))
    return from_polylines(_walk(start, steps), times)


def exp_walk(rng, ntraj, L, box, mean_step):
    start = rng.uniform(0.0, box, size=(ntraj, 3))
    lens = rng.exponential(mean_step, size=(ntraj, L, 1))
    steps = lens * _uniform_dirs(rng, (ntraj, L))
    times = np.broadcast_to(np.arange(L + 1, dtype=np.float64), (ntraj, L + 1))
    return from_polylines(_walk(start, steps), times)


def plummer_orbits(rng, ntraj, L, a=1.0, rmax=10.0, gm=0.01, jitter=1e-4):
    """Circular orbits with radii drawn from a Plummer density profile."""
    r = np.empty(ntraj)
    todo = np.arange(ntraj)
    while todo.size:
        X = rng.uniform(0.0, 1.0, size=todo.size)
        with np.errstate(divide="ignore", invalid="ignore"):
            rr = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        ok = np.isfinite(rr) & (rr <= rmax)
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    normal = _uniform_dirs(rng, (ntraj,))
    # orthonormal basis (u, w) of each orbital plane
    helper = np.where(np.abs(normal[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    u = np.cross(normal, helper)
    u /= np.sqrt((u * u).sum(-1, keepdims=True))
    w = np.cross(normal, u)
    phase = rng.uniform(0.0, 2 * np.pi, size=ntraj)
    omega = np.sqrt(gm / (r * r + a * a) ** 1.5)
    t = np.arange(L + 1, dtype=np.float64)
    ang = phase[:, None] + omega[:, None] * t[None, :]
    verts = r[:, None, None] * (np.cos(ang)[..., None] * u[:, None, :] + np.sin(ang)[..., None] * w[:, None, :])
    verts += rng.normal(0.0, jitter, size=verts.shape)
    times = np.broadcast_to(t, (ntraj, L + 1))
    return from_polylines(verts, times)


def short_queries(rng, ntraj, lmin, lmax, dt, grid, t_end, box, step_kind, step_scale):
    """Query trajectories of log-uniform length with sub-unit segment times."""
    lens = np.rint(np.exp(rng.uniform(np.log(lmin), np.log(lmax), size=ntraj))).astype(np.int64)
    lens = np.clip(lens, lmin, lmax)
    polys, times = [], []
    for L in lens:
        span = L * dt
        nslots = int(np.floor((t_end - span) / grid))
        start_t = grid * rng.integers(0, nslots + 1)
        p = rng.uniform(0.0, box, size=3)
        if step_kind == "exp":
            st = rng.exponential(step_scale, size=(L, 1)) * _uniform_dirs(rng, (int(L),))
        else:
            st = rng.normal(0.0, step_scale, size=(int(L), 3))
        v = np.concatenate([p[None], p[None] + np.cumsum(st, axis=0)], axis=0)
        polys.append(v)
        times.append(start_t + dt * np.arange(L + 1, dtype=np.float64))
    out = from_ragged(polys, times)
    out.meta["lengths"] = lens
    return out


# ---------------------------------------------------------------- configs

CONFIGS = {
    "C1": dict(k=1, ntraj=200, L=100, nq=10, d=(2.0,), bins=100),
    "C2": dict(k=2, ntraj=2500, L=400, nq=100, d=(1.0, 5.0, 25.0), bins=1000),
    "C3": dict(k=3, ntraj=10000, L=500, nq=200, d=(0.001, 0.01), bins=500),
    "C4": dict(k=4, ntraj=2500, L=400, nq=256, d=(1.0, 5.0, 25.0), bins=1000),
    "C5": dict(k=5, ntraj=25000, L=400, nq=None, d=(0.5, 50.0), bins=4000),
}


def make_db(name: str, ntraj: Optional[int] = None, L: Optional[int] = None) -> Segments:
    c = CONFIGS[name]
    k = c["k"]
    ntraj = c["ntraj"] if ntraj is None else ntraj
    L = c["L"] if L is None else L
    rng = rng_for(k, 0)
    if name == "C1":
        return uniform_walk(rng, ntraj, L, 100.0, 1.0)
    if name in ("C2", "C5"):
        return gaussian_walk(rng, ntraj, L, 1000.0, 1.0)
    if name == "C3":
        return plummer_orbits(rng, ntraj, L)
    if name == "C4":
        return exp_walk(rng, ntraj, L, 1000.0, 1.0)
    raise KeyError(name)


def make_queries(name: str, d=None, nq: Optional[int] = None, L: Optional[int] = None,
                 request: int = 0) -> Segments:
    """Query segments of a config, with their per-segment threshold ``d``.

    C1-C3 take one scalar ``d`` (default: the config's first value). C4 draws
    one d per query trajectory from the config's set. C5 builds request
    number ``request`` (one query trajectory with its own d).
    """
    c = CONFIGS[name]
    k = c["k"]
    if name == "C5":
        rng = np.random.Generator(np.random.PCG64([seed_for(k, 1), int(request)]))
        q = short_queries(rng, 1, 10, 5000, 1.0 / 16, 1.0 / 128, 400.0, 1000.0, "gauss", 0.25)
        dlo, dhi = c["d"]
        dv = float(np.exp(rng.uniform(np.log(dlo), np.log(dhi))))
        q = q.with_d(dv)
        q.meta["request"] = int(request)
        return q
    nq = c["nq"] if nq is None else nq
    rng = rng_for(k, 1)
    if name == "C4":
        q = short_queries(rng, nq, 10, 2000, 1.0 / 8, 1.0 / 64, 400.0, 1000.0, "exp", 1.0 / 8)
        rd = rng_for(k, 2)
        per_traj = rd.choice(np.asarray(c["d"]), size=nq)
        return q.with_d(per_traj[q.traj])
    L = c["L"] if L is None else L
    if name == "C1":
        q = uniform_walk(rng, nq, L, 100.0, 1.0)
    elif name == "C2":
        q = gaussian_walk(rng, nq, L, 1000.0, 1.0)
    elif name == "C3":
        q = plummer_orbits(rng, nq, L)
    else:
        raise KeyError(name)
    return q.with_d(c["d"][0] if d is None else d)


def make_config(name: str, d=None, **kw):
    """(database, queries, number of bins) of a config."""
    db = make_db(name, ntraj=kw.get("ntraj"), L=kw.get("L"))
    q = make_queries(name, d=d, nq=kw.get("nq"), L=kw.get("qL", kw.get("L")))
    return db, q, CONFIGS[name]["bins"]
