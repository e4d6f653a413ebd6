"""Small seeded geometric fixtures for correctness tests.

Each function only places segment endpoints; the expected outcomes are
derived in the tests (closed forms, exact rationals, invariants).
"""
from __future__ import annotations

import numpy as np

from .workloads import Segments, from_polylines, from_ragged, concat, BASE_SEED


def _rng(tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([BASE_SEED, tag]))


def segments_from_rows(rows, traj=None) -> Segments:
    """rows: (n, 8) array of x0,y0,z0,t0,x1,y1,z1,t1."""
    r = np.asarray(rows, dtype=np.float64).reshape(-1, 8)
    n = r.shape[0]
    c = np.ascontiguousarray
    return Segments(*[c(r[:, i]) for i in range(8)],
                    traj=np.arange(n, dtype=np.int64) if traj is None else np.asarray(traj, np.int64),
                    seg=np.zeros(n, dtype=np.int64))


def time_only(t0, t1, seed=1) -> Segments:
    """Segments with the given time extents and arbitrary positions."""
    rng = _rng(seed)
    t0 = np.asarray(t0, dtype=np.float64)
    t1 = np.asarray(t1, dtype=np.float64)
    p0 = rng.uniform(0, 10, size=(t0.size, 3))
    p1 = p0 + rng.uniform(-1, 1, size=(t0.size, 3))
    rows = np.column_stack([p0, t0, p1, t1])
    return segments_from_rows(rows)


def random_small(n_e=60, n_q=12, box=4.0, step=1.5, seed=2, d=1.0, tmax=6.0):
    """Tiny random sets with random (non-grid) times, dense enough for hits."""
    rng = _rng(seed)

    def mk(n):
        t0 = rng.uniform(0, tmax, size=n)
        t1 = t0 + rng.uniform(0.05, 2.0, size=n)
        p0 = rng.uniform(0, box, size=(n, 3))
        p1 = p0 + rng.uniform(-step, step, size=(n, 3))
        return segments_from_rows(np.column_stack([p0, t0, p1, t1]))

    db = mk(n_e)
    q = mk(n_q).with_d(d)
    return db, q


def dense_box(ntraj=40, L=30, box=3.0, nq=6, seed=3, d=0.8):
    """Random walks on the unit time grid inside a tiny box: many hits."""
    rng = _rng(seed)

    def walk(n):
        start = rng.uniform(0, box, size=(n, 3))
        steps = rng.uniform(-0.5, 0.5, size=(n, L, 3))
        v = np.concatenate([start[:, None], start[:, None] + np.cumsum(steps, axis=1)], axis=1)
        t = np.broadcast_to(np.arange(L + 1, dtype=np.float64), (n, L + 1))
        return from_polylines(v, t)

    return walk(ntraj), walk(nq).with_d(d)


def all_hit(n_e=256, n_q=16, seed=4):
    """Every temporally overlapping pair is also a spatial hit.

    All points sit still at the same place; only the time extents vary.
    """
    rng = _rng(seed)

    def mk(n):
        t0 = rng.integers(0, 8, size=n).astype(np.float64)
        t1 = t0 + rng.integers(1, 4, size=n)
        p = np.full((n, 3), 1.25)
        return segments_from_rows(np.column_stack([p, t0, p, t1]))

    return mk(n_e), mk(n_q).with_d(0.5)


def stationary_pairs(d=1.0):
    """Query and entry with exactly equal velocity at fixed offsets.

    All values are dyadic, so positions, velocities and offsets are exact in
    binary64: the offsets are 0.5 d, d (exactly at the threshold), 1.5 d and
    0 along x.
    """
    qs, es, kinds = [], [], []
    offsets = [(0.5 * d, "in"), (d, "edge"), (1.5 * d, "out"), (0.0, "in")]
    for i, (h, kind) in enumerate(offsets):
        v = np.array([0.25, -0.5, 0.125]) * i
        p = np.array([1.0, 2.0, 3.0])
        qs.append([*p, 0.0, *(p + 4 * v), 4.0])
        e0 = p + np.array([h, 0.0, 0.0]) - v
        es.append([*e0, -1.0, *(e0 + 5 * v), 4.0])
        kinds.append(kind)
    return segments_from_rows(es), segments_from_rows(qs).with_d(d), kinds


def passing_pairs(seed=5, n=64):
    """Stationary entry at a random point; query passes on a straight line.

    Query travels from c + h*w - 5*s*u to c + h*w + 5*s*u over [t0, t0+10];
    the entry stays at c over a window covering it. With speed s and offset h
    the pair is within d exactly when |t - (t0+5)| <= sqrt(d^2 - h^2)/s.
    Parameters are returned for the closed form.
    """
    rng = _rng(seed)
    rows_q, rows_e, params = [], [], []
    for _ in range(n):
        c = rng.uniform(-50, 50, size=3)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        w = np.cross(u, rng.standard_normal(3))
        w /= np.linalg.norm(w)
        s = rng.uniform(0.1, 3.0)
        d = rng.uniform(0.5, 4.0)
        h = rng.uniform(0.0, 1.3) * d
        t0 = float(rng.integers(-20, 20))
        a = c + h * w - 5 * s * u
        b = c + h * w + 5 * s * u
        rows_q.append([*a, t0, *b, t0 + 10.0])
        te0 = t0 - float(rng.integers(0, 3))
        rows_e.append([*c, te0, *c, t0 + 10.0 + float(rng.integers(0, 3))])
        params.append(dict(c=c, u=u, w=w, s=s, d=d, h=h, t0=t0))
    return segments_from_rows(rows_e), segments_from_rows(rows_q), params


def near_threshold(seed=6, d=1.0, ks=range(4, 53, 4), per_k=4, scale=100.0):
    """Pairs whose constructed closest approach is d*(1 +/- 2^-k).

    Both segments move; the relative motion is a straight pass with its
    closest point inside the common time window. Endpoints are rounded to
    binary64, so the true minimum distance is only close to the constructed
    one; the exact value comes from exact rational arithmetic in the tests.
    """
    rng = _rng(seed)
    rows_q, rows_e, tags = [], [], []
    for k in ks:
        for sgn in (-1.0, 1.0):
            for _ in range(per_k):
                h = d * (1.0 + sgn * 2.0 ** (-k))
                u = rng.standard_normal(3)
                u /= np.linalg.norm(u)
                w = np.cross(u, rng.standard_normal(3))
                w /= np.linalg.norm(w)
                e0 = rng.uniform(-scale, scale, size=3)
                ev = rng.uniform(-2, 2, size=3)
                t0 = float(rng.uniform(0, 10))
                T = float(rng.uniform(1, 4))
                frac = float(rng.uniform(0.2, 0.8))
                spd = float(rng.uniform(0.2, 3.0))
                # relative offset at time t0 + frac*T is h*w
                rel0 = h * w - spd * frac * T * u
                rel1 = h * w + spd * (1 - frac) * T * u
                e1 = e0 + ev * T
                rows_e.append([*e0, t0, *e1, t0 + T])
                rows_q.append([*(e0 + rel0), t0, *(e1 + rel1), t0 + T])
                tags.append((k, sgn))
    return segments_from_rows(rows_e), segments_from_rows(rows_q).with_d(d), tags


def comb_bins(n_gaps=40, per_bin=6, reps=3, seed=7, box=3.0, d=1.5):
    """Bins of very uneven extent: bin 0 holds one entry spanning the whole
    time axis [0, n_gaps + 1] (so its extent covers every later bin), every
    later unit bin k holds short entries inside [k, k + 0.3]. Query segments
    come in groups of `reps` identical spans (k + 0.5, k + 0.6) in the gaps
    between the short bins, plus a few random spans. A gap query overlaps
    bin 0 only, so all gap queries share one candidate range, while the
    extent of two neighbouring gap groups also overlaps the short bin
    between them: identical ranges whose merge is not free (Sec. 6, Alg. 4's
    first pass). Times are multiples of 0.05, exact enough in binary64 for
    strict comparisons to be unambiguous."""
    rng = _rng(seed)
    T = float(n_gaps + 1)
    rows = []
    p = rng.uniform(0, box, 3)
    rows.append([*p, 0.0, *(p + rng.uniform(-1, 1, 3)), T])
    for k in range(1, n_gaps + 1):
        for _ in range(per_bin):
            a = k + 0.05 * rng.integers(0, 3)
            b = a + 0.05 * rng.integers(1, 3)  # inside [k, k + 0.3]
            p = rng.uniform(0, box, 3)
            rows.append([*p, a, *(p + rng.uniform(-0.5, 0.5, 3)), b])
    db = segments_from_rows(np.array(rows))
    qrows = []
    for k in range(1, n_gaps):
        for _ in range(reps):
            p = rng.uniform(0, box, 3)
            qrows.append([*p, k + 0.5, *(p + rng.uniform(-0.5, 0.5, 3)), k + 0.6])
    for _ in range(n_gaps // 2):
        a = 0.05 * rng.integers(0, int(T / 0.05) - 4)
        b = a + 0.05 * rng.integers(1, 40)
        p = rng.uniform(0, box, 3)
        qrows.append([*p, a, *(p + rng.uniform(-0.5, 0.5, 3)), min(b, T + 0.5)])
    q = segments_from_rows(np.array(qrows)[rng.permutation(len(qrows))]).with_d(d)
    return db, q, n_gaps + 1
