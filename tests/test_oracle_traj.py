"""Pins of the trajectory-level union (oracle side, CPU).

* closed form across segment boundaries: a straight pass past a stationary
  point, both cut into segments at different times, is one interval
  |t - t_c| <= sqrt(d^2 - h^2) / s;
* two passes give two disjoint intervals, each with its closed form;
* brute force on tiny random inputs: a sampled time lies in a merged interval
  of (Q, E) exactly when some segment pair of Q and E is within d then;
* invariants: per pair sorted, disjoint and not touching; every segment-level
  interval lies inside exactly one merged interval;
* a planted slip (strict overlap instead of touching) breaks the first pin.
"""
import math

import numpy as np

import gen
from gen import fixtures as fx
from gen import workloads
import oracle
from oracle.trajectories import union_by_trajectory


def _traj(points, times, tid):
    return workloads.from_polylines(np.asarray(points, dtype=np.float64)[None],
                              np.asarray(times, dtype=np.float64)[None], [tid])


def _straight_pass(h=0.75, xs=(-10.0, 10.0), t=(0.0, 20.0), k=8, tid=0):
    ts = np.linspace(t[0], t[1], k + 1)
    xx = xs[0] + (xs[1] - xs[0]) * (ts - t[0]) / (t[1] - t[0])
    pts = np.column_stack([xx, np.full_like(xx, h), np.zeros_like(xx)])
    return _traj(pts, ts, tid)


def _union(db, q, d, lib_merge=union_by_trajectory):
    h = oracle.search(db, q.with_d(d))
    return lib_merge(h.q, h.e, h.ta, h.tb, q.traj, db.traj), h


def test_closed_form_across_boundaries():
    d, h, s = 2.0, 0.75, 1.0
    q = _straight_pass(h=h)
    # stationary entry point at the origin, cut at times that differ from the query's
    db = _traj([[0, 0, 0]] * 4, [0.0, 3.0, 9.5, 20.0], 7)
    u, segs = _union(db, q, d)
    assert len(segs) >= 2  # the pass spans several segment pairs
    w = math.sqrt(d * d - h * h) / s
    assert len(u) == 1 and u.qtraj[0] == 0 and u.etraj[0] == 7
    assert abs(u.ta[0] - (10.0 - w)) <= 1e-9 * 10 and abs(u.tb[0] - (10.0 + w)) <= 1e-9 * 10


def test_two_passes_two_intervals():
    d, h = 2.0, 0.75
    there = np.linspace(0.0, 20.0, 9)
    back = np.linspace(20.0, 40.0, 9)[1:]
    ts = np.concatenate([there, back])
    xx = np.concatenate([-10.0 + there, 10.0 - (back - 20.0)])
    q = _traj(np.column_stack([xx, np.full_like(xx, h), np.zeros_like(xx)]), ts, 3)
    db = _traj([[0, 0, 0]] * 3, [0.0, 17.0, 40.0], 5)
    u, _ = _union(db, q, d)
    w = math.sqrt(d * d - h * h)
    assert len(u) == 2
    for k, tc in enumerate((10.0, 30.0)):
        assert abs(u.ta[k] - (tc - w)) <= 1e-9 * tc and abs(u.tb[k] - (tc + w)) <= 1e-9 * tc


def _pos(s, i, t):
    f = (t - s.t0[i]) / (s.t1[i] - s.t0[i])
    return np.array([s.x0[i] + f * (s.x1[i] - s.x0[i]), s.y0[i] + f * (s.y1[i] - s.y0[i]),
                     s.z0[i] + f * (s.z1[i] - s.z0[i])])


def test_sampled_membership_on_tiny_inputs():
    rng = np.random.default_rng(31)
    for trial in range(4):
        db = gen.make_db("C1", ntraj=4, L=6)
        q = gen.make_queries("C1", nq=3, L=6)
        # pull the queries next to the database so that hits exist
        shift = rng.uniform(-2, 2, size=3)
        for f, k in (("x0", 0), ("x1", 0), ("y0", 1), ("y1", 1), ("z0", 2), ("z1", 2)):
            setattr(q, f, getattr(db, f)[: len(q)] + shift[k] + 0.3 * trial)
        d = 3.0
        u, segs = _union(db, q, d)
        times = np.linspace(0.05, 5.95, 237)
        for qt in np.unique(q.traj):
            for et in np.unique(db.traj):
                sel = (u.qtraj == qt) & (u.etraj == et)
                ivs = list(zip(u.ta[sel], u.tb[sel]))
                for t in times:
                    inside = any(a <= t <= b for a, b in ivs)
                    near = any(abs(t - a) < 1e-6 or abs(t - b) < 1e-6 for a, b in ivs)
                    truth = False
                    for i in np.where(q.traj == qt)[0]:
                        for j in np.where(db.traj == et)[0]:
                            lo, hi = max(q.t0[i], db.t0[j]), min(q.t1[i], db.t1[j])
                            if lo <= t <= hi and lo < hi:
                                dist = np.linalg.norm(_pos(q, i, t) - _pos(db, j, t))
                                truth |= dist <= d
                    if not near:
                        assert inside == truth, (trial, qt, et, t)


def test_invariants():
    db = gen.make_db("C1", ntraj=40, L=30)
    q = gen.make_queries("C1", nq=4, L=30)
    q.x0, q.x1, q.y0, q.y1 = db.x0[: len(q)] + 0.5, db.x1[: len(q)] + 0.5, db.y0[: len(q)], db.y1[: len(q)]
    q.z0, q.z1 = db.z0[: len(q)], db.z1[: len(q)]
    u, h = _union(db, q, 2.5)
    assert len(h) > 20 and 0 < len(u) < len(h)
    for k in range(1, len(u)):
        if (u.qtraj[k], u.etraj[k]) == (u.qtraj[k - 1], u.etraj[k - 1]):
            assert u.ta[k] > u.tb[k - 1]
        else:
            assert (u.qtraj[k], u.etraj[k]) > (u.qtraj[k - 1], u.etraj[k - 1])
    qt, et = q.traj[h.q], db.traj[h.e]
    for k in range(len(h)):
        sel = (u.qtraj == qt[k]) & (u.etraj == et[k]) & (u.ta <= h.ta[k]) & (h.tb[k] <= u.tb)
        assert sel.sum() == 1


def test_strict_overlap_slip_is_caught():
    def strict(q_idx, e_idx, ta, tb, q_traj, e_traj):  # the slip: touching intervals kept apart
        qt = np.asarray(q_traj)[q_idx]
        et = np.asarray(e_traj)[e_idx]
        order = np.lexsort((ta, et, qt))
        out = []
        for k in order:
            if out and out[-1][:2] == [qt[k], et[k]] and ta[k] < out[-1][3]:
                out[-1][3] = max(out[-1][3], tb[k])
            else:
                out.append([qt[k], et[k], ta[k], tb[k]])
        a = np.array(out, dtype=object)
        from oracle.trajectories import TrajHits
        return TrajHits(a[:, 0].astype(np.int64), a[:, 1].astype(np.int64),
                        a[:, 2].astype(float), a[:, 3].astype(float))

    q = _straight_pass()
    db = _traj([[0, 0, 0]] * 4, [0.0, 3.0, 9.5, 20.0], 7)
    u, _ = _union(db, q, 2.0, lib_merge=strict)
    assert len(u) != 1  # the closed-form pin above would fail for this slip


def test_point_queries_closed_form():
    # a query segment with equal end points is a stationary point P; against an
    # entry moving straight from A to B over [0, 8] the hit interval is where
    # |A + v t - P| <= d, a quadratic in t solved here in closed form
    rng = np.random.default_rng(5)
    n_e = 64
    a = rng.uniform(-5, 5, size=(n_e, 3))
    b = a + rng.uniform(-4, 4, size=(n_e, 3))
    db = fx.segments_from_rows(np.column_stack([a, np.zeros(n_e), b, np.full(n_e, 8.0)]))
    p = rng.uniform(-3, 3, size=(16, 3))
    q = fx.segments_from_rows(np.column_stack([p, np.full(16, 0.5), p, np.full(16, 7.5)]))
    d = 3.0
    h = oracle.search(db, q.with_d(d))
    assert len(h) > 50
    n_closed = 0
    for qi in range(16):
        for ei in range(n_e):
            v = (b[ei] - a[ei]) / 8.0
            w0 = a[ei] - p[qi]
            A, B, C = v @ v, 2 * (w0 @ v), w0 @ w0 - d * d
            disc = B * B - 4 * A * C
            if disc < 0:
                continue
            r1, r2 = (-B - math.sqrt(disc)) / (2 * A), (-B + math.sqrt(disc)) / (2 * A)
            lo, hi = max(0.5, r1), min(7.5, r2)
            if lo > hi:
                continue
            n_closed += 1
            k = np.where((h.q == qi) & (h.e == ei))[0]
            assert len(k) == 1, (qi, ei)
            assert abs(h.ta[k[0]] - lo) <= 1e-9 * max(1, abs(lo))
            assert abs(h.tb[k[0]] - hi) <= 1e-9 * max(1, abs(hi))
    assert n_closed == len(h)
