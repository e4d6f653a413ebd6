"""Checks that pin the oracle to facts it does not compute itself.

Each ``pin_*`` function takes a loaded oracle library and returns a list of
failure messages (empty when the pin holds). They are used twice: on the
real oracle (must all hold) and on deliberately broken copies of it (each
copy must break at least one pin), which shows that a plausible slip in the
oracle's arithmetic cannot go unnoticed.
"""
from __future__ import annotations

import math

import numpy as np

import gen
from gen import fixtures as fx
import oracle
from oracle.exact import exact_pair

EPS = 2.0 ** -52


def _rows(s):
    return np.column_stack(s.arrays())


def _hitmap(h):
    return {(int(a), int(b)): (x, y) for a, b, x, y in zip(h.q, h.e, h.ta, h.tb)}


def pin_worked_value(lib):
    """Entry at rest at the origin over [0,10]; query from (-5,0,0) to (5,0,0).

    With d = 2 the pair is within d for |t - 5| <= 2, i.e. exactly [3, 7]:
    a = 1, B = -5, c = 21, B^2 - a c = 4, roots 3 and 7 are exact in binary64.
    With the query passing at height h = 1 and d = 2 the interval is
    5 -/+ sqrt(3).
    """
    f = []
    e = [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 10.0]
    q = [-5.0, 0.0, 0.0, 0.0, 5.0, 0.0, 0.0, 10.0]
    r = oracle.pair(q, e, 2.0, lib=lib)
    if r != (1, 3.0, 7.0):
        f.append(f"[3,7] example gave {r}")
    q2 = [-5.0, 1.0, 0.0, 0.0, 5.0, 1.0, 0.0, 10.0]
    r = oracle.pair(q2, e, 2.0, lib=lib)
    exp = (5 - math.sqrt(3), 5 + math.sqrt(3))
    if r[0] != 1 or abs(r[1] - exp[0]) > 1e-14 or abs(r[2] - exp[1]) > 1e-14:
        f.append(f"h=1 example gave {r}, expected {exp}")
    # never within d: passes at height 3 > 2
    q3 = [-5.0, 3.0, 0.0, 0.0, 5.0, 3.0, 0.0, 10.0]
    if oracle.pair(q3, e, 2.0, lib=lib)[0] != 0:
        f.append("h=3 example should miss")
    # time spans that only touch are not compared
    e4 = [0.0, 0.0, 0.0, 10.0, 0.0, 0.0, 0.0, 11.0]
    if oracle.pair(q, e4, 100.0, lib=lib)[0] != -1:
        f.append("touching spans should not be compared")
    return f


def pin_closed_form(lib):
    """Straight passes by a resting entry: [t_c - w, t_c + w], w = sqrt(d^2-h^2)/s."""
    f = []
    db, q, params = fx.passing_pairs()
    for i, p in enumerate(params):
        d, h, s = p["d"], p["h"], p["s"]
        if abs(h / d - 1.0) < 1e-3:
            continue
        r = oracle.pair(_rows(q)[i], _rows(db)[i], d, lib=lib)
        if h > d:
            if r[0] != 0:
                f.append(f"pass {i}: expected miss, got {r}")
            continue
        w = math.sqrt(d * d - h * h) / s
        tc = p["t0"] + 5.0
        lo, hi = max(tc - w, p["t0"]), min(tc + w, p["t0"] + 10.0)
        if r[0] != 1 or abs(r[1] - lo) > 1e-9 * max(1, abs(lo)) or abs(r[2] - hi) > 1e-9 * max(1, abs(hi)):
            f.append(f"pass {i}: got {r}, expected [{lo}, {hi}]")
    return f


def pin_stationary(lib):
    """Equal velocities: always within d (offset <= d, including = d) or never."""
    f = []
    db, q, kinds = fx.stationary_pairs(1.0)
    for i, k in enumerate(kinds):
        r = oracle.pair(_rows(q)[i], _rows(db)[i], 1.0, lib=lib)
        if k in ("in", "edge"):
            if r != (1, 0.0, 4.0):
                f.append(f"stationary {k}: got {r}, expected (1, 0, 4)")
        elif r[0] != 0:
            f.append(f"stationary {k}: got {r}, expected a miss")
    return f


def pin_symmetry(lib):
    """Swapping the roles of query and entry gives the transposed hit set, bitwise.

    D and V change sign exactly, so a, B and c are bitwise unchanged.
    """
    f = []
    for db, q in (fx.random_small(), fx.dense_box()):
        d = float(q.d[0])
        h1 = oracle.search(db, q, lib=lib)
        h2 = oracle.search(q, db.with_d(d), lib=lib)
        m1 = _hitmap(h1)
        m2 = {(b, a): v for (a, b), v in _hitmap(h2).items()}
        if m1 != m2:
            f.append(f"symmetry broken: {len(m1)} vs {len(m2)} hits, "
                     f"{len(set(m1) ^ set(m2))} pairs differ")
        if h1.n_overlap != h2.n_overlap:
            f.append("symmetry: overlap counts differ")
    return f


def _brute_overlaps(db, q):
    lo = np.maximum(q.t0[:, None], db.t0[None, :])
    hi = np.minimum(q.t1[:, None], db.t1[None, :])
    return int((lo < hi).sum())


def pin_overlap_count(lib):
    """The overlap count equals a direct count of strictly overlapping spans."""
    f = []
    for db, q in (fx.random_small(), fx.dense_box(), fx.all_hit()):
        h = oracle.search(db, q, lib=lib)
        b = _brute_overlaps(db, q)
        if h.n_overlap != b:
            f.append(f"overlap count {h.n_overlap} != {b}")
    return f


def pin_all_hit(lib):
    """All points at one place: every overlapping pair is a hit over its whole span."""
    f = []
    db, q = fx.all_hit()
    h = oracle.search(db, q, lib=lib)
    if len(h) != h.n_overlap:
        f.append(f"all-hit: {len(h)} hits vs {h.n_overlap} overlapping pairs")
    lo = np.maximum(q.t0[h.q], db.t0[h.e])
    hi = np.minimum(q.t1[h.q], db.t1[h.e])
    if not (np.array_equal(lo, h.ta) and np.array_equal(hi, h.tb)):
        f.append("all-hit intervals are not the full spans")
    return f


def _positions(s, idx, t):
    w = (t - s.t0[idx]) / (s.t1[idx] - s.t0[idx])
    return np.stack([getattr(s, a + "0")[idx] + (getattr(s, a + "1")[idx] - getattr(s, a + "0")[idx]) * w
                     for a in "xyz"], axis=-1)


def pin_sampling(lib, nsamp=2001):
    """Dense time sampling of every overlapping pair on tiny inputs.

    A sample within d(1-1e-9) must lie in the reported interval; one beyond
    d(1+1e-9) must lie outside; a hit's interval mid-point must be within
    d(1+1e-9).
    """
    f = []
    for db, q in (fx.random_small(), fx.dense_box(ntraj=12, L=10, nq=4)):
        h = oracle.search(db, q, lib=lib)
        hm = _hitmap(h)
        for i in range(len(q)):
            lo = np.maximum(q.t0[i], db.t0)
            hi = np.minimum(q.t1[i], db.t1)
            for j in np.nonzero(lo < hi)[0]:
                t = np.linspace(lo[j], hi[j], nsamp)
                dist = np.linalg.norm(_positions(q, i, t) - _positions(db, j, t), axis=-1)
                d = q.d[i]
                inside = dist <= d * (1 - 1e-9)
                outside = dist >= d * (1 + 1e-9)
                iv = hm.get((i, int(j)))
                step = (hi[j] - lo[j]) / (nsamp - 1)
                if iv is None:
                    if inside.any():
                        f.append(f"pair ({i},{j}) within d at a sample but not reported")
                    continue
                ta, tb = iv
                tol = 1e-9 * max(1.0, abs(ta), abs(tb))
                if (inside & ((t < ta - tol) | (t > tb + tol))).any():
                    f.append(f"pair ({i},{j}): sample within d outside [{ta},{tb}]")
                if (outside & (t > ta + tol) & (t < tb - tol)).any():
                    f.append(f"pair ({i},{j}): sample beyond d inside [{ta},{tb}]")
                if tb - ta > 2 * step and not (dist <= d * (1 + 1e-9))[(t >= ta) & (t <= tb)].any():
                    f.append(f"pair ({i},{j}): no sample within d in [{ta},{tb}]")
                tm = np.array([(ta + tb) / 2])
                dm = np.linalg.norm(_positions(q, i, tm) - _positions(db, j, tm))
                if dm > d * (1 + 1e-9):
                    f.append(f"pair ({i},{j}): mid-point at distance {dm} > d")
                if not (lo[j] <= ta <= tb <= hi[j]):
                    f.append(f"pair ({i},{j}): interval outside the common span")
    return f


def _error_bound2(qrow, erow, d):
    """Generous bound on the binary64 error of the decision, in squared distance."""
    q = np.asarray(qrow)
    e = np.asarray(erow)
    ext = np.abs(q[4:7] - q[0:3]).sum() + np.abs(e[4:7] - e[0:3]).sum()
    mag = np.abs(q[[0, 1, 2, 4, 5, 6]]).max() + np.abs(e[[0, 1, 2, 4, 5, 6]]).max()
    span = 4.0 * (d + ext + mag)
    return 64 * EPS * span * span


def pin_exact(lib):
    """Exact-rational re-decision of every pair of tiny random inputs.

    Decisions must agree except where the exact minimum distance is within
    the binary64 error bound of d; interval ends must agree to 1e-9.
    """
    f = []
    cases = [fx.random_small(), fx.dense_box(ntraj=10, L=8, nq=3), fx.near_threshold()[:2]]
    for db, q in cases:
        qr, er = _rows(q), _rows(db)
        for i in range(len(q)):
            for j in range(len(db)):
                d = float(q.d[i])
                r = oracle.pair(qr[i], er[j], d, lib=lib)
                x = exact_pair(qr[i], er[j], d)
                if r[0] != x["code"]:
                    margin = abs(float(x["min_dist2"]) - d * d) if x["min_dist2"] is not None else 0.0
                    if x["code"] == -1 or r[0] == -1 or margin > _error_bound2(qr[i], er[j], d):
                        f.append(f"pair ({i},{j}): oracle {r[0]} vs exact {x['code']} (margin {margin:.3g})")
                    continue
                if r[0] == 1:
                    for got, want in ((r[1], x["ta"]), (r[2], x["tb"])):
                        # near tangency the interval ends are ill-conditioned
                        dd2 = float(x["min_dist2"])
                        cond = max(1.0, d * d / max(d * d - dd2, 1e-300)) if dd2 < d * d else 1e30
                        tol = 1e-9 * max(1.0, abs(want)) * math.sqrt(min(cond, 1e12))
                        if abs(got - want) > tol:
                            f.append(f"pair ({i},{j}): end {got} vs exact {want}")
    return f


def pin_near_threshold(lib):
    """Closest approach d(1 -/+ 2^-k): decisions follow the exact predicate
    outside the error bound, for every k down to 2^-52."""
    f = []
    db, q, tags = fx.near_threshold()
    qr, er = _rows(q), _rows(db)
    for i, (k, sgn) in enumerate(tags):
        d = float(q.d[i])
        r = oracle.pair(qr[i], er[i], d, lib=lib)
        x = exact_pair(qr[i], er[i], d)
        if r[0] != x["code"]:
            margin = abs(float(x["min_dist2"]) - d * d)
            if margin > _error_bound2(qr[i], er[i], d):
                f.append(f"k={k} sgn={sgn}: oracle {r[0]} vs exact {x['code']}")
        if k <= 20 and x["code"] != (1 if sgn < 0 else 0):
            f.append(f"k={k} sgn={sgn}: fixture not on the intended side")
    return f


def pin_r8_collapse(lib):
    """Pairs whose computed entry time falls after the computed exit time
    (tests/golden/r8_collapse.txt: a pass that comes within d right at the
    end of the common span) report the single time of closest approach,
    clamped to the span: t_a == t_b, inside [tlo, thi], equal to the exact
    clamped vertex within the endpoint tolerance, and the exact minimum
    distance is d up to the decision's error bound."""
    from golden_io import r8_collapse
    f = []
    cases = r8_collapse()
    if len(cases) < 4:
        return [f"r8 fixture holds {len(cases)} pairs"]
    for k, (qr, er, d) in enumerate(cases):
        r = oracle.pair(qr, er, d, lib=lib)
        x = exact_pair(qr, er, d)
        tlo, thi = max(qr[3], er[3]), min(qr[7], er[7])
        if r[0] != 1:
            f.append(f"r8 pair {k}: code {r[0]}")
            continue
        if not (r[1] == r[2]):
            f.append(f"r8 pair {k}: interval [{r[1]}, {r[2]}] is not one time")
        if not (tlo <= r[1] <= thi):
            f.append(f"r8 pair {k}: {r[1]} outside [{tlo}, {thi}]")
        v = x["vertex"]
        if not abs(r[1] - v) <= 1e-9 * max(1.0, abs(v)):
            f.append(f"r8 pair {k}: {r[1]} vs exact clamped vertex {v}")
        margin = abs(float(x["min_dist2"]) - d * d)
        if margin > _error_bound2(qr, er, d):
            f.append(f"r8 pair {k}: not near tangency (margin {margin:.3g})")
    return f


ALL_PINS = [pin_worked_value, pin_closed_form, pin_stationary, pin_symmetry,
            pin_overlap_count, pin_all_hit, pin_sampling, pin_exact, pin_near_threshold,
            pin_r8_collapse]


def run_all(lib):
    out = {}
    for p in ALL_PINS:
        try:
            out[p.__name__] = p(lib)
        except Exception as exc:  # a broken oracle may also crash a pin
            out[p.__name__] = [f"raised {type(exc).__name__}: {exc}"]
    return out
