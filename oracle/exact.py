"""Exact rational re-decision of one pair (test infrastructure only).

The binary64 inputs are taken as exact rationals. Positions along each
segment are the exact linear interpolation between its end points (paper
Sec. 3: segments are linearly interpolated), over the exact common time span
(max t_start, min t_end). The squared distance minus d^2 is then an exact
quadratic in time, and its minimum over the span decides the pair without
any rounding. Interval ends are the quadratic's roots evaluated with 60
significant decimal digits. This is slow: use it on tiny inputs only.
"""
from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction as F


def _frac_row(row):
    return [F(float(v)) for v in row]


def _to_dec(x: F) -> Decimal:
    return Decimal(x.numerator) / Decimal(x.denominator)


def exact_pair(qrow, erow, d):
    """Returns dict(code, min_dist2, ta, tb, vertex) with code -1 / 0 / 1 as the oracle.

    ``min_dist2`` is the exact minimum squared distance over the common span
    (a Fraction), ``ta``/``tb`` floats for hits, ``vertex`` the time of
    closest approach clamped to the common span (a float; the start of the
    span when the distance is constant).
    """
    getcontext().prec = 60
    q = _frac_row(qrow)
    e = _frac_row(erow)
    dd = F(float(d)) ** 2
    tlo = max(q[3], e[3])
    thi = min(q[7], e[7])
    if not tlo < thi:
        return dict(code=-1, min_dist2=None, ta=None, tb=None, vertex=None)

    def pos(s, t):
        w = (t - s[3]) / (s[7] - s[3])
        return [s[k] + (s[k + 4] - s[k]) * w for k in range(3)]

    def vel(s):
        return [(s[k + 4] - s[k]) / (s[7] - s[3]) for k in range(3)]

    pq, pe = pos(q, tlo), pos(e, tlo)
    vq, ve = vel(q), vel(e)
    D = [pq[k] - pe[k] for k in range(3)]
    V = [vq[k] - ve[k] for k in range(3)]
    a = sum(v * v for v in V)
    B = sum(D[k] * V[k] for k in range(3))
    c = sum(x * x for x in D) - dd
    T = thi - tlo

    def f(tau):
        return (a * tau + 2 * B) * tau + c

    if a == 0:
        fmin = c
        tv = F(0)
    else:
        tv = -B / a
        tv = min(max(tv, F(0)), T)
        fmin = min(f(tv), c, f(T))
    res = dict(code=1 if fmin <= 0 else 0, min_dist2=fmin + dd, ta=None, tb=None,
               vertex=float(_to_dec(tlo + tv)))
    if res["code"] == 1:
        if a == 0:
            lo, hi = Decimal(0), _to_dec(T)
        else:
            disc = _to_dec(B * B - a * c)
            if disc < 0:
                disc = Decimal(0)
            s = disc.sqrt()
            ad, Bd = _to_dec(a), _to_dec(B)
            r1 = (-Bd - s) / ad
            r2 = (-Bd + s) / ad
            lo = max(r1, Decimal(0))
            hi = min(r2, _to_dec(T))
            if lo > hi:
                lo = hi = min(max(-Bd / ad, Decimal(0)), _to_dec(T))
        res["ta"] = float(_to_dec(tlo) + lo)
        res["tb"] = float(_to_dec(tlo) + hi)
    return res
