"""The response-time model of the paper's Sec. 8 (oracle side).

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``).

Written from the paper:

* GPU component (Sec. 8.1): for a batch with i interactions over c
  candidate entries, T(i, c) = T1(alpha i, c) + T2(beta i, c) + T3(gamma i, c)
  - 2 Theta(i, c), where T1, T2, T3 are the times of batches whose
  interactions are all hits, all temporal misses, all temporal hits but
  spatial misses, and Theta the overhead of a batch with no work (each of
  the three terms contains it once, hence the subtraction).
* T1..T3 and Theta come from benchmarks: curves of time against
  interactions, one per candidate count c; a value is read off the two
  curves whose c bracket the asked c, each by linear interpolation in i,
  then interpolated linearly in c.
* beta is exact: over the candidate pairs of the batch (query segment x
  entry of its candidate range), the fraction whose spans do not overlap,
  by two nested loops; gamma = 1 - alpha - beta.
* CPU component (Sec. 8.2): a fitted curve a + b s^e for the invocation
  overhead and sigma / bandwidth for returning sigma result bytes.
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np


def beta_nested_loops(q_t0, q_t1, e_t0, e_t1, first, last) -> float:
    """Exact temporal-miss fraction of a batch by two nested loops.

    first/last: candidate range (entry indices, inclusive) of each query
    segment; last < first means no candidates. Overlap means a common span
    of positive length.
    """
    n_int = 0
    n_miss = 0
    for k in range(len(q_t0)):
        for e in range(int(first[k]), int(last[k]) + 1):
            n_int += 1
            if not (max(q_t0[k], e_t0[e]) < min(q_t1[k], e_t1[e])):
                n_miss += 1
    return n_miss / n_int if n_int else 0.0


def interp_curve(xs: Sequence[float], ys: Sequence[float], x: float) -> float:
    """Linear interpolation along one benchmark curve; linear extrapolation
    from the two nearest points outside it."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    if xs.size == 1:
        return float(ys[0])
    k = int(np.searchsorted(xs, x, side="right")) - 1
    k = min(max(k, 0), xs.size - 2)
    x0, x1, y0, y1 = xs[k], xs[k + 1], ys[k], ys[k + 1]
    return float(y0 + (y1 - y0) * (x - x0) / (x1 - x0))


def interp_table(table: Dict[float, tuple], i: float, c: float) -> float:
    """table: {c: (interactions array, times array)}. Bracketing curves in c,
    each read at i, then linear in c (clamped to the table's c range)."""
    cs = sorted(table)
    if c <= cs[0]:
        return interp_curve(*table[cs[0]], i)
    if c >= cs[-1]:
        return interp_curve(*table[cs[-1]], i)
    k = int(np.searchsorted(cs, c, side="right")) - 1
    c0, c1 = cs[k], cs[k + 1]
    t0 = interp_curve(*table[c0], i)
    t1 = interp_curve(*table[c1], i)
    return t0 + (t1 - t0) * (c - c0) / (c1 - c0)


def t_gpu(tables: Dict[str, Dict[float, tuple]], alpha: float, beta: float, i: float,
          c: float) -> float:
    """Sec. 8.1's GPU time of one batch."""
    gamma = 1.0 - alpha - beta
    return (interp_table(tables["hit"], alpha * i, c) + interp_table(tables["tmiss"], beta * i, c)
            + interp_table(tables["smiss"], gamma * i, c) - 2.0 * interp_table(tables["noop"], i, c))


def t_cpu(a: float, b: float, e: float, s: float, sigma: float, bandwidth: float) -> float:
    """Sec. 8.2: invocation overhead curve plus result transfer."""
    return a + b * s ** e + sigma / bandwidth
