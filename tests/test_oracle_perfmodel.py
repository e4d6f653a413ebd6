"""Pins of the response-time model's formulas (oracle side, CPU).

* beta by nested loops on Fig. 1's lookup: a query over [8, 10] meets
  l9..l14, of which l10, l13 and l14 cannot overlap it (Sec. 4), so 3 of the
  6 interactions are temporal misses;
* beta by nested loops equals 1 - (overlapping pairs)/(interactions) with
  the overlapping pairs counted from the sorted time arrays by binary
  searches (an independent count; it also checks that candidate ranges hold
  every overlapping entry) on random inputs;
* interpolation: benchmark values at grid points, midpoints, linear
  extrapolation, linear in c between curves, clamping outside the c range;
* the GPU formula: with every curve starting at the no-op time, alpha = 1
  gives T1, beta = 1 gives T2, alpha = beta = 0 gives T3; with linear curves
  the closed form Theta + (alpha r1 + beta r2 + gamma r3) i; a planted slip
  (subtracting Theta once) breaks it;
* the CPU formula's two parts add.
"""
import numpy as np

from golden_io import fig1
from oracle import batching as ob
from oracle import perfmodel as pm


def test_beta_fig1_lookup():
    t0, t1, _, lk = fig1()
    o = ob.entry_order(t0)
    assert lk["first"] == 9 and lk["last"] == 14
    beta = pm.beta_nested_loops([lk["t0"]], [lk["t1"]], t0[o], t1[o], [lk["first"]], [lk["last"]])
    assert beta == 0.5
    assert beta == 1 - len(lk["overlap"]) / 6


def test_beta_matches_sorted_count():
    rng = np.random.default_rng(9)
    for trial in range(3):
        t0 = np.round(rng.uniform(0, 50, 300), 2)
        t1 = t0 + np.round(rng.exponential(2.0, 300), 2) + 0.01
        o = ob.entry_order(t0)
        e0, e1 = t0[o], t1[o]
        bins = ob.bin_table(e0, e1, 17)
        qa = rng.uniform(-2, 52, 60)
        qb = qa + rng.exponential(1.5, 60) + 0.01
        first, last = [], []
        for a, b in zip(qa, qb):
            r = ob.candidate_range(bins, a, b)
            first.append(r[0] if r else 0)
            last.append(r[1] if r else -1)
        first, last = np.array(first), np.array(last)
        beta = pm.beta_nested_loops(qa, qb, e0, e1, first, last)
        n_int = int(np.sum(np.maximum(last - first + 1, 0)))
        s0, s1 = np.sort(t0), np.sort(t1)
        n_ovl = int((np.searchsorted(s0, qb, side="left") - np.searchsorted(s1, qa, side="right")).sum())
        assert n_int > 0 and abs(beta - (1 - n_ovl / n_int)) < 1e-12


def test_interpolation():
    xs, ys = [0.0, 10.0, 30.0], [1.0, 3.0, 4.0]
    for x, y in zip(xs, ys):
        assert pm.interp_curve(xs, ys, x) == y
    assert pm.interp_curve(xs, ys, 5.0) == 2.0
    assert pm.interp_curve(xs, ys, 20.0) == 3.5
    assert pm.interp_curve(xs, ys, 50.0) == 5.0      # extends the last segment
    assert pm.interp_curve(xs, ys, -10.0) == -1.0    # and the first
    table = {100.0: ([0.0, 1000.0], [1.0, 2.0]), 300.0: ([0.0, 1000.0], [1.0, 4.0])}
    assert pm.interp_table(table, 500.0, 100.0) == 1.5
    assert pm.interp_table(table, 500.0, 200.0) == 2.0   # halfway between 1.5 and 2.5
    assert pm.interp_table(table, 500.0, 50.0) == 1.5    # clamped to the nearest curve
    assert pm.interp_table(table, 500.0, 900.0) == 2.5


def _linear_tables(theta, r):
    xs = [0.0, 1e6, 4e6]
    return {k: {c: (xs, [theta + rate * x for x in xs]) for c in (256.0, 4096.0)}
            for k, rate in r.items()}


def test_gpu_formula_special_cases_and_closed_form():
    theta = 0.05
    r = {"hit": 3e-7, "tmiss": 1e-7, "smiss": 0.5e-7, "noop": 0.0}
    t = _linear_tables(theta, r)
    i, c = 2.5e6, 1000.0
    t1 = pm.interp_table(t["hit"], i, c)
    assert abs(pm.t_gpu(t, 1.0, 0.0, i, c) - t1) < 1e-12
    assert abs(pm.t_gpu(t, 0.0, 1.0, i, c) - pm.interp_table(t["tmiss"], i, c)) < 1e-12
    assert abs(pm.t_gpu(t, 0.0, 0.0, i, c) - pm.interp_table(t["smiss"], i, c)) < 1e-12
    for a, b in ((0.1, 0.3), (0.01, 0.9), (0.5, 0.5)):
        g = 1 - a - b
        want = theta + (a * r["hit"] + b * r["tmiss"] + g * r["smiss"]) * i
        assert abs(pm.t_gpu(t, a, b, i, c) - want) < 1e-12

    def slip(tables, alpha, beta, i, c):  # Theta subtracted once
        gamma = 1 - alpha - beta
        return (pm.interp_table(tables["hit"], alpha * i, c) + pm.interp_table(tables["tmiss"], beta * i, c)
                + pm.interp_table(tables["smiss"], gamma * i, c) - pm.interp_table(tables["noop"], i, c))

    assert abs(slip(t, 0.1, 0.3, i, c) - pm.t_gpu(t, 0.1, 0.3, i, c)) > 1e-3


def test_cpu_formula():
    assert pm.t_cpu(0.1, 2.0, 0.5, 16.0, 0.0, 1.0) == 0.1 + 2.0 * 4.0
    assert pm.t_cpu(0.0, 0.0, 1.0, 1.0, 3e6, 1.5e6) == 2.0
