"""Parity at the full workload sizes, in the launch configuration the benchmark
times (range tiling, 256-thread workgroups, one resident wave per slot).

The oracle cannot brute-force these sizes whole, so each case checks:

* every reported hit, one by one, with the oracle's pair evaluation: it is a
  hit there too and its interval ends agree within the tolerance;
* a seeded random sample of query segments against every entry with the
  oracle's full search: the device reports exactly those hits for them (this
  is what catches a missed hit);
* the overlapping-pair count equals the closed form from the sorted time
  arrays;
* the filter + refine form and the plain binary64 form report the same set.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_1405_7461_amd as tds
from gpu_util import TOL, say

pytestmark = pytest.mark.gpu

BENCH_OPTS = dict(tiling="range", block_size=256)


def _overlap_closed_form(db, q) -> int:
    t0s, t1s = np.sort(db.t0), np.sort(db.t1)
    return int((np.searchsorted(t0s, q.t1, side="left") - np.searchsorted(t1s, q.t0, side="right")).sum())


def _rows(seg, i):
    return np.array([seg.x0[i], seg.y0[i], seg.z0[i], seg.t0[i], seg.x1[i], seg.y1[i], seg.z1[i], seg.t1[i]])


def _check_hits_one_by_one(db, q, h, label, limit=20000):
    n = len(h)
    idx = np.arange(n) if n <= limit else np.random.default_rng(7).choice(n, limit, replace=False)
    for k in idx:
        qi, ei = int(h.query[k]), int(h.entry[k])
        code, ta, tb = oracle.pair(_rows(q, qi), _rows(db, ei), float(q.d[qi]))
        assert code == 1, f"{label}: reported hit ({qi}, {ei}) is not a hit for the oracle ({code})"
        for got, want in ((h.ta[k], ta), (h.tb[k], tb)):
            assert abs(got - want) <= TOL * max(1.0, abs(want)), f"{label}: ({qi}, {ei}) end {got} vs {want}"
        assert int(h.traj[k]) == int(db.traj[ei]), f"{label}: trajectory id of entry {ei}"


def _check_sample(db, q, h, nsample, seed, label, extra=None):
    sel = np.random.default_rng(seed).choice(len(q), min(nsample, len(q)), replace=False)
    if extra is not None:
        sel = np.union1d(sel, extra)
    sel = np.sort(sel)
    want = oracle.search(db, q.subset(sel))
    # device hits of the sampled segments, renumbered to sample positions
    pos = np.full(len(q), -1, np.int64)
    pos[sel] = np.arange(len(sel))
    keep = pos[np.asarray(h.query)] >= 0
    gq, ge = pos[np.asarray(h.query)[keep]], np.asarray(h.entry)[keep]
    order = np.lexsort((ge, gq))
    gq, ge = gq[order], ge[order]
    assert len(gq) == len(want), f"{label}: sample has {len(gq)} device hits vs oracle {len(want)}"
    assert np.array_equal(gq, want.q) and np.array_equal(ge, want.e), f"{label}: sampled hit sets differ"
    return len(want)


def _search(ix, q, mode):
    qh = tds.Query(ix)
    try:
        qh.batch(q, q.d, mode=mode, count_overlap=True, **BENCH_OPTS)
        h = qh.fetch().sorted()
        st = qh.stats()
    finally:
        qh.close()
    return h, st


def _hit_segments(q, h, per_d, limit, seed):
    """Segments that hold device hits, with their copies at the other
    thresholds (the batch repeats the query set once per d, per_d segments
    each): at most `limit` of them, seeded."""
    base = np.unique(np.asarray(h.query) % per_d)
    if len(base) > limit:
        base = np.sort(np.random.default_rng(seed).choice(base, limit, replace=False))
    ncopies = len(q) // per_d
    return np.concatenate([base + k * per_d for k in range(ncopies)])


def _full_case(db, q, m, nsample, label, hit_sample=0, per_d=None):
    n_ovl = _overlap_closed_form(db, q)
    ix = tds.build_index(db, m)
    try:
        h32, st32 = _search(ix, q, "fp32_refine")
        h64, st64 = _search(ix, q, "fp64")
    finally:
        ix.close()
    say(f"{label}: {len(db)} entries, {len(q)} query segments, {len(h64)} hits, N_ovl {n_ovl}, "
        f"filter survivors {st32['n_refine']}")
    for st in (st32, st64):
        assert st["n_overlap"] == n_ovl
    assert np.array_equal(h32.query, h64.query) and np.array_equal(h32.entry, h64.entry), label
    assert np.array_equal(h32.ta, h64.ta) and np.array_equal(h32.tb, h64.tb), label
    _check_hits_one_by_one(db, q, h64, label)
    extra = _hit_segments(q, h64, per_d, hit_sample, 98) if hit_sample else None
    ns = _check_sample(db, q, h64, nsample, 99, label, extra)
    nx = 0 if extra is None else len(extra)
    say(f"{label}: all hits confirmed pair by pair; sample of {nsample} random segments and {nx} "
        f"segments with hits (every d) matched the oracle ({ns} hits)")
    return h64


def test_c2_full_size():
    db = gen.make_db("C2")
    qb = gen.make_queries("C2")
    q = gen.concat([qb.with_d(d) for d in (1.0, 5.0, 25.0)])
    h = _full_case(db, q, 1000, 512, "C2 full")
    assert len(h) > 1000


def test_c3_full_size():
    db = gen.make_db("C3")
    qb = gen.make_queries("C3")
    q = gen.concat([qb.with_d(d) for d in (0.001, 0.01)])
    # 512 random (segment, d) pairs and every d of up to 192 segments with
    # hits: hits are rare at these thresholds, so random segments alone
    # would mostly check empty answers
    h = _full_case(db, q, gen.CONFIGS["C3"]["bins"], 512, "C3 full", hit_sample=192, per_d=len(qb))
    assert len(h) > 0


def test_c4_full_size():
    db = gen.make_db("C4")
    q = gen.make_queries("C4")
    h = _full_case(db, q, 1000, 512, "C4 full")
    assert len(h) > 100


def test_c5_requests_full_index():
    db = gen.make_db("C5")
    ix = tds.build_index(db, gen.CONFIGS["C5"]["bins"])
    try:
        for r in (0, 1, 2, 3):
            q = gen.make_queries("C5", request=r)
            h, st = _search(ix, q, "fp32_refine")
            assert st["n_overlap"] == _overlap_closed_form(db, q)
            _check_hits_one_by_one(db, q, h, f"C5 request {r}")
            ns = _check_sample(db, q, h, 12, 100 + r, f"C5 request {r}")
            say(f"C5 request {r}: {len(q)} segments, {len(h)} hits, sample hits {ns}")
    finally:
        ix.close()
