"""GreedySetSplit and Periodic tiles (Sec. 6, Alg. 4) on the GPU against the
oracle's batches.

* Fig. 2 on the device: batch sizes and interactions of the hand-worked
  golden (tests/golden/fig2_greedy.txt) for both variants;
* tiles identical to the oracle's batches (members in order, candidate
  range) and n_eval equal to the oracle's interaction total on C1, reduced
  C2 and reduced C4, for several bounds of both variants, with hits equal to
  the oracle's search;
* full-size C4 (uneven queries with per-trajectory d): tiles identical to
  the oracle's, every hit confirmed pair by pair, a sampled oracle search;
* Periodic tiles identical to the oracle's (runs of s segments with
  candidates in (t_start, caller index) order) on the same cases and on
  full-size C4, whose short query trajectories at arbitrary times make the
  order within a t_start bin matter;
* edge cases: no segment with candidates, bound 1, bound >= |Q|, t_start
  bins holding more query segments than one workgroup sorts in LDS;
* the two-segment cases of tests/golden/fig1_sec4_ranges.txt and the comb
  fixture (bins of very uneven extent, query groups with identical ranges
  whose merges are not free): tiles identical to the oracle's batches.
"""
import numpy as np
import pytest

import gen
from gen import fixtures as fx
import oracle
from oracle import batching as ob
import paper_1405_7461_amd as tds
from golden_io import fig1, fig1_sec4, fig2, fig2_greedy
from gpu_util import compare, say

pytestmark = pytest.mark.gpu
VARIANTS = {"min": "greedy_min", "max": "greedy_max"}
TILINGS = dict(VARIANTS, periodic="periodic")


def _oracle_batches(db, q, m, bound, variant):
    o = ob.entry_order(db.t0)
    bins = ob.bin_table(db.t0[o], db.t1[o], m)
    if variant == "periodic":
        return bins, ob.periodic(bins, q.t0, q.t1, bound)
    return bins, ob.greedy_set_split(bins, q.t0, q.t1, bound, variant)


def _device(ix, q, variant, bound, mode="fp32_refine"):
    qh = tds.Query(ix)
    try:
        qh.batch(q, q.d, mode=mode, tiling=TILINGS[variant], batch_size=bound)
        h = qh.fetch().sorted()
        st = qh.stats()
        tiles, members = qh.tiles()
    finally:
        qh.close()
    return h, st, tiles, members


def _compare_tiles(bins, want, tiles, members, st, label):
    assert len(tiles) == len(want), f"{label}: {len(tiles)} tiles vs oracle {len(want)} batches"
    assert st["n_tiles"] == len(want)
    pos = 0
    for k, (t, b) in enumerate(zip(tiles, want)):
        assert t["q_first"] == pos and t["n_query"] == b.n, f"{label}: tile {k} members"
        assert np.array_equal(members[pos:pos + b.n], b.members), f"{label}: tile {k} order"
        f, l = ob.batch_range(bins, b)
        assert (t["e_first"], t["n_entry"]) == (f, l - f + 1), f"{label}: tile {k} range"
        pos += b.n
    assert len(members) == pos
    assert st["n_eval"] == ob.total_interactions(bins, want), f"{label}: n_eval"


def _fig_case():
    t0, t1, _, _ = fig1()
    rng = np.random.default_rng(3)
    n = t0.size
    p0 = rng.uniform(0, 5, (n, 3))
    db = fx.segments_from_rows(np.column_stack([p0, t0, p0 + rng.uniform(-1, 1, (n, 3)), t1]))
    batches, _ = fig2()
    qa = np.concatenate([[a] * k for k, a, b in batches])
    qb = np.concatenate([[b] * k for k, a, b in batches])
    p = rng.uniform(0, 5, (qa.size, 3))
    q = fx.segments_from_rows(np.column_stack([p, qa, p + 0.5, qb])).with_d(1.0)
    return db, q


def test_fig2_on_device():
    db, q = _fig_case()
    ix = tds.build_index(db, 4)
    try:
        for variant, bound, sizes, total in fig2_greedy():
            h, st, tiles, members = _device(ix, q, variant, bound)
            assert list(tiles["n_query"]) == sizes, (variant, bound)
            assert st["n_eval"] == total, (variant, bound)
            bins, want = _oracle_batches(db, q, 4, bound, variant)
            _compare_tiles(bins, want, tiles, members, st, f"Fig. 2 {variant} {bound}")
            compare(h, oracle.search(db, q), db, f"Fig. 2 {variant} {bound}")
    finally:
        ix.close()


def _cases():
    yield "C1", gen.make_config("C1")
    db = gen.make_db("C2", ntraj=300)
    qb = gen.make_queries("C2", nq=20)
    yield "C2r", (db, gen.concat([qb.with_d(x) for x in (1.0, 5.0, 25.0)]), 1000)
    yield "C4r", (gen.make_db("C4", ntraj=300), gen.make_queries("C4", nq=24), 1000)
    # two bins: about 12,000 query segments per t_start bin, more than one
    # workgroup sorts in LDS (the counting fallback orders them)
    yield "C2r coarse", (db, gen.concat([qb.with_d(x) for x in (1.0, 5.0, 25.0)]), 2)


@pytest.mark.parametrize("variant", ["min", "max"])
def test_tiles_and_hits_match_oracle(variant):
    for label, (db, q, m) in _cases():
        want_hits = oracle.search(db, q)
        ix = tds.build_index(db, m)
        try:
            for bound in (1, 7, 128, 5000):
                h, st, tiles, members = _device(ix, q, variant, bound)
                bins, want = _oracle_batches(db, q, m, bound, variant)
                _compare_tiles(bins, want, tiles, members, st, f"{label} {variant} {bound}")
                compare(h, want_hits, db, f"{label} {variant} {bound}")
                say(f"{label} {variant} bound {bound}: {len(want)} tiles, n_eval {st['n_eval']}, "
                    f"{len(h)} hits")
        finally:
            ix.close()


def test_periodic_tiles_match_oracle():
    for label, (db, q, m) in _cases():
        want_hits = oracle.search(db, q)
        ix = tds.build_index(db, m)
        try:
            for s in (1, 7, 128, 5000):
                h, st, tiles, members = _device(ix, q, "periodic", s)
                bins, want = _oracle_batches(db, q, m, s, "periodic")
                _compare_tiles(bins, want, tiles, members, st, f"{label} periodic {s}")
                compare(h, want_hits, db, f"{label} periodic {s}")
                say(f"{label} periodic {s}: {len(want)} tiles, n_eval {st['n_eval']}, {len(h)} hits")
        finally:
            ix.close()


def test_full_size_c4_periodic_tiles():
    db = gen.make_db("C4")
    q = gen.make_queries("C4")
    ix = tds.build_index(db, 1000)
    try:
        for s in (64, 128):
            h, st, tiles, members = _device(ix, q, "periodic", s)
            bins, want = _oracle_batches(db, q, 1000, s, "periodic")
            _compare_tiles(bins, want, tiles, members, st, f"C4 full periodic {s}")
            say(f"C4 full periodic {s}: {len(want)} tiles, n_eval {st['n_eval']}, {len(h)} hits")
    finally:
        ix.close()


def test_full_size_c4_tiles():
    from test_gpu_fullsize import _check_hits_one_by_one, _check_sample
    db = gen.make_db("C4")
    q = gen.make_queries("C4")
    ix = tds.build_index(db, 1000)
    try:
        for variant, bound in (("min", 256), ("max", 1024)):
            h, st, tiles, members = _device(ix, q, variant, bound)
            bins, want = _oracle_batches(db, q, 1000, bound, variant)
            _compare_tiles(bins, want, tiles, members, st, f"C4 full {variant} {bound}")
            _check_hits_one_by_one(db, q, h, f"C4 full {variant}", limit=5000)
            ns = _check_sample(db, q, h, 256, 5, f"C4 full {variant}")
            say(f"C4 full {variant} {bound}: {len(want)} tiles, n_eval {st['n_eval']}, {len(h)} hits, "
                f"sample {ns}")
    finally:
        ix.close()


def test_edge_cases():
    db = gen.make_db("C1", ntraj=30)
    q = gen.make_queries("C1", nq=4)
    ix = tds.build_index(db, 50)
    try:
        far = q.subset(np.arange(len(q)))
        far.t0 = far.t0 + 1e6
        far.t1 = far.t1 + 1e6
        for v in TILINGS:
            h, st, tiles, members = _device(ix, far, v, 16)
            assert len(h) == 0 and len(tiles) == 0 and len(members) == 0 and st["n_eval"] == 0
            h, st, tiles, _ = _device(ix, q, v, 1 << 16)
            assert len(tiles) == 1
            compare(h, oracle.search(db, q), db, f"one tile {v}")
    finally:
        ix.close()


def _time_case(spans, rng):
    t0, t1, _, _ = fig1()
    n = t0.size
    p0 = rng.uniform(0, 5, (n, 3))
    db = fx.segments_from_rows(np.column_stack([p0, t0, p0 + rng.uniform(-1, 1, (n, 3)), t1]))
    p = rng.uniform(0, 5, (len(spans), 3))
    qa = np.array([a for a, _ in spans])
    qb = np.array([b for _, b in spans])
    q = fx.segments_from_rows(np.column_stack([p, qa, p + 0.5, qb])).with_d(2.0)
    return db, q


def test_fig1_sec4_greedy_on_device():
    rng = np.random.default_rng(17)
    _, greedy = fig1_sec4()
    for variant, bound, spans, sizes, total in greedy:
        db, q = _time_case(spans, rng)
        ix = tds.build_index(db, 4)
        try:
            h, st, tiles, members = _device(ix, q, variant, bound)
        finally:
            ix.close()
        label = f"fig1 {variant} {bound} {spans}"
        assert list(tiles["n_query"]) == sizes, label
        assert st["n_eval"] == total, label
        bins, want = _oracle_batches(db, q, 4, bound, variant)
        _compare_tiles(bins, want, tiles, members, st, label)
        compare(h, oracle.search(db, q), db, label)


def test_comb_bins_tiles_match_oracle():
    """Identical candidate ranges whose merged extent takes in another bin:
    the first pass must not merge them (Sec. 4 ranges, Alg. 4)."""
    db, q, m = fx.comb_bins()
    o = ob.entry_order(db.t0)
    bins = ob.bin_table(db.t0[o], db.t1[o], m)
    one = ob.singletons(bins, q.t0, q.t1)
    rr = [ob.batch_range(bins, b) for b in one]
    runs = 1 + sum(rr[k] != rr[k - 1] for k in range(1, len(rr)))
    assert len(ob.free_merges(bins, one)) > runs  # the fixture hits the case
    want_hits = oracle.search(db, q)
    ix = tds.build_index(db, m)
    try:
        for variant in ("min", "max", "periodic"):
            for bound in (1, 2, 3, 7, 64, 1000):
                h, st, tiles, members = _device(ix, q, variant, bound)
                _, want = _oracle_batches(db, q, m, bound, variant)
                _compare_tiles(bins, want, tiles, members, st, f"comb {variant} {bound}")
                compare(h, want_hits, db, f"comb {variant} {bound}")
                say(f"comb {variant} {bound}: {len(want)} tiles, n_eval {st['n_eval']}")
    finally:
        ix.close()
