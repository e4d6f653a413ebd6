"""HIP path against the oracle, element by element (GPU).

Every case compares the sorted (query, entry) hit set exactly and the
interval ends to 1e-9 relative (they are expected to be bitwise equal, as
both sides evaluate the same binary64 expression).
"""
import numpy as np
import pytest

import gen
from gen import fixtures as fx
import oracle
import paper_1405_7461_amd as tds
from paper_1405_7461_amd import _lib as L
from golden_io import fig1, fig1_sec4, r8_collapse
from gpu_util import compare, run, say

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32_refine"]


def test_fig1_index_on_device():
    t0, t1, bins, lk = fig1()
    db = fx.time_only(t0, t1)
    ix = tds.build_index(db, 4)
    got = ix.bins()
    assert [tuple(r) for r in got[["bin", "start", "end", "first", "last"]]] == \
        [(j, s, e, f, l) for j, s, e, f, l in bins]
    info = ix.info()
    assert info["n"] == 15 and info["nonempty_bins"] == 4 and info["bin_width"] == 3.0
    q = fx.segments_from_rows([[0, 0, 0, lk["t0"], 0, 0, 0, lk["t1"]]]).with_d(1e9)
    h, st, (f, l) = run(db, q, 4, index=ix)
    assert (f[0], l[0]) == (lk["first"], lk["last"])
    # with a huge d every overlapping entry is a hit
    assert sorted(h.entry.tolist()) == lk["overlap"]
    assert st["n_overlap"] == len(lk["overlap"])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("tiling", ["periodic", "range"])
def test_c1_full(mode, tiling):
    db, q, m = gen.make_config("C1")
    say(f"C1 {mode} {tiling}: db {len(db)} q {len(q)}")
    want = oracle.search(db, q)
    got, st, _ = run(db, q, m, mode=mode, tiling=tiling, kernel_overlap=True)
    bit = compare(got, want, db, "C1")
    assert bit
    assert st["n_overlap"] == want.n_overlap
    assert st["n_overlap_k"] == want.n_overlap
    if mode == "fp32_refine":
        assert st["n_refine"] >= st["n_hit"]
    assert st["n_eval"] >= st["n_overlap"]


def _fixture_cases():
    db, q = fx.random_small()
    yield "random_small", db, q, 3
    db, q = fx.random_small(n_e=700, n_q=300, box=6.0, seed=12, d=0.9)
    yield "random_mid", db, q, 17
    db, q = fx.dense_box()
    yield "dense_box", db, q, 9
    db, q = fx.all_hit()
    yield "all_hit", db, q, 5
    db, q, _ = fx.near_threshold()
    yield "near_threshold", db, q, 4
    db, q, params = fx.passing_pairs()
    yield "passing", db, q.with_d(np.array([p["d"] for p in params])), 8
    db, q, _ = fx.stationary_pairs()
    yield "stationary", db, q, 1
    # pairs whose computed roots cross (reading R8: the interval collapses to
    # the clamped vertex), each query against every fixture entry
    pairs = r8_collapse()
    q = fx.segments_from_rows([p[0] for p in pairs]).with_d(np.array([p[2] for p in pairs]))
    db = fx.segments_from_rows([p[1] for p in pairs])
    yield "r8_collapse", db, q, 3
    db, q, m = fx.comb_bins()
    yield "comb_bins", db, q, m


@pytest.mark.parametrize("mode", MODES)
def test_fixtures(mode):
    for name, db, q, m in _fixture_cases():
        say(f"fixture {name} {mode}")
        want = oracle.search(db, q)
        for tiling in ("periodic", "range"):
            got, st, _ = run(db, q, m, mode=mode, tiling=tiling)
            compare(got, want, db, f"{name}/{tiling}")
        if name == "all_hit":
            assert len(want) == want.n_overlap


@pytest.mark.parametrize("mode", MODES)
def test_launch_shape_invariance(mode):
    db, q = fx.dense_box(ntraj=300, L=40, box=8.0, nq=30, seed=31, d=1.1)
    want = oracle.search(db, q)
    assert len(want) > 200
    for m in (1, 7, 40, 1000):
        ix = tds.build_index(db, m)
        for block in (64, 128, 256, 512, 1024):
            for bs, grid in ((1, 0), (7, 1), (128, 3), (1000, 0)):
                for tiling in ("periodic", "range"):
                    say(f"invariance {mode} m={m} block={block} bs={bs} grid={grid} {tiling}")
                    got, st, _ = run(db, q, m, index=ix, mode=mode, block_size=block,
                                     batch_size=bs, grid=grid, tiling=tiling)
                    compare(got, want, db, f"m={m} block={block} bs={bs} {tiling}")
                    assert st["n_overlap"] == want.n_overlap


@pytest.mark.parametrize("mode", MODES)
def test_c2_reduced(mode):
    db = gen.make_db("C2", ntraj=300)
    qb = gen.make_queries("C2", nq=20)
    q = gen.concat([qb.with_d(d) for d in (1.0, 5.0, 25.0)])
    say(f"C2 reduced {mode}: db {len(db)} q {len(q)}")
    want = oracle.search(db, q)
    assert len(want) > 100
    for tiling, bs in (("periodic", 100), ("range", 512)):
        got, st, _ = run(db, q, 1000, mode=mode, tiling=tiling, batch_size=bs)
        compare(got, want, db, f"C2r/{tiling}")
        assert st["n_overlap"] == want.n_overlap


@pytest.mark.parametrize("mode", MODES)
def test_c3_reduced(mode):
    db = gen.make_db("C3", ntraj=2000, L=40)
    qb = gen.make_queries("C3", nq=30, L=40)
    q = gen.concat([qb.with_d(d) for d in (0.001, 0.01, 0.05)])
    say(f"C3 reduced {mode}: db {len(db)} q {len(q)}")
    want = oracle.search(db, q)
    assert len(want) > 10
    got, st, _ = run(db, q, 40, mode=mode, tiling="range", batch_size=256)
    compare(got, want, db, "C3r")


@pytest.mark.parametrize("mode", MODES)
def test_c4_reduced(mode):
    db = gen.make_db("C4", ntraj=300)
    q = gen.make_queries("C4", nq=24)
    say(f"C4 reduced {mode}: db {len(db)} q {len(q)}")
    want = oracle.search(db, q)
    got, st, _ = run(db, q, 1000, mode=mode, tiling="range", batch_size=256)
    compare(got, want, db, "C4r")
    got, st, _ = run(db, q, 400, mode=mode, tiling="periodic", batch_size=64)
    compare(got, want, db, "C4r/periodic")


def test_c5_requests_reduced():
    db = gen.make_db("C5", ntraj=500)
    ix = tds.build_index(db, 800)
    for r in range(4):
        q = gen.make_queries("C5", request=r)
        say(f"C5 request {r}: {len(q)} segments, d={q.d[0]:.3f}")
        want = oracle.search(db, q)
        for mode in MODES:
            got, st, _ = run(db, q, 800, index=ix, mode=mode, tiling="range", batch_size=128)
            compare(got, want, db, f"C5 req {r} {mode}")


def test_overflow_retry():
    # Every temporally overlapping pair hits, so one work unit selects up to
    # 256 pairs: more than a wave's slab of 64, the rest spills, and with room
    # for one spilled selection the search must grow and run again.
    db, q = fx.all_hit(n_e=4096, n_q=16)
    want = oracle.search(db, q)
    assert len(want) > 5000
    for mode in MODES:
        got, st, _ = run(db, q, 8, mode=mode, capacity=1, max_retries=2)
        compare(got, want, db, f"retry {mode}")
        assert st["retries"] == 1
        assert st["n_refine"] >= len(want)
    with pytest.raises(tds.TdsError) as e:
        run(db, q, 8, capacity=1, max_retries=0)
    assert e.value.code == L.TDS_EOVERFLOW
    # device output under a re-run: the translation enqueued before the wait
    # predates the re-run and is redone
    got, st, _ = run(db, q, 8, mode="fp32_refine", capacity=1, max_retries=2, out="device")
    compare(got, want, db, "retry device output")
    assert st["retries"] == 1
    # page-locked host output, which the record kernel writes directly
    got, st, _ = run(db, q, 8, mode="fp32_refine", capacity=1, max_retries=2, out="pinned")
    compare(got, want, db, "retry page-locked output")
    assert st["retries"] == 1
    # the same handle fetched repeatedly: its output buffer is sized from the
    # previous batch, so the early translation covers every hit (host,
    # device and page-locked host output)
    ix = tds.build_index(db, 8)
    qh = tds.Query(ix)
    try:
        for rep, out in enumerate(("host", "device", "pinned", "host", "device", "pinned")):
            qh.batch(q, q.d, mode="fp32_refine", tiling="range")
            compare(qh.fetch(out=out).sorted(), want, db, f"repeated fetch {rep} {out}")
    finally:
        qh.close()
        ix.close()
    # a dense box under the same small capacity
    db, q = fx.dense_box(ntraj=200, L=30, box=4.0, nq=20, seed=41, d=1.5)
    want = oracle.search(db, q)
    assert len(want) > 1000
    for mode in MODES:
        got, st, _ = run(db, q, 30, mode=mode, capacity=1, max_retries=4)
        compare(got, want, db, f"dense box {mode}")


def test_empty_inputs():
    db, q = fx.random_small()
    ix = tds.build_index(db, 8)
    got, st, _ = run(db, q.subset(np.arange(0)), 8, index=ix)
    assert len(got) == 0 and st["n_eval"] == 0
    ix0 = tds.build_index(db.subset(np.arange(0)), 8)
    got, st, _ = run(None, q, 8, index=ix0)
    assert len(got) == 0
    assert ix0.info()["n"] == 0
    # query entirely outside the database's time extent
    far = q.subset(np.arange(len(q)))
    far.t0 += 1e6
    far.t1 += 1e6
    got, st, _ = run(db, far, 8, index=ix)
    assert len(got) == 0 and st["n_eval"] == 0


def test_device_inputs_and_outputs():
    import torch
    db, q = fx.dense_box(ntraj=100, L=20, nq=10, seed=51)
    want = oracle.search(db, q)

    class Dev:
        pass

    dq = Dev()
    for f in gen.workloads.FIELDS:
        setattr(dq, f, torch.as_tensor(getattr(q, f), device="cuda"))
    ddb = Dev()
    for f in gen.workloads.FIELDS:
        setattr(ddb, f, torch.as_tensor(getattr(db, f), device="cuda"))
    ddb.traj = torch.as_tensor(db.traj, device="cuda")
    ix = tds.build_index(ddb, 20)
    qh = tds.Query(ix)
    qh.batch(dq, torch.as_tensor(q.d, device="cuda"), mode="fp32_refine", tiling="range")
    h = qh.fetch(out="device")
    assert h.query.is_cuda
    compare(h.sorted(), want, db, "device io")
    qh.close()


def test_invalid_device_query_reported_at_fetch():
    import torch
    db, q = fx.random_small()
    ix = tds.build_index(db, 4)

    class Dev:
        pass

    dq = Dev()
    for f in gen.workloads.FIELDS:
        setattr(dq, f, torch.as_tensor(getattr(q, f), device="cuda"))
    dq.t1[3] = dq.t0[3]
    qh = tds.Query(ix)
    qh.batch(dq, torch.as_tensor(q.d, device="cuda"))
    with pytest.raises(tds.TdsError) as e:
        qh.fetch()
    assert e.value.code == L.TDS_EINVAL
    # the handle is usable again afterwards
    dq.t1[3] = dq.t0[3] + 0.5
    q2 = q.subset(np.arange(len(q)))
    q2.t1[3] = q2.t0[3] + 0.5
    qh.batch(dq, torch.as_tensor(q.d, device="cuda"))
    compare(qh.fetch().sorted(), oracle.search(db, q2), db, "after error")
    qh.close()


def test_host_query_validation():
    db, q = fx.random_small()
    ix = tds.build_index(db, 4)
    bad = q.subset(np.arange(len(q)))
    bad.x0[1] = np.nan
    with pytest.raises(tds.TdsError) as e:
        run(db, bad, 4, index=ix)
    assert e.value.code == L.TDS_EINVAL
    with pytest.raises(tds.TdsError):
        run(db, q.with_d(-1.0), 4, index=ix)
    with pytest.raises(tds.TdsError):
        run(db, q, 4, index=ix, block_size=96)
    # host values are checked by the preparation kernel: the batch is
    # accepted, its fetch reports the segment, and the handle then runs a
    # valid batch (pageable and page-locked output)
    qh = tds.Query(ix)
    try:
        for bad_d in (False, True):
            bq = q.subset(np.arange(len(q)))
            if bad_d:
                bq = bq.with_d(1.0)
                bq.d[len(bq) // 2] = -1.0
            else:
                bq.t1[2] = bq.t0[2]
            qh.batch(bq, bq.d, mode="fp32_refine", tiling="range")
            with pytest.raises(tds.TdsError) as e:
                qh.fetch()
            assert e.value.code == L.TDS_EINVAL and "invalid query segment" in str(e.value)
            for out in ("host", "pinned"):
                qh.batch(q, q.d, mode="fp32_refine", tiling="range")
                compare(qh.fetch(out=out).sorted(), oracle.search(db, q), db, f"after error ({out})")
    finally:
        qh.close()


def test_torch_allocator_hook():
    """Device buffers served by torch's caching allocator give the same hits."""
    import torch
    db, q, m = gen.make_config("C1")
    want = oracle.search(db, q)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    tds.use_torch_allocator()
    try:
        ix = tds.build_index(db, m)
        during_index = torch.cuda.memory_allocated()
        assert during_index - before >= len(db) * 64  # the binary64 entry arrays at least
        for mode in MODES:
            got, st, _ = run(db, q, m, index=ix, mode=mode)
            compare(got, want, db, f"torch allocator {mode}")
        ix.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() <= before + (1 << 20)
    finally:
        tds.use_torch_allocator(False)
    # buffers made afterwards come from HIP again
    got, st, _ = run(db, q, m)
    compare(got, want, db, "hip allocator again")


def test_extreme_magnitudes():
    # Chunks that mix ordinary entries with entries beyond 2^100 (whose boxes
    # are unbounded, so the chunk's largest half-width is infinite and every
    # pair goes to the refine) and with very long segments; query segments
    # copy some of the huge entries (distance 0: hits among huge values) and
    # sit among the ordinary ones. A second case at the scale 1e-6 with a
    # threshold of 1e-7.
    rng = np.random.default_rng(17)

    def rows_for(n, scale, huge_every, long_every, seed_shift=0.0):
        out = []
        for i in range(n):
            p0 = rng.uniform(-5, 5, 3) * scale
            p1 = p0 + rng.normal(0, 0.5, 3) * scale
            if huge_every and i % huge_every == 7:
                p0, p1 = p0 * 1e31 / scale, p1 * 1e31 / scale
            if long_every and i % long_every == 13:
                p1 = p0 + rng.normal(0, 200, 3) * scale
            t0 = rng.uniform(0, 5)
            out.append([*p0, t0 + seed_shift, *p1, t0 + seed_shift + rng.uniform(0.5, 2)])
        return np.array(out)

    e = rows_for(600, 1.0, 50, 50)
    qrows = rows_for(40, 1.0, 0, 0)
    qrows = np.vstack([qrows, e[7::100]])  # copies of huge entries
    db = fx.segments_from_rows(e)
    q = fx.segments_from_rows(qrows).with_d(1.0)
    want = oracle.search(db, q)
    assert len(want) > 5
    for mode in MODES:
        got, _, _ = run(db, q, 8, mode=mode)
        compare(got, want, db, f"huge and long {mode}")
    e = rows_for(600, 1e-6, 0, 0)
    db = fx.segments_from_rows(e)
    q = fx.segments_from_rows(e[::15] + np.array([1e-8, 0, 0, 0, 1e-8, 0, 0, 0])).with_d(1e-7)
    want = oracle.search(db, q)
    assert len(want) >= 40
    for mode in MODES:
        got, _, _ = run(db, q, 8, mode=mode)
        compare(got, want, db, f"scale 1e-6 {mode}")


@pytest.mark.parametrize("mode", MODES)
def test_r8_collapse_pairs(mode):
    """Every fixture pair takes the collapse branch in the oracle; the device
    reports the same single time, bitwise."""
    pairs = r8_collapse()
    q = fx.segments_from_rows([p[0] for p in pairs]).with_d(np.array([p[2] for p in pairs]))
    db = fx.segments_from_rows([p[1] for p in pairs])
    want = oracle.search(db, q)
    diag = {(int(a), int(b)): (x, y) for a, b, x, y in zip(want.q, want.e, want.ta, want.tb)}
    for k in range(len(pairs)):
        assert diag[(k, k)][0] == diag[(k, k)][1]  # the collapse: one time
    got, st, _ = run(db, q, 3, mode=mode, tiling="range")
    assert compare(got, want, db, f"r8 {mode}")


def test_fig1_sec4_ranges_on_device():
    """The candidate ranges the device computes for the hand-worked intervals
    of tests/golden/fig1_sec4_ranges.txt (Fig. 1's bins)."""
    t0, t1, _, _ = fig1()
    db = fx.time_only(t0, t1)
    ranges, _ = fig1_sec4()
    q = fx.segments_from_rows([[0, 0, 0, a, 0, 0, 0, b] for a, b, _, _ in ranges]).with_d(1e9)
    h, st, (f, l) = run(db, q, 4)
    for k, (a, b, wf, wl) in enumerate(ranges):
        if wl < wf:
            assert l[k] < f[k], (a, b)
        else:
            assert (f[k], l[k]) == (wf, wl), (a, b)
    compare(h, oracle.search(db, q), db, "fig1 sec4 ranges")


def test_outlier_band_stays_local():
    """One entry of huge magnitude and extent widens the binary32 band only
    for the chunk that holds it: the pairs passed to the refine grow by at
    most that chunk's share, not by every pair of the batch."""
    db = gen.make_db("C2", ntraj=300)
    qb = gen.make_queries("C2", nq=20)
    q = gen.concat([qb.with_d(x) for x in (1.0, 5.0)])
    row = np.array([[3e12, -2e12, 1e12, 200.0, -4e12, 5e12, 2e12, 201.0]])
    out = fx.segments_from_rows(row)
    out.traj[:] = 999999
    db2 = gen.concat([db, out])
    want = oracle.search(db2, q)
    _, st1, _ = run(db, q, 1000, mode="fp32_refine", tiling="range")
    got, st2, _ = run(db2, q, 1000, mode="fp32_refine", tiling="range")
    compare(got, want, db2, "outlier")
    # query segments whose range holds the outlier's chunk (time step 200)
    n_step = int(np.sum((q.t0 < 201.0) & (q.t1 > 200.0)))
    say(f"outlier: refined {st1['n_refine']} -> {st2['n_refine']} ({n_step} query segments at its step)")
    assert st2["n_refine"] - st1["n_refine"] <= st2["chunk"] * n_step
    assert st2["n_refine"] < st1["n_refine"] + 0.05 * st2["n_eval"]


def test_handle_reuse_across_batches():
    """One query handle runs batches of several tilings, sizes and modes in a
    row (each batch starts from the counters the previous batch's last
    kernel cleared, or from a clearing kernel after a buffer grew, an empty
    batch or an invalid one); every batch equals the oracle."""
    db = gen.make_db("C4", ntraj=300)
    qa = gen.make_queries("C4", nq=12)
    qb = gen.make_queries("C4", nq=40)
    want_a, want_b = oracle.search(db, qa), oracle.search(db, qb)
    ix = tds.build_index(db, 800)
    qh = tds.Query(ix)
    import torch
    empty = qa.subset(np.arange(0))
    # device segments are checked by the preparation kernel: an invalid one
    # fails the batch at fetch time, after its kernels ran
    bad = qa.subset(np.arange(4))
    bad.t1 = bad.t0.copy()  # t_end == t_start: invalid
    for f in ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1"):
        setattr(bad, f, torch.as_tensor(getattr(bad, f), device="cuda"))
    seq = [("a", "range", "fp32_refine"), ("a", "range", "fp32_refine"), ("b", "periodic", "fp64"),
           ("a", "greedy_min", "fp32_refine"), ("empty", "range", "fp64"), ("b", "greedy_max", "fp32_refine"),
           ("bad", "range", "fp32_refine"), ("a", "range", "fp64"), ("b", "range", "fp32_refine"),
           ("a", "periodic", "fp32_refine")]
    try:
        for k, (which, tiling, mode) in enumerate(seq):
            q = {"a": qa, "b": qb, "empty": empty, "bad": bad}[which]
            d = q.d if which != "bad" else torch.ones(4, dtype=torch.float64, device="cuda")
            qh.batch(q, d, mode=mode, tiling=tiling, batch_size=64)
            if which == "bad":
                with pytest.raises(tds.TdsError):
                    qh.fetch()
                continue
            got = qh.fetch().sorted()
            if which == "empty":
                assert len(got) == 0
                continue
            compare(got, want_a if which == "a" else want_b, db, f"batch {k}: {which} {tiling} {mode}")
    finally:
        qh.close()
        ix.close()


def _staggered(seg, seed):
    """The segments with each trajectory's times shifted by its own offset in
    [0, 1), so that start times spread over every bin of a fine bin table."""
    rng = np.random.Generator(np.random.PCG64(seed))
    off = rng.random(int(seg.traj.max()) + 1)
    out = seg.subset(np.arange(len(seg)))
    out.t0 = out.t0 + off[out.traj]
    out.t1 = out.t1 + off[out.traj]
    return out


@pytest.mark.parametrize("mode", MODES)
def test_bucket_offsets_in_and_beyond_lds(mode):
    """Bucket counts whose offsets fit LDS are scanned inside the scatter
    (every workgroup scans them itself); more buckets take the separate
    one-workgroup scan and scatter. Range tiling with 1,500 non-empty bins
    (6,000 buckets) and with 3,000 (12,000), Periodic with m = 3,000 and
    10,000 (m buckets): every result equals the oracle."""
    db = _staggered(gen.make_db("C2", ntraj=120), 41)
    q = db.subset(np.flatnonzero(db.traj < 12))  # 12 trajectories moved by 0.5 in x
    q.x0 = q.x0 + 0.5
    q.x1 = q.x1 + 0.5
    q = q.with_d(2.0)
    want = oracle.search(db, q)
    assert len(want) >= len(q)
    for m, tiling in ((1500, "range"), (3000, "range"), (3000, "periodic"), (10000, "periodic")):
        ix = tds.build_index(db, m)
        try:
            nb = ix.info()["nonempty_bins"]
            say(f"buckets {mode} {tiling} m={m}: {nb} non-empty bins")
            if tiling == "range":
                assert nb * 4 > 8192 if m == 3000 else nb * 4 <= 8192
            got, st, _ = run(db, q, m, index=ix, mode=mode, tiling=tiling, batch_size=64)
            compare(got, want, db, f"{tiling} m={m}")
        finally:
            ix.close()


def test_partial_fetch_is_a_valid_subset():
    # cap < number of hits: min(cap, n) records in an unspecified order, each
    # one of the batch's hits with its interval, none twice; n_total is n;
    # a later full fetch of the same batch returns every hit (device,
    # pageable host and page-locked host output, both forms)
    db, q = fx.dense_box(ntraj=200, L=30, box=4.0, nq=20, seed=43, d=1.5)
    want = oracle.search(db, q)
    n = len(want)
    assert n > 300
    key = {(int(a), int(b)): (ta, tb) for a, b, ta, tb in zip(want.q, want.e, want.ta, want.tb)}
    ix = tds.build_index(db, 30)
    qh = tds.Query(ix)
    try:
        for mode in ("fp64", "fp32_refine"):
            for out in ("device", "host", "pinned"):
                for cap in (0, 1, n // 3, n - 1):
                    qh.batch(q, q.d, mode=mode, tiling="range")
                    part = qh.fetch(out=out, cap=cap).numpy()
                    label = f"{mode} {out} cap {cap}"
                    assert len(part.query) == cap, label
                    pairs = set(zip(part.query.tolist(), part.entry.tolist()))
                    assert len(pairs) == cap, f"{label}: duplicate records"
                    for a, b, ta, tb in zip(part.query, part.entry, part.ta, part.tb):
                        wa, wb = key[(int(a), int(b))]
                        assert abs(ta - wa) <= 1e-9 * max(1.0, abs(wa)), label
                        assert abs(tb - wb) <= 1e-9 * max(1.0, abs(wb)), label
                    compare(qh.fetch(out=out).sorted(), want, db, f"{label}, then in full")
    finally:
        qh.close()
        ix.close()


def test_two_handles_on_one_stream():
    # each handle's fetch waits for its own work on the shared stream (an
    # event after it), in either fetch order, with host and device output
    import torch
    db, q = fx.dense_box(ntraj=120, L=25, box=4.0, nq=16, seed=47, d=1.2)
    q2 = q.with_d(0.6)
    want1, want2 = oracle.search(db, q), oracle.search(db, q2)
    ix = tds.build_index(db, 25)
    s = torch.cuda.Stream()
    ha, hb = tds.Query(ix), tds.Query(ix)
    try:
        for order in ("ab", "ba"):
            for out in ("host", "device"):
                ha.batch(q, q.d, mode="fp32_refine", tiling="range", stream=s)
                hb.batch(q2, q2.d, mode="fp64", tiling="range", stream=s)
                got = {}
                for k in order:
                    with torch.cuda.stream(s):
                        got[k] = (ha if k == "a" else hb).fetch(out=out).sorted()
                compare(got["a"], want1, db, f"handle a ({order}, {out})")
                compare(got["b"], want2, db, f"handle b ({order}, {out})")
    finally:
        ha.close()
        hb.close()
        ix.close()
