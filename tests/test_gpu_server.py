"""The library's serving runtime (tds_server_*) on the GPU.

* Every request's hits are the same when it runs alone (tds_query_batch) and
  when the native scheduler batches it with others over several streams,
  at staggered (Poisson) arrivals and all at once; two against the oracle.
* Requests that find the waiting queue full are refused (TDS_EBUSY): at
  submission when they have already arrived, at arrival otherwise.
* The alpha estimate moves from its prior towards the observed hit rate.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_1405_7461_amd as tds
from paper_1405_7461_amd import _lib as L
from paper_1405_7461_amd.serving import poisson_arrivals
from gpu_util import compare, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c5_small():
    db = gen.make_db("C5", ntraj=600)
    ix = tds.build_index(db, 800)
    reqs = [gen.make_queries("C5", request=i) for i in range(32)]
    alone = []
    qh = tds.Query(ix)
    for q in reqs:
        qh.batch(q, q.d, mode="fp32_refine", tiling="range")
        alone.append(qh.fetch().sorted())
    qh.close()
    yield db, ix, reqs, alone
    ix.close()


def _same(a, b):
    return (np.array_equal(a.query, b.query) and np.array_equal(a.entry, b.entry)
            and np.array_equal(a.traj, b.traj) and np.array_equal(a.ta, b.ta)
            and np.array_equal(a.tb, b.tb))


@pytest.mark.parametrize("arrivals", ["poisson", "at_once"])
def test_server_alone_equals_batched(c5_small, arrivals):
    db, ix, reqs, alone = c5_small
    # a small batch bound forces several batches in flight on the streams
    srv = tds.NativeServer(ix, streams=3, max_batch_segments=4096, reserve_segments=4096,
                           pool_bytes=64 << 20, mode="fp32_refine", tiling="range")
    t0 = srv.now() + 0.01
    arr = poisson_arrivals(len(reqs), rate=2000.0, seed=21) if arrivals == "poisson" else np.zeros(len(reqs))
    ids = [srv.submit(q, q.d, t0 + float(a)) for q, a in zip(reqs, arr)]
    infos = [srv.wait(i, timeout=60.0) for i in ids]
    batches = {inf["batch"] for inf in infos}
    say(f"server ({arrivals}): {len(batches)} batches, stats {srv.stats()}, "
        f"max requests per batch {max(inf['n_batch_requests'] for inf in infos)}")
    assert len(batches) > 1
    for k, (i, inf) in enumerate(zip(ids, infos)):
        assert inf["status"] == L.TDS_OK
        assert inf["arrival"] <= inf["admit"] <= inf["done"]
        got = srv.results(i).sorted()
        assert inf["n_hit"] == len(got)
        assert _same(alone[k], got), f"request {k}"
    for k in range(2):
        compare(srv.results(ids[k]).sorted(), oracle.search(db, reqs[k]), db, f"request {k}")
    for i in ids:
        srv.release(i)
    srv.close()


def test_server_refuses_when_queue_full(c5_small):
    db, ix, reqs, alone = c5_small
    srv = tds.NativeServer(ix, streams=1, max_batch_segments=4096, reserve_segments=4096,
                           max_waiting=5, mode="fp32_refine", tiling="range")
    # twelve requests that arrive at the same future time: the scheduler moves
    # them to the ready queue together, so exactly five are accepted
    t = srv.now() + 0.05
    ids = [srv.submit(q, q.d, t) for q in reqs[:12]]
    infos = [srv.wait(i, timeout=60.0) for i in ids]
    status = [inf["status"] for inf in infos]
    say(f"queue full at arrival: statuses {status}")
    assert status.count(L.TDS_OK) == 5 and status.count(L.TDS_EBUSY) == 7
    for k, (i, inf) in enumerate(zip(ids, infos)):
        if inf["status"] == L.TDS_OK:
            assert _same(alone[k], srv.results(i).sorted())
    srv.close()
    # already-arrived requests are refused at submission once five wait; the
    # one executor is kept busy by a large first request (10,000 segments
    # spanning the whole time extent, binary64: about 2.4e9 pair tests)
    srv = tds.NativeServer(ix, streams=1, max_batch_segments=1, reserve_segments=10000,
                           max_waiting=5, mode="fp64", tiling="range")
    big = db.subset(np.arange(10000)).with_d(0.5)
    big.t0 = np.zeros(10000)
    big.t1 = np.full(10000, 400.0)
    refused = 0
    accepted = [srv.submit(big, big.d, 0.0)]
    for q in reqs[8:30]:
        try:
            accepted.append(srv.submit(q, q.d, 0.0))
        except tds.TdsError as e:
            assert e.code == L.TDS_EBUSY
            refused += 1
    for i in accepted:
        assert srv.wait(i, timeout=60.0)["status"] == L.TDS_OK
    say(f"queue full at submission: {refused} refused, {len(accepted)} accepted")
    assert refused > 0
    srv.close()


def test_server_alpha_moves(c5_small):
    db, ix, reqs, alone = c5_small
    srv = tds.NativeServer(ix, streams=2, max_batch_segments=2048, reserve_segments=2048,
                           alpha_prior=0.5, mode="fp32_refine", tiling="range")
    before = srv.alpha()
    ids = [srv.submit(q, q.d, 0.0) for q in reqs[:16]]
    for i in ids:
        srv.wait(i, timeout=60.0)
    after = srv.alpha()
    srv.close()
    assert np.all(before == 0.5)
    # hits are rare: every epoch that saw candidates moved far below the prior
    moved = after < 0.5
    say(f"alpha: {moved.sum()} of {len(after)} epochs updated, min {after.min():.3g}")
    assert moved.sum() > 0 and np.all(after[moved] < 0.26)
