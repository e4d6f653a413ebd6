"""Batching and serving forms on the GPU.

* Serving: every request's hits are the same when it runs alone and when it
  shares batches with other requests under continuous batching.
* Autotuner: all searched launch configurations report the same hits, and the
  chosen configuration reproduces the oracle.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_1405_7461_amd as tds
from paper_1405_7461_amd.autotune import tune
from paper_1405_7461_amd.serving import Request, Server, poisson_arrivals
from gpu_util import compare, run, say

pytestmark = pytest.mark.gpu


def _c5_requests(n):
    reqs = []
    for i in range(n):
        q = gen.make_queries("C5", request=i)
        reqs.append(Request(rid=i, seg=q, d=q.d.copy()))
    return reqs


def test_serving_alone_equals_mixed():
    db = gen.make_db("C5", ntraj=600)
    ix = tds.build_index(db, 800)
    reqs = _c5_requests(24)
    alone = {}
    qh = tds.Query(ix)
    for r in reqs:
        qh.batch(r.seg, r.d, mode="fp32_refine", tiling="range")
        alone[r.rid] = qh.fetch().sorted()
    qh.close()
    # arrivals faster than the two streams serve them one by one, so
    # requests wait and are batched together
    arr = poisson_arrivals(len(reqs), rate=20000.0, seed=11)
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    # the executors' buffers, grown by a warm-up, count against the pool,
    # with 2e5 bytes of result estimates beyond them; two streams overlap
    # the batches
    srv = Server(ix, pool_bytes=64e6, streams=2, k_safety=2.0,
                 opts=dict(mode="fp32_refine", tiling="range"))
    srv.warmup(reqs[:2])
    assert min(srv.reserved) > 0
    srv.pool_bytes = sum(srv.reserved) + 2e5
    stats = srv.run(reqs)
    srv.close()
    say(f"serving: {stats}")
    assert stats["n_batches"] > 1 and max(b["n_req"] for b in srv.batches) > 1
    for r in reqs:
        a, b = alone[r.rid], r.hits.sorted()
        assert np.array_equal(a.query, b.query) and np.array_equal(a.entry, b.entry)
        assert np.array_equal(a.ta, b.ta) and np.array_equal(a.tb, b.tb)
        assert np.array_equal(a.traj, b.traj)
    # and two of them against the oracle
    for r in reqs[:2]:
        compare(r.hits.sorted(), oracle.search(db, r.seg), db, f"request {r.rid}")


def test_autotune_consistent(tmp_path):
    db = gen.make_db("C4", ntraj=400)
    q = gen.make_queries("C4", nq=20)
    res = tune(db, q, q.d, num_bins=(200, 800), blocks=(64, 256), batch_sizes=(64, 256), reps=1,
               cache=tmp_path / "tune.json", log=say)
    # per bin count and block size: range, then Periodic, GreedySetSplit-Min
    # and -Max at each of the two sizes
    assert len(res.trials) == 2 * 2 * (1 + 3 * 2)
    assert {t.opts["tiling"] for t in res.trials} == {"range", "periodic", "greedy_min", "greedy_max"}
    assert (tmp_path / "tune.json").exists()
    got, st, _ = run(db, q, res.num_bins, **res.opts)
    compare(got, oracle.search(db, q), db, "tuned")
    # a second call is served from the cache
    res2 = tune(db, q, q.d, num_bins=(200, 800), cache=tmp_path / "tune.json")
    assert res2.num_bins == res.num_bins and res2.opts == res.opts and not res2.trials
