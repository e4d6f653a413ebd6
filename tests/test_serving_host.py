"""Serving scheduler logic on the CPU, with the oracle standing in for the GPU.

Checks admission by estimated result bytes, continuous batching (requests
that arrive while a batch runs join a later batch), splitting of a batch's
hits back to its requests, and the alpha-per-epoch estimate.
"""
import time

import numpy as np

from gen import fixtures as fx
import oracle
from paper_1405_7461_amd import api
from paper_1405_7461_amd.serving import AlphaModel, Request, Server, poisson_arrivals


class OracleExecutor:
    def __init__(self, db, delay=0.002):
        self.db = db
        self.delay = delay
        self.calls = []

    def __call__(self, seg, d, capacity):
        from gen.workloads import Segments
        n = len(seg.t0)
        q = Segments(*[np.asarray(getattr(seg, f)) for f in ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1")],
                     traj=np.zeros(n, np.int64), seg=np.zeros(n, np.int64), d=np.asarray(d))
        h = oracle.search(self.db, q)
        time.sleep(self.delay)
        self.calls.append((n, capacity))
        return (api.Hits(h.q, h.e, self.db.traj[h.e], h.ta, h.tb),
                {"retries": 0, "ms_pair": 0.0})


def _requests(nq=12):
    db, q = fx.dense_box(ntraj=60, L=20, box=4.0, nq=nq, seed=77, d=0.9)
    reqs = []
    for i in range(nq):
        sel = np.nonzero(q.traj == i)[0]
        sub = q.subset(sel)
        reqs.append(Request(rid=i, seg=sub, d=np.full(len(sel), 0.5 + 0.1 * i)))
    return db, reqs


def test_batches_split_back_to_requests():
    db, reqs = _requests()
    arr = poisson_arrivals(len(reqs), rate=2000.0, seed=3)
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    ex = [OracleExecutor(db), OracleExecutor(db)]
    it = iter(ex)
    srv = Server(None, pool_bytes=24 * 4.0 * 3, streams=2, executor_factory=lambda: next(it))
    stats = srv.run(reqs)
    assert stats["n_requests"] == len(reqs)
    assert stats["n_batches"] >= 4          # the pool admits at most three at a time
    assert max(b["n_req"] for b in srv.batches) <= 3
    for r in reqs:
        assert r.arrival <= r.t_admit + 1e-9 <= r.t_done + 1e-9
        want = oracle.search(db, r.seg.with_d(r.d))
        got = r.hits.sorted()
        assert np.array_equal(got.query, want.q) and np.array_equal(got.entry, want.e)
        assert np.array_equal(got.ta, want.ta) and np.array_equal(got.tb, want.tb)


def test_single_oversized_request_still_runs():
    db, reqs = _requests(3)
    for r in reqs:
        r.arrival = 0.0
    it = iter([OracleExecutor(db)])
    srv = Server(None, pool_bytes=1.0, streams=1, executor_factory=lambda: next(it))
    srv.run(reqs)
    assert all(b["n_req"] == 1 for b in srv.batches)   # each admitted alone
    assert all(r.hits is not None for r in reqs)


def test_alpha_model_tracks_hit_fraction():
    am = AlphaModel(0.0, 100.0, epochs=10, prior=1e-3, smoothing=0.0)
    t0 = np.array([5.0, 15.0, 15.0, 95.0])
    ev = np.array([100.0, 200.0, 200.0, 50.0])
    hits = np.array([10.0, 4.0, 0.0, 50.0])
    am.update(t0, ev, hits)
    assert np.isclose(am.alpha[0], 0.1) and np.isclose(am.alpha[1], 0.01) and np.isclose(am.alpha[9], 1.0)
    assert np.isclose(am.alpha[5], 1e-3)   # unseen epochs keep the prior
    assert np.isclose(am.expected_hits([5.0, 95.0], [10.0, 10.0]), 1.0 + 10.0)


def test_poisson_arrivals_rate():
    a = poisson_arrivals(20000, rate=50.0, seed=1)
    assert np.all(np.diff(a) > 0)
    assert abs(len(a) / a[-1] - 50.0) < 2.0
