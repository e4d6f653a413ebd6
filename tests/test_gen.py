"""Workload generators: shapes, determinism, and the recipes' stated sizes."""
import numpy as np

import gen


def test_deterministic():
    a = gen.make_db("C1")
    b = gen.make_db("C1")
    for x, y in zip(a.arrays(), b.arrays()):
        assert np.array_equal(x, y)


def test_c1_c2_shapes():
    db = gen.make_db("C1")
    assert len(db) == 200 * 100
    assert db.t0.min() == 0 and db.t1.max() == 100
    q = gen.make_queries("C1")
    assert len(q) == 1000 and np.all(q.d == 2.0)
    db2 = gen.make_db("C2", ntraj=25)
    assert len(db2) == 25 * 400
    # the database's steps are Gaussian with unit variance per axis
    dx = db2.x1 - db2.x0
    assert 0.9 < dx.std() < 1.1


def test_segments_chain():
    db = gen.make_db("C2", ntraj=3, L=5)
    # consecutive segments of one trajectory share their vertex
    for t in range(3):
        s = np.nonzero(db.traj == t)[0]
        assert np.array_equal(db.x1[s[:-1]], db.x0[s[1:]])
        assert np.array_equal(db.t1[s[:-1]], db.t0[s[1:]])


def test_c3_plummer():
    db = gen.make_db("C3", ntraj=200, L=10)
    r = np.sqrt(db.x0 ** 2 + db.y0 ** 2 + db.z0 ** 2)
    assert r.max() < 10.01
    # Plummer: half-mass radius ~ 1.305 a
    assert 0.9 < np.median(r[db.seg == 0]) < 1.8


def test_c4_queries():
    q = gen.make_queries("C4", nq=40)
    lens = q.meta["lengths"]
    assert lens.min() >= 10 and lens.max() <= 2000
    assert np.all(np.isin(q.d, [1.0, 5.0, 25.0]))
    # durations 1/8 and starts on the 1/64 grid: exact in binary32 as well
    assert np.all(q.t1 - q.t0 == 0.125)
    assert np.all((q.t0 * 64) == np.round(q.t0 * 64))
    assert q.t1.max() <= 400


def test_c5_requests():
    r = [gen.make_queries("C5", request=i) for i in range(20)]
    for q in r:
        assert 10 <= len(q) <= 5000
        assert 0.5 <= q.d[0] <= 50 and np.all(q.d == q.d[0])
        assert np.all(q.t1 - q.t0 == 1.0 / 16)
    assert len({len(q) for q in r}) > 5
