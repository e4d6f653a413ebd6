"""Helpers shared by the GPU tests: run the library, compare with the oracle."""
import sys

import numpy as np

import oracle
import paper_1405_7461_amd as tds

TOL = 1e-9  # interval ends: |got - want| <= TOL * max(1, |want|)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(db, q, m, index=None, out="host", **opts):
    opts.setdefault("count_overlap", True)
    ix = index if index is not None else tds.build_index(db, m)
    qh = tds.Query(ix)
    try:
        qh.batch(q, q.d, **opts)
        h = qh.fetch(out=out)
        st = qh.stats()
        rng = qh.ranges()
    finally:
        qh.close()
    return h.sorted(), st, rng


def compare(got, want: "oracle.Hits", db=None, label=""):
    """Identical (query, entry) sets; ends within TOL; trajectory ids copied."""
    gq, ge = np.asarray(got.query), np.asarray(got.entry)
    assert len(gq) == len(want), f"{label}: {len(gq)} hits vs oracle {len(want)}"
    assert np.array_equal(gq, want.q) and np.array_equal(ge, want.e), f"{label}: hit sets differ"
    for g, w in ((got.ta, want.ta), (got.tb, want.tb)):
        err = np.abs(np.asarray(g) - w) / np.maximum(1.0, np.abs(w))
        assert err.size == 0 or err.max() <= TOL, f"{label}: end error {err.max()}"
    if db is not None and len(gq):
        assert np.array_equal(np.asarray(got.traj), db.traj[ge]), f"{label}: traj ids"
    bitwise = bool(np.array_equal(got.ta, want.ta) and np.array_equal(got.tb, want.tb))
    return bitwise
