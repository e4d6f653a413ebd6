"""The response-time model on the GPU (Sec. 8).

* each synthetic benchmark batch holds one class of interactions only (all
  hits, all temporal misses, all spatial misses, no candidates), checked
  with the device's own counts;
* beta from the device's exact overlap count equals the host plan's and the
  oracle's nested loops;
* calibration fills every curve; alpha per epoch meets the paper's 5%
  criterion on C1; a prediction is finite and of the measured magnitude.
"""
import time

import numpy as np
import pytest

import gen
import paper_1405_7461_amd as tds
from paper_1405_7461_amd import perfmodel as M
from oracle import batching as ob
from oracle import perfmodel as pm
from gpu_util import say

pytestmark = pytest.mark.gpu


def test_benchmark_classes():
    rng = np.random.default_rng(1)
    for ent, kind, want in (("near", "hit", "hit"), ("split", "tmiss", "tmiss"),
                            ("near", "smiss", "smiss"), ("near", "noop", "noop")):
        e = M._entries(ent, 1024, rng)
        q = M._queries(kind, 64, rng)
        ix = tds.build_index(e, 1)
        qh = tds.Query(ix)
        try:
            qh.batch(q, q.d, mode="fp32_refine", tiling="range", count_overlap=True)
            h = qh.fetch()
            st = qh.stats()
        finally:
            qh.close()
            ix.close()
        n_int, n_ovl = st["n_eval"], st["n_overlap"]
        if want == "hit":
            assert n_int == 64 * 1024 and n_ovl == n_int and len(h) == n_int
        elif want == "tmiss":
            assert n_int == 64 * 1024 and n_ovl == 0 and len(h) == 0
        elif want == "smiss":
            assert n_int == 64 * 1024 and n_ovl == n_int and len(h) == 0
        else:
            assert n_int == 0 and len(h) == 0


def test_beta_device_host_oracle():
    db, q, m = gen.make_config("C1")
    ix = tds.build_index(db, m)
    qh = tds.Query(ix)
    try:
        qh.batch(q, q.d, mode="fp32_refine", tiling="range", count_overlap=True)
        qh.fetch()
        st = qh.stats()
        w = M.workload_terms(ix, q)
    finally:
        qh.close()
    beta_dev = 1 - st["n_overlap"] / st["n_eval"]
    assert w["interactions"] == st["n_eval"] and w["n_overlap"] == st["n_overlap"]
    o = ob.entry_order(db.t0)
    bins = ob.bin_table(db.t0[o], db.t1[o], m)
    sub = np.arange(0, len(q), 10)  # nested loops on every tenth segment
    rr = [ob.candidate_range(bins, q.t0[k], q.t1[k]) for k in sub]
    first = np.array([r[0] if r else 0 for r in rr])
    last = np.array([r[1] if r else -1 for r in rr])
    beta_or = pm.beta_nested_loops(q.t0[sub], q.t1[sub], db.t0[o], db.t1[o], first, last)
    s0, s1 = ix.sorted_times()
    n_ovl_sub = (np.searchsorted(s0, q.t1[sub], side="left") - np.searchsorted(s1, q.t0[sub], side="right")).sum()
    assert abs(beta_or - (1 - n_ovl_sub / np.sum(np.maximum(last - first + 1, 0)))) < 1e-12
    say(f"C1 beta: device {beta_dev:.6f}, host plan {1 - w['n_overlap'] / w['interactions']:.6f}")
    ix.close()


def test_periodic_interactions_host_equals_device():
    """The model's Periodic interactions follow the device's order exactly,
    also where query segments of one t_start bin have different ends (C4)."""
    db = gen.make_db("C4", ntraj=300)
    q = gen.make_queries("C4", nq=24)
    ix = tds.build_index(db, 1000)
    qh = tds.Query(ix)
    try:
        for s in (1, 7, 64, 1000):
            qh.batch(q, q.d, mode="fp32_refine", tiling="periodic", batch_size=s)
            qh.fetch()
            st = qh.stats()
            w = M.workload_terms(ix, q, tiling="periodic", batch_size=s)
            assert w["interactions"] == st["n_eval"] and w["n_tiles"] == st["n_tiles"], s
    finally:
        qh.close()
        ix.close()


def test_calibrate_alpha_predict():
    t0 = time.perf_counter()
    model = M.calibrate(qs=(16, 256, 2048), cs=(256, 4096), reps=2, log=say)
    say(f"calibration {time.perf_counter() - t0:.1f} s, cpu fit {model.cpu}")
    for k in ("hit", "tmiss", "smiss", "noop"):
        for c, (xs, ys) in model.tables[k].items():
            assert len(xs) >= 2 and np.all(np.isfinite(ys)) and np.all(ys > 0)
    db, q, m = gen.make_config("C1")
    ix = tds.build_index(db, m)
    try:
        rep = gen.workloads.uniform_walk(gen.workloads.rng_for(1, 7), 10, 100, 100.0, 1.0).with_d(2.0)
        est = M.estimate_alpha(model, ix, rep, num_epochs=50, s=64)
        say(f"alpha estimate: {est}")
        assert est["rel_error"] <= 0.05 or est["rounds"] == 8
        p = model.predict(ix, q, host_inputs=True, host_output=True)
        qh = tds.Query(ix)
        try:
            ms = []
            for _ in range(6):
                t1 = time.perf_counter()
                qh.batch(q, q.d, mode="fp32_refine", tiling="range")
                qh.fetch()
                ms.append((time.perf_counter() - t1) * 1e3)
        finally:
            qh.close()
        say(f"C1 predicted {p} measured {np.median(ms):.4f} ms")
        assert np.isfinite(p["ms"]) and 0.2 < p["ms"] / np.median(ms) < 5.0
    finally:
        ix.close()
