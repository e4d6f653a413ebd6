#!/usr/bin/env python3
"""Benchmark: segment-pair tests/s of the distance-threshold search on one GPU.

Headline workload (the precision form): a database of 5,000,000 segments
(10,000 trajectories x 500 unit-time steps on circular orbits whose radii
follow a Plummer density, scale radius 1, with N(0, 1e-4^2) jitter per
axis) indexed with 500 temporal bins, and 100,000 query segments (200 new
trajectories of the same generator) searched at d = 0.001 and d = 0.01: one
step is one query batch of the 200,000 (segment, d) pairs through the whole
hot path (query records, candidate ranges, sort, tiles, pair kernel,
compaction, overflow check, translation of the hits into caller indices in
device memory). Both exact forms are timed from the same index: the binary32
filter + binary64 refine (headline) and the plain binary64 kernel.

value = N_ovl / T_step, where N_ovl is the number of (query, entry) pairs
whose time spans overlap with positive length (independent of the
implementation) and T_step the wall time of one step with inputs already in
device memory.

Extras in the same JSON line: the at-scale plain workload (1M-segment
Gaussian walk, 40,000 query segments x d in {1, 5, 25}) in both forms and
under each tiling, host-memory (PCIe-inclusive) steps, trajectory-level
answers, the batching form (uneven queries, autotuned), the response-time
model, the serving form (10M-segment index, Poisson arrivals) and the oracle
timed on the host's cores (all, and one).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "segment-pair tests/s + p99 query latency; FP32+FP64-refine vs FP64, exact hits"
D_VALUES = (1.0, 5.0, 25.0)      # the at-scale plain workload
NUM_BINS = 1000
# batches in flight in the timed steps of the headline forms (query handles on
# their own streams)
PIPE_DEPTH = 3
HEAD_D = (0.001, 0.01)           # the precision-form workload
PLAIN_WORKLOAD = ("C2 plain at scale: 1M-segment Gaussian random walk (2,500 x 400), "
                  "40,000 query segments x d in {1,5,25} (120,000 per step), 1,000 bins")
HEAD_WORKLOAD = ("C3 precision form: 5M segments on Plummer-sphere circular orbits (10,000 x 500), "
                 "100,000 query segments x d in {0.001, 0.01} (200,000 per step), 500 bins")

# MI355X peaks (published figures, and the unit counts behind them): binary32
# vector 157.3 TFLOP/s = 256 CUs x 4 SIMDs x 32 lanes x 2 flops (FMA) x 2.4 GHz,
# which non-packed binary32 multiply-adds reach (the issue-rate probe measures
# v_fmac_f32 at 2.4 cycles per wave64 instruction); binary64 vector 78.6
# TFLOP/s = 16 lanes x 2 flops per SIMD-cycle (v_fma_f64 at 4.4 cycles).
FP32_PEAK = 157.3e12
FP64_PEAK = 78.6e12
# Algorithmic work per pair:
FP64_FLOPS_PER_PAIR = 49          # binary64 decision per overlapping pair, FMA = 2
# binary32 ball test per candidate pair: s = e2 + (-2C).c as three
# multiply-adds (6 flops) and its comparison with the query's threshold
FILTER_FLOPS_PER_PAIR = 7


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SRC = os.path.join(ROOT, "paper_1405_7461_amd", "csrc", "tds_kernels.hip")


def measured_traffic(summary: str):
    """HBM bytes per launch of the pair kernel from a committed counter summary.

    The summary (profiles/*.txt) records the FETCH_SIZE + WRITE_SIZE reading per
    dispatch, already scaled by the copy-kernel calibration, together with the
    SHA-256 of the kernel source it was taken on; a changed source gives None.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    try:
        fields = dict(line.split(":", 1) for line in open(path) if ":" in line)
    except OSError:
        return None
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256", "").strip() != src:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def overlap_count(db, q) -> int:
    """Pairs with max(t_start) < min(t_end), counted from sorted time arrays."""
    t0s = np.sort(db.t0)
    t1s = np.sort(db.t1)
    return int((np.searchsorted(t0s, q.t1, side="left") - np.searchsorted(t1s, q.t0, side="right")).sum())


def make_workload(name="C3"):
    import gen
    db = gen.make_db(name)
    qb = gen.make_queries(name)
    q = gen.concat([qb.with_d(d) for d in (HEAD_D if name == "C3" else D_VALUES)])
    return db, q, gen.CONFIGS[name]["bins"]


def to_device(seg):
    import torch

    class Dev:
        pass

    out = Dev()
    for f in ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1"):
        setattr(out, f, torch.as_tensor(getattr(seg, f), device="cuda"))
    out.d = torch.as_tensor(seg.d, device="cuda")
    return out


def run_form(ix, dq, opts, steps, warmup, n_ovl, depth=1):
    """Time one form on one batch.

    A step is a C caller's whole pass over the batch: tds_query_batch, then
    tds_fetch_results into device memory (which waits for the batch). The
    device arrays, options and output buffers are set up once; every step's
    hit count is checked against an untimed first pass.

    depth 1: `steps` steps one at a time (each waits for its results before
    the next is enqueued), with HIP events on the pair kernel's dispatch.
    depth > 1, three phases of `steps` steps each:
      1. one at a time, with the pair kernel's events (its launch time: the
         roofline's; in the phases below kernels of other batches overlap it);
      2. one at a time without events: the latency of a batch alone (p50/p99);
      3. the timed throughput: `depth` batches in flight on `depth` query
         handles, each on its own stream (the fetch of step i follows the
         enqueue of step i + depth - 1), no events: ms_per_step = this
         phase's wall time / steps."""
    import torch
    import paper_1405_7461_amd as tds
    import ctypes as C
    from paper_1405_7461_amd import _lib as L
    lib = L.lib()
    qh = tds.Query(ix)
    stream = torch.cuda.current_stream()
    # one untimed pass that also counts overlapping pairs (checked against N_ovl)
    qh.batch(dq, dq.d, count_overlap=True, stream=stream, **opts)
    counted_hits = len(qh.fetch(out="device"))
    counted = qh.stats()["n_overlap"]
    prep = tds.prepare(dq, dq.d)
    cap = max(1024, 2 * counted_hits)
    seg, dptr = C.byref(prep.segments), prep.dptr
    nh = C.c_int64()
    out0 = torch.empty((cap, 5), dtype=torch.int64, device="cuda")

    def one_at_a_time(o, n, on_step=None):
        optr, sh = C.c_void_p(out0.data_ptr()), stream.cuda_stream
        lat = []
        for i in range(n):
            stream.synchronize()
            t0 = time.perf_counter()
            rc = lib.tds_query_batch(qh.handle, seg, dptr, C.byref(o), sh)
            rc = rc or lib.tds_fetch_results(qh.handle, optr, cap, L.TDS_MEM_DEVICE, C.byref(nh))
            stream.synchronize()
            t1 = time.perf_counter()
            L.check(rc)
            assert nh.value == counted_hits, (nh.value, counted_hits)
            lat.append(t1 - t0)
            if on_step:
                on_step(i)
        return np.array(lat)

    pair_ms, stats = [], None

    def keep(i):
        nonlocal stats
        if i >= warmup:
            stats = qh.stats()
            pair_ms.append(stats["ms_pair"])

    lat = one_at_a_time(tds.api.query_opts(timing="pair", **opts), warmup + steps, keep)[warmup:]
    ms = float(lat.mean() * 1e3)
    extra = {}
    if depth > 1:
        timed_ms = ms
        lat = one_at_a_time(tds.api.query_opts(**opts), warmup + steps)[warmup:]
        seq_ms = float(lat.mean() * 1e3)
        o = tds.api.query_opts(**opts)
        hs = [qh] + [tds.Query(ix) for _ in range(depth - 1)]
        sts = [stream] + [torch.cuda.Stream() for _ in range(depth - 1)]
        outs = [out0] + [torch.empty((cap, 5), dtype=torch.int64, device="cuda") for _ in range(depth - 1)]

        def fetch(i):
            k = i % depth
            L.check(lib.tds_fetch_results(hs[k].handle, C.c_void_p(outs[k].data_ptr()), cap,
                                          L.TDS_MEM_DEVICE, C.byref(nh)))
            assert nh.value == counted_hits, (nh.value, counted_hits)

        def run(n):
            for i in range(n):
                k = i % depth
                L.check(lib.tds_query_batch(hs[k].handle, seg, dptr, C.byref(o), sts[k].cuda_stream))
                if i >= depth - 1:
                    fetch(i - depth + 1)
            for i in range(max(0, n - depth + 1), n):
                fetch(i)

        run(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        for h in hs[1:]:
            h.close()
        extra = dict(depth=depth,
                     one_at_a_time=dict(ms_per_step=seq_ms, value=n_ovl / (seq_ms / 1e3)),
                     one_at_a_time_with_pair_events_ms=timed_ms)
    # stage breakdown from a few more steps with every stage timed
    prep_ms, refine_ms = [], []
    for i in range(3):
        qh.batch(prep, None, timing=True, stream=stream, **opts)
        qh.fetch(out="device")
        st = qh.stats()
        prep_ms.append(st["ms_prep"])
        refine_ms.append(st["ms_refine"])
    qh.close()
    return dict(ms_per_step=ms, value=n_ovl / (ms / 1e3), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), pair_ms=float(np.mean(pair_ms)),
                n_hit=int(counted_hits), n_eval=int(stats["n_eval"]), n_overlap=int(counted),
                n_refine=int(stats["n_refine"]), retries=int(stats["retries"]),
                n_items=int(stats["n_items"]), grid=int(stats["grid"]), prep_ms=float(np.median(prep_ms)),
                refine_ms=float(np.median(refine_ms)), opts=opts, **extra)


def cpu_baseline(db, q, target_s=10.0, nthreads=None, seed=12345, label="all the workload's d"):
    """The oracle on a bounded sample of query segments (against all entries).

    The sample doubles until one run takes at least target_s / 4; the rate
    is its overlapping pairs per second of wall time."""
    import oracle
    nthreads = oracle.default_threads() if nthreads is None else int(nthreads)
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(q))
    k = 4
    while True:
        sub = q.subset(np.sort(order[:k]))
        t0 = time.perf_counter()
        h = oracle.search(db, sub, nthreads=nthreads)
        dt = time.perf_counter() - t0
        if dt >= target_s / 4 or k >= len(q):
            break
        k = min(len(q), int(k * max(2.0, target_s / max(dt, 1e-3))))
    return dict(value=h.n_overlap / dt, unit="pair-tests/s", cores=nthreads, kind="oracle",
                sample=f"{k} of {len(q)} query segments (random, {label}) against all "
                       f"{len(db)} entries: {k * len(db):.3g} brute-force pairs, "
                       f"{h.n_overlap} overlapping, {len(h)} hits, {dt:.2f} s wall on {nthreads} threads",
                seconds=dt)


def to_pinned(seg):
    """The query arrays copied into page-locked host memory (numpy views)."""
    import torch

    class Pinned:
        pass

    out = Pinned()
    out.keep = []
    for f in ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1", "d"):
        a = np.asarray(getattr(seg, f), dtype=np.float64)
        t = torch.empty(a.shape, dtype=torch.float64, pin_memory=True)
        t.numpy()[...] = a
        out.keep.append(t)
        setattr(out, f, t.numpy())
    return out


def host_memory_form(ix, q, opts, steps=5, warmup=1):
    """The step with inputs in host memory and the hits returned to host
    memory: query upload and result download over PCIe included. Measured
    twice: with ordinary (pageable) numpy arrays, and with the inputs and
    the result buffer in page-locked memory (as a server's staging buffers
    are), where the uploads run at the link's DMA rate and the record kernel
    writes the hits straight to host memory."""
    import paper_1405_7461_amd as tds

    def timed(src, out):
        qh = tds.Query(ix)
        prep = tds.prepare(src, src.d)
        lat, n_hit = [], 0
        for i in range(warmup + steps):
            t0 = time.perf_counter()
            qh.batch(prep, None, **opts)
            h = qh.fetch(out=out)
            t1 = time.perf_counter()
            if i >= warmup:
                lat.append(t1 - t0)
                n_hit = len(h)
        qh.close()
        return dict(ms_per_step=float(np.mean(lat) * 1e3), n_hit=n_hit,
                    p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3))

    r = timed(q, "host")
    up = len(q) * 9 * 8
    r.update(bytes_in=up, bytes_out=r["n_hit"] * 40)
    r["pinned"] = timed(to_pinned(q), "pinned")
    return r


def trajectory_form(ix, db, dq, q, opts, log_fn=log, steps=10, warmup=2):
    """Trajectory-level answers: the segment hits of a batch merged per
    (query trajectory, entry trajectory) into maximal intervals, on the
    headline batch and on a hit-dense batch (every database trajectory
    shifted by 0.5 along x, d = 5: about one million segment hits)."""
    import torch
    import paper_1405_7461_amd as tds
    stream = torch.cuda.current_stream()
    per_d = len(q) // len(D_VALUES)
    # each (query trajectory, d) is one query: the copy index goes into the high bits
    head_ids = q.traj + (np.repeat(np.arange(len(D_VALUES), dtype=np.int64), per_d) << 32)
    shifted = db.subset(np.arange(len(db))).with_d(5.0)
    shifted.x0 = shifted.x0 + 0.5
    shifted.x1 = shifted.x1 + 0.5
    cases = [("C2 headline batch (120,000 query segments, ids per trajectory and d)", dq, head_ids),
             ("hit-dense: the 2,500 database trajectories shifted by 0.5 in x, d = 5 "
              "(1,000,000 query segments)", to_device(shifted), shifted.traj)]
    import ctypes as C
    from paper_1405_7461_amd import _lib as L
    lib = L.lib()
    out = []
    for label, qdev, ids in cases:
        qh = tds.Query(ix)
        prep = tds.prepare(qdev, qdev.d)
        ids_dev = torch.as_tensor(ids, device="cuda")
        # sizes from one untimed pass; then, as a C caller with a buffer of
        # that size, one call merges and copies the records
        qh.batch(prep, None, stream=stream, **opts)
        n_hit = len(qh.fetch(out="device"))
        n_out = len(qh.fetch_trajectories(ids_dev, out="device"))
        rec = torch.empty((max(n_out, 1), 4), dtype=torch.int64, device="cuda")
        nn = C.c_int64()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        wall, gpu, seg_ms = [], [], []
        for i in range(warmup + steps):
            stream.synchronize()
            t0 = time.perf_counter()
            qh.batch(prep, None, stream=stream, **opts)
            h = qh.fetch(out="device")
            stream.synchronize()
            t1 = time.perf_counter()
            ev0.record(stream)
            L.check(lib.tds_fetch_trajectories(qh.handle, C.c_void_p(ids_dev.data_ptr()), L.TDS_MEM_DEVICE,
                                               C.c_void_p(rec.data_ptr()), rec.shape[0], L.TDS_MEM_DEVICE,
                                               C.byref(nn)))
            ev1.record(stream)
            stream.synchronize()
            t2 = time.perf_counter()
            if i >= warmup:
                seg_ms.append((t1 - t0) * 1e3)
                wall.append((t2 - t1) * 1e3)
                gpu.append(ev0.elapsed_time(ev1))
        assert len(h) == n_hit and nn.value == n_out
        st = qh.stats()
        qh.close()
        merge_ms = float(np.mean(gpu))
        # algorithmic bytes: per segment hit its 24-B record, two 8-B trajectory
        # ids and the 4-B query permutation; per merged interval a 32-B record
        alg = 44 * n_hit + 32 * n_out
        r = dict(workload=label, n_segment_hits=n_hit, n_intervals=n_out,
                 step_ms_segments=float(np.mean(seg_ms)), merge_ms_gpu=merge_ms,
                 merge_ms_wall=float(np.mean(wall)), retries=int(st["retries"]),
                 segment_hits_per_s=n_hit / (merge_ms / 1e3),
                 roofline=dict(bound="hbm", achieved=alg / (merge_ms / 1e3) / 1e9, peak=8000.0,
                               unit="GB/s", frac=alg / (merge_ms / 1e3) / 8e12,
                               per_unit="44 B per segment hit + 32 B per merged interval"))
        log_fn(f"trajectories [{label[:24]}]: {n_hit} segment hits -> {n_out} intervals, merge "
               f"{merge_ms:.3f} ms GPU / {r['merge_ms_wall']:.3f} ms wall, segment step "
               f"{r['step_ms_segments']:.3f} ms, retries {r['retries']}")
        out.append(r)
    return out


def _tiling_summary(trials):
    """Fastest trial of each tiling (Periodic and GreedySetSplit over their sizes)."""
    best = {}
    for t in trials:
        k = t.opts["tiling"]
        if k not in best or t.ms < best[k].ms:
            best[k] = t
    return {k: dict(ms_per_step=round(t.ms, 4), pair_ms=round(t.pair_ms, 4), prep_ms=round(t.prep_ms, 4),
                    n_eval=int(t.n_eval), n_tiles=int(t.n_tiles), num_bins=t.num_bins,
                    batch_size=t.opts.get("batch_size"), block_size=t.opts["block_size"])
            for k, t in best.items()}


def batching_form(log_fn=log, reps=10):
    """C4: uneven query set, per-query d, one persistent launch, autotuned over
    the tilings (range buckets, Periodic, GreedySetSplit-Min/-Max of Alg. 4)."""
    import torch
    import gen
    import paper_1405_7461_amd as tds
    from paper_1405_7461_amd.autotune import tune
    db = gen.make_db("C4")
    q = gen.make_queries("C4")
    n_ovl = overlap_count(db, q)
    dq = to_device(q)
    t0 = time.perf_counter()
    res = tune(db, dq, dq.d, mode="fp32_refine", num_bins=(400, 1000, 2000),
               tilings=("range", "periodic", "greedy_min", "greedy_max"), batch_sizes=(64, 256, 1024),
               blocks=(256, 1024), reps=2, use_cache=False, cache=None)
    tune_s = time.perf_counter() - t0
    ix = tds.build_index(db, res.num_bins)
    r = run_form(ix, dq, res.opts, reps, 2, n_ovl)
    ix.close()
    out = dict(workload="C4: 1M-segment exponential-step walk (2,500 x 400); 256 query trajectories of "
                        "log-uniform length 10-2000 (segments of 1/8), per-trajectory d in {1,5,25}",
               n_query_segments=len(q), n_overlap=n_ovl, tuned=dict(num_bins=res.num_bins, **res.opts),
               tune_s=round(tune_s, 2), trials=len(res.trials), value=r["value"], unit="pair-tests/s",
               ms_per_step=r["ms_per_step"], pair_ms=r["pair_ms"], n_hit=r["n_hit"], n_eval=r["n_eval"],
               best_per_tiling=_tiling_summary(res.trials))
    log_fn(f"batching (C4): {out['value']:.4g} pair-tests/s, {out['ms_per_step']:.3f} ms/step, tuned {out['tuned']}")
    for k, v in out["best_per_tiling"].items():
        log_fn(f"  best {k}: {v}")
    return out


def tiling_comparison(ix, dq, n_ovl, log_fn=log, steps=10, warmup=2):
    """The headline batch under each tiling at one launch shape."""
    out = {}
    for name, extra in (("range", {}), ("periodic", dict(batch_size=128)),
                        ("greedy_min", dict(batch_size=256)), ("greedy_max", dict(batch_size=1024))):
        opts = dict(mode="fp32_refine", tiling=name, block_size=256, **extra)
        r = run_form(ix, dq, opts, steps, warmup, n_ovl)
        out[name] = dict(batch_size=extra.get("batch_size"), ms_per_step=round(r["ms_per_step"], 4),
                         pair_ms=round(r["pair_ms"], 4), prep_ms=round(r["prep_ms"], 4),
                         n_eval=r["n_eval"], n_hit=r["n_hit"], value=r["value"])
        log_fn(f"tiling {name}: {out[name]}")
    hits = {v["n_hit"] for v in out.values()}
    assert len(hits) == 1, out
    return out


def model_form(log_fn=log, steps=8, warmup=2):
    """Sec. 8's response-time model re-fitted here: calibration, alpha per
    epoch from a representative query set, predicted against measured times
    for the headline batch and for Periodic batch sizes (the paper's Table 3:
    the model's choice of s against the measured best)."""
    import gen
    from gen import workloads as W
    import paper_1405_7461_amd as tds
    from paper_1405_7461_amd import perfmodel as M
    t0 = time.perf_counter()
    model = M.calibrate(qs=(64, 1024, 16384, 131072), cs=(256, 1024, 4096, 16384, 65536), reps=3,
                        max_hits=1 << 24)
    cal_s = time.perf_counter() - t0
    out = dict(calibration_s=round(cal_s, 2), cpu_fit=dict(model.cpu.__dict__), scenarios={})
    sizes = (32, 64, 128, 256, 512, 1024)
    for name in ("C2", "C4"):
        db = gen.make_db(name)
        if name == "C2":
            q = gen.concat([gen.make_queries("C2").with_d(d) for d in D_VALUES])
            rep0 = W.gaussian_walk(W.rng_for(2, 7), 20, 400, 1000.0, 1.0)
            rep = gen.concat([rep0.with_d(d) for d in D_VALUES])
        else:
            q = gen.make_queries("C4")
            rng = W.rng_for(4, 7)
            rep = W.short_queries(rng, 64, 10, 2000, 1.0 / 8, 1.0 / 64, 400.0, 1000.0, "exp", 1.0 / 8)
            rep = rep.with_d(W.rng_for(4, 8).choice(np.asarray(D_VALUES), size=64)[rep.traj])
        n_ovl = overlap_count(db, q)
        ix = tds.build_index(db, NUM_BINS)
        est = M.estimate_alpha(model, ix, rep, num_epochs=50, s=256)
        dq = to_device(q)
        rows = []
        for tiling, s in [("range", 0)] + [("periodic", s) for s in sizes]:
            opts = dict(mode="fp32_refine", tiling=tiling, block_size=256)
            if s:
                opts["batch_size"] = s
            r = run_form(ix, dq, opts, steps, warmup, n_ovl)
            p = model.predict(ix, q, tiling=tiling, batch_size=s or 128)
            rows.append(dict(tiling=tiling, s=s or None, measured_ms=round(r["ms_per_step"], 4),
                             predicted_ms=round(p["ms"], 4),
                             rel_error=round(p["ms"] / r["ms_per_step"] - 1, 3),
                             interactions_model=p["interactions"], interactions_device=r["n_eval"],
                             alpha=p["alpha"], beta=p["beta"]))
        ix.close()
        per = [x for x in rows if x["tiling"] == "periodic"]
        chosen = min(per, key=lambda x: x["predicted_ms"])
        best = min(per, key=lambda x: x["measured_ms"])
        out["scenarios"][name] = dict(
            alpha_estimate=est, rows=rows, model_s=chosen["s"], actual_s=best["s"],
            slowdown=round(chosen["measured_ms"] / best["measured_ms"] - 1, 4),
            mean_abs_rel_error=round(float(np.mean([abs(x["rel_error"]) for x in rows])), 3))
        log_fn(f"model {name}: alpha {est}, model s {chosen['s']}, actual s {best['s']}, slowdown "
               f"{out['scenarios'][name]['slowdown']:.2%}, mean |error| "
               f"{out['scenarios'][name]['mean_abs_rel_error']:.1%}")
        for x in rows:
            log_fn(f"  {x}")
    return out


def serving_form(log_fn=log, n_requests=6000, rates=(0.5, 0.8, 0.95), streams=4, max_batch=16384):
    """C5: 10M-segment resident index; requests served by the library's
    native scheduler (tds_server_*: admission by estimated result bytes,
    continuous batching over `streams` HIP streams, per-request split in
    native code). Open-loop load: each request is submitted with its arrival
    time (all at 0 for the saturation run, Poisson at 3 fractions of the
    saturation rate otherwise); latency = done - arrival on the server's
    clock. The request arrays are generated once and reused by every run."""
    import gen
    import paper_1405_7461_amd as tds
    from paper_1405_7461_amd.serving import poisson_arrivals
    t0 = time.perf_counter()
    db = gen.make_db("C5")
    ix = tds.build_index(db, gen.CONFIGS["C5"]["bins"])
    t1s, t0s = np.sort(db.t1), np.sort(db.t0)
    del db
    build_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    reqs = [gen.make_queries("C5", request=i) for i in range(n_requests)]
    n_ovl = np.array([int((np.searchsorted(t0s, q.t1, side="left")
                           - np.searchsorted(t1s, q.t0, side="right")).sum()) for q in reqs])
    n_seg = np.array([len(q) for q in reqs])
    gen_s = time.perf_counter() - t0
    log_fn(f"serving: index {build_s:.1f} s, {n_requests} requests ({n_seg.sum()} segments, "
           f"{n_ovl.sum():.4g} overlapping pairs) generated in {gen_s:.1f} s")

    def serve(arrivals, warm=False):
        srv = tds.NativeServer(ix, streams=streams, max_batch_segments=max_batch,
                               mode="fp32_refine", tiling="range")
        if warm:  # first batches of a fresh server: untimed
            ids = [srv.submit(q, q.d, 0.0) for q in reqs[:256]]
            for i in ids:
                srv.wait(i)
        # every request is submitted before the first one arrives, so the
        # Python submission loop never paces the load
        base = srv.now() + 1.5
        ids = [srv.submit(q, q.d, base + float(a)) for q, a in zip(reqs, arrivals)]
        assert srv.now() < base, "submission took longer than the lead time"
        infos = [srv.wait(i) for i in ids]
        st = srv.stats()
        srv.close()
        assert all(x["status"] == 0 for x in infos)
        arr = np.array([x["arrival"] for x in infos])
        done = np.array([x["done"] for x in infos])
        adm = np.array([x["admit"] for x in infos])
        lat = done - arr
        wall = done.max() - arr.min()
        return dict(wall_s=wall, p50_ms=float(np.percentile(lat, 50) * 1e3),
                    p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                    p99_wait_ms=float(np.percentile(adm - arr, 99) * 1e3),
                    p99_service_ms=float(np.percentile(done - adm, 99) * 1e3),
                    batches=int(st["batches"]), retries=int(st["retries"]),
                    mean_batch_requests=float(np.mean([x["n_batch_requests"] for x in infos])),
                    hits=int(sum(x["n_hit"] for x in infos)), busy_s=float(st["busy_s"]),
                    stage_s=float(st["stage_s"]), wait_s=float(st["wait_s"]),
                    split_s=float(st["split_s"]), device_bytes=int(st["device_bytes"]))

    sat = serve(np.zeros(n_requests), warm=True)
    sat_rate = n_requests / sat["wall_s"]
    log_fn(f"serving saturation: {sat_rate:.0f} req/s, {n_ovl.sum() / sat['wall_s']:.4g} pair-tests/s, "
           f"{sat['batches']} batches, p50 {sat['p50_ms']:.2f} ms")
    runs = []
    for k, f in enumerate(rates):
        arr = poisson_arrivals(n_requests, f * sat_rate, seed=14057461 + 500 + k)
        st = serve(arr)
        runs.append(dict(rate_frac=f, rate_req_s=f * sat_rate, p50_ms=st["p50_ms"], p99_ms=st["p99_ms"],
                         p99_wait_ms=st["p99_wait_ms"], p99_service_ms=st["p99_service_ms"],
                         retries=st["retries"], pair_tests_s=float(n_ovl.sum() / st["wall_s"]),
                         mean_batch_requests=st["mean_batch_requests"], batches=st["batches"]))
        log_fn(f"serving at {f:.2f} x saturation ({f * sat_rate:.0f} req/s): p50 {st['p50_ms']:.3f} ms, "
               f"p99 {st['p99_ms']:.3f} ms, {runs[-1]['pair_tests_s']:.4g} pair-tests/s")
    # the kernel's own throughput on one batch of the same requests, inputs
    # and outputs in device memory
    big = gen.concat(reqs[:80])
    dq = to_device(big)
    n_big = int(n_ovl[:80].sum())
    kb = run_form(ix, dq, dict(mode="fp32_refine", tiling="range", block_size=256), 10, 2, n_big)
    ix.close()
    log_fn(f"serving: one batch of 80 requests ({len(big)} segments) device-resident: "
           f"{kb['ms_per_step']:.3f} ms, {kb['value']:.4g} pair-tests/s")
    return dict(workload="C5: 10M-segment Gaussian walk (25,000 x 400) resident; requests of log-uniform "
                         "length 10-5000 (segments of 1/16), d log-uniform in [0.5, 50]; Poisson arrivals",
                engine="native scheduler (tds_server_*), fp32_refine, range tiles",
                streams=streams, max_batch_segments=max_batch, n_requests=n_requests,
                build_s=round(build_s, 2),
                saturation_req_s=sat_rate, saturation_pair_tests_s=float(n_ovl.sum() / sat["wall_s"]),
                saturation_p50_ms=sat["p50_ms"], saturation_batches=sat["batches"],
                saturation_busy_s=sat["busy_s"],
                saturation_busy_parts_s=dict(stage=sat["stage_s"], wait=sat["wait_s"], split=sat["split_s"]),
                device_bytes=sat["device_bytes"],
                kernel_batch=dict(requests=80, segments=len(big), ms_per_step=kb["ms_per_step"],
                                  pair_tests_s=kb["value"]),
                rates=runs)


def copy_probe(mib: int):
    """A plain copy kernel of known size: reads and writes MIB MiB each."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    log(f"copy probe: {mib} MiB read + {mib} MiB written per launch, 3 launches")


def valu_probe(log_fn=log):
    """Issue rates of the vector instructions the pair kernels are built from,
    measured on this GPU with the probe library (dependence chains of one
    instruction kind on every SIMD, 8 waves per SIMD), with the shader clock
    under load from per-wave clock stamps."""
    import ctypes
    import torch
    from paper_1405_7461_amd.build import PROBE_LIB
    lib = ctypes.CDLL(str(PROBE_LIB))
    lib.tds_probe_valu.restype = ctypes.c_int
    lib.tds_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p] + \
        [ctypes.POINTER(ctypes.c_double)] * 3
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    simds = 4 * cus
    blocks = cus * 8          # 256-thread blocks: 8 waves per SIMD
    stream = torch.cuda.current_stream().cuda_stream
    out = {"simds": simds, "waves_per_simd": 8}
    names = ("v_sub_f32", "v_max3_f32_abs", "v_min3_f32", "v_fma_f64", "v_add_u32", "v_pk_sub_u16",
             "v_pk_max_u16", "v_max_f32_e64_abs", "v_pk_add_f16", "v_min_f32", "v_cmp_le_f32",
             "v_fma_f32", "v_fmac_f32", "v_mul_f32", "v_add_f32", "v_or_b32", "v_or3_b32", "v_max_f32",
             "v_sub_f32_e64_abs", "v_fma_f32_sgpr", "v_fmac_f32_sgpr", "v_fma_f32_3banks",
             "v_fma_f32_same_bank", "v_mfma_f32_16x16x4_f32", "v_mfma_f32_32x32x2_f32")
    for kind, name in enumerate(names):
        best = None
        for _ in range(3):
            ms, wi, hz = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            rc = lib.tds_probe_valu(kind, blocks, 20000, ctypes.c_void_p(stream), ctypes.byref(ms),
                                    ctypes.byref(wi), ctypes.byref(hz))
            assert rc == 0, (name, rc)
            if best is None or ms.value < best[0]:
                best = (ms.value, wi.value, hz.value)
        ms, wi, hz = best
        rate = wi / (ms / 1e3)                       # wave instructions per second
        cyc = simds * hz / rate                      # cycles per wave instruction per SIMD
        out[name] = dict(ms=round(ms, 4), wave_instr=wi, clock_ghz=round(hz / 1e9, 3),
                         cycles_per_wave_instr=round(cyc, 3), lane_ops_per_s=rate * 64,
                         lane_ops_per_s_at_2_4ghz=64 * simds * 2.4e9 / cyc)
        log_fn(f"probe {name}: {cyc:.2f} cycles per wave64 instruction per SIMD at "
               f"{hz / 1e9:.2f} GHz ({rate * 64:.4g} lane ops/s)")
    return out


def roofline_of(name, r, n_ovl):
    """Roofline of a form's pair kernel from its HIP-event launch time."""
    if name == "fp32_refine":
        ach = FILTER_FLOPS_PER_PAIR * r["n_eval"] / (r["pair_ms"] / 1e3)
        return dict(bound="alu", achieved=ach / 1e12, peak=FP32_PEAK / 1e12, unit="TFLOP/s",
                    frac=ach / FP32_PEAK, kernel="k_pair<fp32_refine>",
                    per_unit=f"{FILTER_FLOPS_PER_PAIR} binary32 flops per candidate pair (three "
                             "multiply-adds, FMA = 2, and the threshold comparison)",
                    units_per_launch=r["n_eval"], launch_ms=r["pair_ms"])
    ach = FP64_FLOPS_PER_PAIR * n_ovl / (r["pair_ms"] / 1e3)
    return dict(bound="alu", achieved=ach / 1e12, peak=FP64_PEAK / 1e12, unit="TFLOP/s",
                frac=ach / FP64_PEAK, kernel="k_pair<fp64>",
                per_unit=f"{FP64_FLOPS_PER_PAIR} binary64 flops per overlapping pair",
                units_per_launch=n_ovl, launch_ms=r["pair_ms"])


def time_forms(ix, dq, n_ovl, names, steps, warmup, tag):
    forms = {
        "fp32_refine": dict(mode="fp32_refine", tiling="range", block_size=256),
        "fp64": dict(mode="fp64", tiling="range", block_size=256),
    }
    results = {}
    for name in names:
        r = run_form(ix, dq, forms[name], steps, warmup, n_ovl, depth=PIPE_DEPTH)
        assert r["n_overlap"] == n_ovl, (r["n_overlap"], n_ovl)
        r["roofline"] = roofline_of(name, r, n_ovl)
        results[name] = r
        log(f"{tag} {name}: {r['ms_per_step']:.3f} ms/step with {r.get('depth', 1)} batches in flight "
            f"({r['one_at_a_time']['ms_per_step']:.3f} one at a time), {r['value']:.4g} pair-tests/s, "
            f"p50/p99 {r['p50_ms']:.3f}/{r['p99_ms']:.3f} ms, pair kernel "
            f"{r['pair_ms']:.3f} ms ({r['roofline']['frac']:.3f} of its roof), hits {r['n_hit']}, "
            f"N_eval {r['n_eval']}, refined {r['n_refine']}, retries {r['retries']}")
    if "fp32_refine" in results and "fp64" in results:
        assert results["fp32_refine"]["n_hit"] == results["fp64"]["n_hit"]
    return results, forms


def _strip(results):
    return {k: {kk: vv for kk, vv in v.items() if kk != "opts"} for k, v in results.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp32_refine,fp64")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline workload's forms (for profiler runs)")
    ap.add_argument("--workload", default="C3", choices=("C3", "C2"),
                    help="workload of the headline forms: the precision form (default) or, for "
                         "profiling, the at-scale plain workload")
    ap.add_argument("--no-plain", action="store_true", help="skip the at-scale plain workload")
    ap.add_argument("--no-host", action="store_true", help="skip the host-memory (PCIe) steps")
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-trajectories", action="store_true")
    ap.add_argument("--no-model", action="store_true",
                    help="skip the response-time model (calibration and predictions)")
    ap.add_argument("--no-tilings", action="store_true",
                    help="skip the at-scale plain batch under the other tilings")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the vector-ALU issue-rate probes")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the forms, run a plain device copy of MIB MiB three times "
                         "(calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library does not "
              "shard a search across GPUs", file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_plain = args.no_host = args.no_batching = args.no_serving = True
        args.no_trajectories = args.no_model = args.no_tilings = args.no_cpu_baseline = True
        args.no_probe = True

    import torch
    import paper_1405_7461_amd as tds
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    # ------------------------------------------------ headline: precision form
    t0 = time.perf_counter()
    db, q, m = make_workload(args.workload)
    n_ovl = overlap_count(db, q)
    log(f"headline workload: {len(db)} entries, {len(q)} query segments, N_ovl={n_ovl} "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    t0 = time.perf_counter()
    ix = tds.build_index(db, m)
    log(f"index built in {time.perf_counter() - t0:.2f} s: {ix.info()}")
    dq = to_device(q)
    torch.cuda.synchronize()
    results, forms = time_forms(ix, dq, n_ovl, args.forms.split(","), args.steps, args.warmup, args.workload)
    if args.copy_probe:
        copy_probe(args.copy_probe)
    head_name = "fp32_refine" if "fp32_refine" in results else list(results)[0]
    head = results[head_name]
    roof = dict(head["roofline"])
    roof["traffic"] = measured_traffic(f"k_pair_{'fp32' if head_name == 'fp32_refine' else 'fp64'}_"
                                       f"{args.workload.lower()}_hbm.txt")
    roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)"
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "pair-tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_name == "fp32_refine" else "f64",
        "data": "synthetic",
        "config": {"workload": HEAD_WORKLOAD if args.workload == "C3" else PLAIN_WORKLOAD, "form": head_name,
                   "n_overlap_per_step": n_ovl, "batches_in_flight": head.get("depth", 1),
                   **{k: v for k, v in head["opts"].items()}},
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"],
                       "of": "one batch alone: tds_query_batch + tds_fetch_results into device memory"},
        "roofline": roof,
        "forms": _strip(results),
    }
    if "fp32_refine" in results and "fp64" in results:
        line["fp32_refine_vs_fp64"] = results["fp32_refine"]["value"] / results["fp64"]["value"]
    if not args.no_host:
        hm = host_memory_form(ix, q, forms[head_name])
        hm["value"] = n_ovl / (hm["ms_per_step"] / 1e3)
        hm["pinned"]["value"] = n_ovl / (hm["pinned"]["ms_per_step"] / 1e3)
        assert hm["n_hit"] == hm["pinned"]["n_hit"] == results[head_name]["n_hit"]
        line["host_memory"] = hm
        log(f"C3 {head_name} with host inputs and outputs: {hm['ms_per_step']:.3f} ms/step, "
            f"{hm['value']:.4g} pair-tests/s; page-locked: {hm['pinned']['ms_per_step']:.3f} ms/step, "
            f"{hm['pinned']['value']:.4g} pair-tests/s")
    if not args.no_probe:
        line["valu_probe"] = valu_probe()
    if not args.no_cpu_baseline:
        cb = cpu_baseline(db, q, target_s=10.0, label="both d")
        cb["one_core"] = cpu_baseline(db, q, target_s=6.0, nthreads=1, seed=54321, label="both d")
        line["cpu_baseline"] = cb
        log(f"oracle: {cb['value']:.4g} pair-tests/s on {cb['cores']} threads, "
            f"{cb['one_core']['value']:.4g} on 1")
    ix.close()
    del db, q, dq

    # ------------------------------------------------ at-scale plain workload
    if not args.no_plain:
        db2, q2, m2 = make_workload("C2")
        n2 = overlap_count(db2, q2)
        ix2 = tds.build_index(db2, m2)
        dq2 = to_device(q2)
        r2, forms2 = time_forms(ix2, dq2, n2, ["fp32_refine", "fp64"], args.steps, args.warmup, "C2")
        line["plain"] = dict(workload=PLAIN_WORKLOAD,
                             n_overlap_per_step=n2, forms=_strip(r2))
        if not args.no_tilings:
            line["tilings"] = tiling_comparison(ix2, dq2, n2)
        if not args.no_trajectories:
            line["trajectories"] = trajectory_form(ix2, db2, dq2, q2, forms2["fp32_refine"])
        ix2.close()
    if not args.no_batching:
        line["batching"] = batching_form()
    if not args.no_model:
        line["model"] = model_form()
    if not args.no_serving:
        line["serving"] = serving_form()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
