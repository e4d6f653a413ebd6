"""C ABI: symbols, and the host-side index logic pinned to the paper's Figs. 1-2.

CPU only: nothing here launches a kernel.
"""
import re
from pathlib import Path

import numpy as np
import pytest

import paper_1405_7461_amd as tds
from paper_1405_7461_amd import _lib as L
from golden_io import fig1, fig2

HEADER = Path(__file__).resolve().parents[1] / "include" / "tds.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tds_\w+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"{name} not bound in _lib.SIGNATURES"


def test_abi_version():
    assert L.lib().tds_abi_version() == 1


def test_struct_sizes_match_header():
    # tds_hit is five 8-byte fields; tds_bin five; tds_segments 16 + 9 pointers
    import ctypes as C
    assert C.sizeof(L.tds_hit) == 40
    assert C.sizeof(L.tds_bin) == 40
    assert C.sizeof(L.tds_segments) == 16 + 9 * 8
    assert C.sizeof(L.tds_query_opts) == 6 * 4 + 8 + 2 * 4
    assert C.sizeof(L.tds_traj_hit) == 32


def test_fig1_bin_table():
    t0, t1, bins, _ = fig1()
    got = tds.plan_bins(t0, t1, 4)
    assert len(got) == 4
    for g, (j, start, end, first, last) in zip(got, bins):
        assert (g["bin"], g["start"], g["end"], g["first"], g["last"]) == (j, start, end, first, last)
    # bin counts 6/3/3/3
    assert list(got["last"] - got["first"] + 1) == [6, 3, 3, 3]


def test_lookup_example():
    t0, t1, _, lk = fig1()
    bins = tds.plan_bins(t0, t1, 4)
    f, l = tds.plan_ranges(bins, [lk["t0"]], [lk["t1"]])
    assert (f[0], l[0]) == (lk["first"], lk["last"])
    cand = np.arange(f[0], l[0] + 1)
    ovl = cand[(t0[cand] < lk["t1"]) & (t1[cand] > lk["t0"])]
    assert list(ovl) == lk["overlap"]


def test_fig2_interaction_totals():
    t0, t1, _, _ = fig1()
    bins = tds.plan_bins(t0, t1, 4)
    batches, totals = fig2()
    for s, (want, printed) in totals.items():
        k = s // 10
        total = 0
        for g in range(0, len(batches), k):
            grp = batches[g:g + k]
            a = min(b[1] for b in grp)
            b_ = max(b[2] for b in grp)
            f, l = tds.plan_ranges(bins, [a], [b_])
            total += sum(b[0] for b in grp) * (l[0] - f[0] + 1)
        assert total == want, (s, total)
    # only the single-batch total is reading-independent
    assert totals[60][0] == totals[60][1]


def test_ranges_superset_of_overlaps():
    rng = np.random.default_rng(7)
    n = 3000
    t0 = np.sort(rng.uniform(0, 50, n))
    t1 = t0 + rng.exponential(2.0, n) + 1e-3
    qa = rng.uniform(-5, 55, 400)
    qb = qa + rng.exponential(1.0, 400) + 1e-3
    for m in (1, 7, 100, 5000):
        bins = tds.plan_bins(t0, t1, m)
        assert bins["last"][-1] == n - 1 and bins["first"][0] == 0
        f, l = tds.plan_ranges(bins, qa, qb)
        for i in range(qa.size):
            ov = np.nonzero((t0 < qb[i]) & (t1 > qa[i]))[0]
            if ov.size:
                assert f[i] <= ov.min() and ov.max() <= l[i]
        if m == 1:
            nonempty = l >= f
            assert np.all(f[nonempty] == 0) and np.all(l[nonempty] == n - 1)


def test_plan_bins_rejects_bad_input():
    with pytest.raises(tds.TdsError):
        tds.plan_bins([0.0, 2.0, 1.0], [1.0, 3.0, 2.0], 2)  # not sorted
    with pytest.raises(tds.TdsError):
        tds.plan_bins([0.0, 1.0], [1.0, 1.0], 2)  # empty span
    with pytest.raises(tds.TdsError):
        tds.plan_bins([0.0], [1.0], 0)
    with pytest.raises(tds.TdsError):
        tds.plan_bins([np.nan], [1.0], 3)


def test_build_index_validates_before_the_device():
    from gen import fixtures as fx
    db, _ = fx.random_small()
    bad = db.subset(np.arange(len(db)))
    bad.t1[5] = bad.t0[5] - 1.0
    with pytest.raises(tds.TdsError) as e:
        tds.build_index(bad, 10)
    assert e.value.code == L.TDS_EINVAL
    with pytest.raises(tds.TdsError) as e:
        tds.build_index(db, 0)
    assert e.value.code == L.TDS_EINVAL
    bad2 = db.subset(np.arange(len(db)))
    bad2.y1[2] = np.inf
    with pytest.raises(tds.TdsError) as e:
        tds.build_index(bad2, 10)
    assert e.value.code == L.TDS_EINVAL


def test_set_allocator_arguments():
    lib = L.lib()
    assert lib.tds_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None) == L.TDS_OK
    rc = lib.tds_set_allocator(L.ALLOC_FN(lambda n, s, c: None), L.FREE_FN(), None)
    assert rc == L.TDS_EINVAL and b"both" in lib.tds_last_error()
    rc = lib.tds_set_allocator(L.ALLOC_FN(), L.FREE_FN(lambda p, s, c: None), None)
    assert rc == L.TDS_EINVAL
    assert lib.tds_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None) == L.TDS_OK


def test_fetch_trajectories_arguments():
    import ctypes as C
    lib = L.lib()
    n = C.c_int64(-1)
    assert lib.tds_fetch_trajectories(None, None, L.TDS_MEM_HOST, None, 0, L.TDS_MEM_HOST,
                                      C.byref(n)) == L.TDS_EINVAL
    assert b"tds_fetch_trajectories" in lib.tds_last_error()


def test_query_tiles_arguments():
    import ctypes as C
    lib = L.lib()
    assert C.sizeof(L.tds_tile_info) == 16
    a, b = C.c_int64(), C.c_int64()
    assert lib.tds_query_tiles(None, None, 0, None, 0, C.byref(a), C.byref(b)) == L.TDS_EINVAL
    assert b"tds_query_tiles" in lib.tds_last_error()


def test_index_times_arguments():
    import ctypes as C
    lib = L.lib()
    assert lib.tds_index_times(None, None, None, 0) == L.TDS_EINVAL
    assert b"tds_index_times" in lib.tds_last_error()


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_plan_ranges_equal_oracle(seed):
    """The library's candidate ranges equal the oracle's Sec. 4 ranges (the
    bins that overlap the interval, scanned one by one) on entries of very
    uneven durations, where the last bin starting before an interval's end
    often ends before its start."""
    from oracle import batching as ob
    rng = np.random.default_rng(seed)
    n = 2000
    t0 = np.sort(np.round(rng.uniform(0, 100, n), 2))
    t1 = t0 + np.where(rng.uniform(size=n) < 0.05, rng.exponential(20.0, n), rng.exponential(0.3, n)) + 0.01
    qa = rng.uniform(-5, 105, 3000)
    qb = qa + rng.exponential(0.5, 3000) + 1e-3
    differs = 0
    for m in (1, 9, 64, 500):
        bins = tds.plan_bins(t0, t1, m)
        obins = ob.bin_table(t0, t1, m)
        f, l = tds.plan_ranges(bins, qa, qb)
        for i in range(qa.size):
            r = ob.candidate_range(obins, qa[i], qb[i])
            assert (f[i], l[i]) == ((0, -1) if r is None else r), (m, i)
            # the superset end (last bin starting before the interval's end)
            j2 = np.searchsorted(bins["start"], qb[i], side="left") - 1
            differs += int(r is not None and bins["last"][j2] != r[1])
    assert differs > 0  # the case where the two readings part is exercised


def test_server_and_reserve_arguments():
    # the serving and reservation entry points reject bad arguments before any
    # device work
    import ctypes as C
    lib = L.lib()
    assert C.sizeof(L.tds_server_opts) == 48 + C.sizeof(L.tds_query_opts)
    assert C.sizeof(L.tds_request_info) == 48
    assert C.sizeof(L.tds_server_stats) == 72
    opts = L.tds_query_opts(L.TDS_MODE_FP64, L.TDS_TILE_RANGE, 0, 0, 0, -1, 0, 0, 0)
    assert lib.tds_query_reserve(None, 10, 10, C.byref(opts)) == L.TDS_EINVAL
    assert b"tds_query_reserve" in lib.tds_last_error()
    n = C.c_int64()
    assert lib.tds_query_device_bytes(None, C.byref(n)) == L.TDS_EINVAL
    so = L.tds_server_opts()
    h = C.c_void_p()
    assert lib.tds_server_create(None, C.byref(so), C.byref(h)) == L.TDS_EINVAL
    assert b"tds_server_create" in lib.tds_last_error()
    rid = C.c_int64()
    assert lib.tds_server_submit(None, None, None, 0.0, C.byref(rid)) == L.TDS_EINVAL
    assert lib.tds_server_wait(None, 0, 0.0, C.byref(L.tds_request_info())) == L.TDS_EINVAL
    assert lib.tds_server_results(None, 0, None, 0, C.byref(n)) == L.TDS_EINVAL
    assert lib.tds_server_release(None, 0) == L.TDS_EINVAL
    assert lib.tds_server_stats_get(None, C.byref(L.tds_server_stats())) == L.TDS_EINVAL
    m = C.c_int32()
    assert lib.tds_server_alpha(None, None, 0, C.byref(m)) == L.TDS_EINVAL
    assert lib.tds_server_now(None) == 0.0
    lib.tds_server_destroy(None)  # a null server is ignored
