"""Issue-rate probe library (libtds_probe.so): the benchmark's measured
instruction rates come from it.

CPU: its entry point rejects bad arguments before any HIP call.
GPU: every probe kind runs and reports a plausible rate and clock.
"""
import ctypes

import pytest

from paper_1405_7461_amd.build import PROBE_LIB

N_KINDS = 25  # kinds 0 .. 24


def _lib():
    if not PROBE_LIB.exists():
        pytest.skip("probe library not built")
    lib = ctypes.CDLL(str(PROBE_LIB))
    lib.tds_probe_valu.restype = ctypes.c_int
    lib.tds_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p] + \
        [ctypes.POINTER(ctypes.c_double)] * 3
    return lib


def _call(lib, kind, blocks=1, iters=1, null=False):
    ms, wi, hz = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    if null:
        return lib.tds_probe_valu(kind, blocks, iters, None, None, ctypes.byref(wi), ctypes.byref(hz)), 0, 0, 0
    rc = lib.tds_probe_valu(kind, blocks, iters, None, ctypes.byref(ms), ctypes.byref(wi), ctypes.byref(hz))
    return rc, ms.value, wi.value, hz.value


def test_probe_rejects_bad_arguments():
    lib = _lib()
    assert _call(lib, -1)[0] == -1
    assert _call(lib, N_KINDS)[0] == -1
    assert _call(lib, 0, blocks=0)[0] == -1
    assert _call(lib, 0, iters=0)[0] == -1
    assert _call(lib, 0, null=True)[0] == -1


def test_bench_names_every_kind():
    import bench
    import inspect
    src = inspect.getsource(bench.valu_probe)
    names = src[src.index("names = ("):src.index(")", src.index("names = ("))]
    assert names.count('"') == 2 * N_KINDS


@pytest.mark.gpu
def test_every_kind_runs():
    import torch
    torch.cuda.init()
    lib = _lib()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for kind in range(N_KINDS):
        rc, ms, wi, hz = _call(lib, kind, blocks=cus, iters=200)
        print(f"probe kind {kind}: rc {rc}, {ms:.4f} ms, {wi:.4g} wave instructions, {hz / 1e9:.2f} GHz",
              flush=True)
        assert rc == 0, kind
        assert ms > 0.0 and wi == cus * 4 * 200 * 8, kind
        assert 0.5e9 < hz < 3.5e9, kind
