"""Python binding of the C ABI: build_index / query_batch / fetch_results.

Argument marshalling only. Inputs are numpy arrays (host memory) or torch
float64 tensors on the GPU (device memory); every step of the search runs in
the library's HIP kernels. torch is used for device buffers and streams.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _lib as L

FIELDS = ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1")
MODES = {"fp64": L.TDS_MODE_FP64, "fp32_refine": L.TDS_MODE_FP32_REFINE}
TILINGS = {"periodic": L.TDS_TILE_PERIODIC, "range": L.TDS_TILE_RANGE,
           "greedy_min": L.TDS_TILE_GREEDY_MIN, "greedy_max": L.TDS_TILE_GREEDY_MAX}


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return torch.cuda.current_stream().cuda_stream or None
        return None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def _segments(seg, with_traj=True):
    """tds_segments for an object with x0..t1 (and optionally traj) arrays."""
    arrs = [getattr(seg, f) for f in FIELDS]
    traj = getattr(seg, "traj", None) if with_traj else None
    keep = []
    if _is_torch(arrs[0]):
        import torch
        mem = L.TDS_MEM_DEVICE
        ptrs = []
        for a in arrs:
            if a.dtype != torch.float64 or not a.is_cuda:
                raise TypeError("device segments must be float64 CUDA tensors")
            a = a.contiguous()
            keep.append(a)
            ptrs.append(a.data_ptr())
        tptr = None
        if traj is not None:
            t = traj.to(device=arrs[0].device, dtype=torch.int64).contiguous()
            keep.append(t)
            tptr = t.data_ptr()
        n = int(arrs[0].numel())
    else:
        mem = L.TDS_MEM_HOST
        ptrs = []
        for a in arrs:
            a = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(a)
            ptrs.append(a.ctypes.data)
        tptr = None
        if traj is not None:
            t = np.ascontiguousarray(traj, dtype=np.int64)
            keep.append(t)
            tptr = t.ctypes.data
        n = int(np.asarray(arrs[0]).shape[0])
    s = L.tds_segments(n, mem, 0, *ptrs, tptr)
    return s, keep, mem


@dataclass
class Hits:
    """Search results in the caller's indices (numpy arrays or torch tensors)."""
    query: object
    entry: object
    traj: object
    ta: object
    tb: object

    def __len__(self):
        return int(self.query.shape[0])

    def sorted(self) -> "Hits":
        """Host copy sorted by (query, entry)."""
        h = self.numpy()
        o = np.lexsort((h.entry, h.query))
        return Hits(h.query[o], h.entry[o], h.traj[o], h.ta[o], h.tb[o])

    def numpy(self) -> "Hits":
        if _is_torch(self.query):
            return Hits(*[x.cpu().numpy() for x in (self.query, self.entry, self.traj, self.ta, self.tb)])
        return self


class Index:
    """A database resident on the GPU (tds_build_index)."""

    def __init__(self, db, num_bins: int, stream=None):
        s, keep, _ = _segments(db, with_traj=True)
        opts = L.tds_index_opts(int(num_bins), 0)
        h = C.c_void_p()
        L.check(L.lib().tds_build_index(C.byref(s), C.byref(opts), _stream_handle(stream), C.byref(h)))
        del keep
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = L.tds_index_info()
        L.check(L.lib().tds_index_info_get(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in L.tds_index_info._fields_}

    def bins(self) -> np.ndarray:
        n = C.c_int64()
        L.check(L.lib().tds_index_bins(self._h, None, 0, C.byref(n)))
        out = (L.tds_bin * max(n.value, 1))()
        L.check(L.lib().tds_index_bins(self._h, out, n.value, C.byref(n)))
        return _bins_array(out, n.value)

    def sorted_times(self):
        """(t_start in the index's order, t_end sorted on its own), host arrays."""
        if getattr(self, "_times", None) is None:
            n = int(self.info()["n"])
            a = np.empty(max(n, 1), np.float64)
            b = np.empty(max(n, 1), np.float64)
            L.check(L.lib().tds_index_times(self._h, a.ctypes.data, b.ctypes.data, n))
            self._times = (a[:n], b[:n])
        return self._times

    def close(self):
        if self._h:
            L.lib().tds_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BIN_DTYPE = np.dtype([("start", "f8"), ("end", "f8"), ("first", "i8"), ("last", "i8"), ("bin", "i8")])


def _bins_array(cbins, n) -> np.ndarray:
    return np.frombuffer(bytes(cbins)[: n * BIN_DTYPE.itemsize], dtype=BIN_DTYPE).copy()


@dataclass
class TrajHits:
    """Trajectory-level results: maximal intervals per trajectory pair."""
    query_traj: object
    entry_traj: object
    ta: object
    tb: object

    def __len__(self):
        return int(self.query_traj.shape[0])


def point_segments(x, y, z, t0, t1):
    """Stationary query points over [t0, t1] as segments with equal end points.

    A point query is the special case of a query segment whose velocity is
    zero; the same kernels answer it.
    """
    class Seg:
        pass

    s = Seg()
    s.x0 = s.x1 = np.ascontiguousarray(x, dtype=np.float64)
    s.y0 = s.y1 = np.ascontiguousarray(y, dtype=np.float64)
    s.z0 = s.z1 = np.ascontiguousarray(z, dtype=np.float64)
    s.t0 = np.ascontiguousarray(t0, dtype=np.float64)
    s.t1 = np.ascontiguousarray(t1, dtype=np.float64)
    return s


class Prepared:
    """Query segments and thresholds marshalled once for repeated batches.

    Holds the tds_segments struct, the threshold pointer and references that
    keep the arrays alive; passing it to Query.batch skips the per-call
    conversion (the library reads the same memory again, so arrays changed in
    place are seen by the next batch).
    """

    def __init__(self, q, d):
        s, keep, mem = _segments(q, with_traj=False)
        if mem == L.TDS_MEM_DEVICE:
            import torch
            dd = d if _is_torch(d) else torch.as_tensor(np.broadcast_to(d, (s.n,)), dtype=torch.float64,
                                                        device=q.x0.device)
            dd = dd.to(torch.float64).contiguous()
            if dd.numel() != s.n:
                dd = dd.expand(s.n).contiguous()
            dptr = dd.data_ptr()
        else:
            dd = np.ascontiguousarray(np.broadcast_to(np.asarray(d, dtype=np.float64), (s.n,)))
            dptr = dd.ctypes.data
        keep.append(dd)
        self.segments, self.dptr, self.keep, self.mem = s, dptr, keep, mem
        self.n = int(s.n)


def prepare(q, d) -> Prepared:
    return Prepared(q, d)


def query_opts(mode="fp64", tiling="periodic", batch_size=0, block_size=0, capacity=0, grid=0,
               max_retries=-1, timing=False, count_overlap=False, kernel_overlap=False):
    """tds_query_opts; timing: True records every stage, "pair" only the pair kernel."""
    tflag = L.TDS_QF_TIMING_PAIR if timing == "pair" else (L.TDS_QF_TIMING if timing else 0)
    flags = (tflag | (L.TDS_QF_COUNT_OVERLAP if count_overlap else 0)
             | (L.TDS_QF_KERNEL_OVERLAP if kernel_overlap else 0))
    return L.tds_query_opts(MODES[mode], TILINGS[tiling], int(batch_size), int(block_size), 0,
                            int(max_retries), int(capacity), int(grid), flags)


class Query:
    """One query handle (tds_query_create): buffers reused across batches."""

    def __init__(self, index: Index):
        self.index = index
        h = C.c_void_p()
        L.check(L.lib().tds_query_create(index.handle, C.byref(h)))
        self._h = h
        self._keep = None
        self._nq = 0
        self._stream = None
        self._rows_hint = 1024  # output rows for the next fetch

    @property
    def handle(self):
        """The tds_query pointer (for callers of the C ABI)."""
        return self._h

    def batch(self, q, d, mode="fp64", tiling="periodic", batch_size=0, block_size=0,
              capacity=0, grid=0, max_retries=-1, timing=False, count_overlap=False,
              kernel_overlap=False, stream=None):
        p = q if isinstance(q, Prepared) else Prepared(q, d)
        s, dptr, keep = p.segments, p.dptr, p.keep
        o = query_opts(mode, tiling, batch_size, block_size, capacity, grid, max_retries, timing,
                       count_overlap, kernel_overlap)
        L.check(L.lib().tds_query_batch(self._h, C.byref(s), dptr, C.byref(o), _stream_handle(stream)))
        self._stream = stream
        self._keep = keep  # device inputs must outlive the batch
        self._nq = int(s.n)
        return self

    def fetch(self, out: str = "host", cap: Optional[int] = None) -> Hits:
        """Results of the last batch. The output buffer is sized from the
        previous batch's hit count, so one library call usually suffices; a
        larger result is fetched again into a buffer of its size.

        out: "device" (CUDA tensors), "host" (numpy), or "pinned" (numpy
        arrays over page-locked host memory, which the library's record
        kernel writes directly: no staging copy)."""
        n = C.c_int64()
        rows = max(self._rows_hint, 1) if cap is None else max(int(cap), 1)
        if out == "device":
            import torch
            mk = lambda r: torch.empty((r, 5), dtype=torch.int64, device="cuda")
            ptr, mem = (lambda b: b.data_ptr()), L.TDS_MEM_DEVICE
        elif out == "pinned":
            import torch
            mk = lambda r: torch.empty((r, 5), dtype=torch.int64, pin_memory=True).numpy()
            ptr, mem = (lambda b: b.ctypes.data), L.TDS_MEM_HOST
        else:
            mk = lambda r: np.empty((r, 5), dtype=np.int64)
            ptr, mem = (lambda b: b.ctypes.data), L.TDS_MEM_HOST
        buf = mk(rows)
        L.check(L.lib().tds_fetch_results(self._h, C.c_void_p(ptr(buf)), rows, mem, C.byref(n)))
        total = int(n.value)
        m = total if cap is None else min(int(cap), total)
        if m > rows:
            buf = mk(m)
            L.check(L.lib().tds_fetch_results(self._h, C.c_void_p(ptr(buf)), m, mem, C.byref(n)))
        self._rows_hint = max(1024, total + total // 4)
        if out == "device":
            import torch
            if m:  # the records are written on the batch's stream
                qs = self._stream
                if qs is not None and not isinstance(qs, int) and qs != torch.cuda.current_stream():
                    torch.cuda.current_stream().wait_stream(qs)
            buf = buf[:m]
            res = Hits(buf[:, 0], buf[:, 1], buf[:, 2], buf[:, 3].view(torch.float64),
                       buf[:, 4].view(torch.float64))
        else:
            arr = buf[:m]
            res = Hits(arr[:, 0].copy(), arr[:, 1].copy(), arr[:, 2].copy(),
                       arr[:, 3].copy().view(np.float64), arr[:, 4].copy().view(np.float64))
        self._keep = None
        return res

    def fetch_trajectories(self, query_traj, out: str = "host", cap: Optional[int] = None) -> "TrajHits":
        """Maximal intervals per (query trajectory, entry trajectory) of the batch.

        query_traj: trajectory id of each query segment of the batch (numpy
        or a CUDA int64 tensor). Sorted by (query_traj, entry_traj, t_a).
        """
        if _is_torch(query_traj):
            import torch
            qt = query_traj.to(torch.int64).contiguous()
            qptr, qmem = qt.data_ptr(), L.TDS_MEM_DEVICE
        else:
            qt = np.ascontiguousarray(query_traj, dtype=np.int64)
            qptr, qmem = qt.ctypes.data, L.TDS_MEM_HOST
        n = C.c_int64()
        L.check(L.lib().tds_fetch_trajectories(self._h, C.c_void_p(qptr), qmem, None, 0, L.TDS_MEM_HOST,
                                               C.byref(n)))
        total = int(n.value)
        m = total if cap is None else min(int(cap), total)
        # the first call merged; a call without ids copies those records
        if out == "device":
            import torch
            buf = torch.empty((max(m, 1), 4), dtype=torch.int64, device="cuda")
            if m:
                L.check(L.lib().tds_fetch_trajectories(self._h, None, qmem,
                                                       C.c_void_p(buf.data_ptr()), m, L.TDS_MEM_DEVICE,
                                                       C.byref(n)))
                qs = self._stream
                if qs is not None and not isinstance(qs, int) and qs != torch.cuda.current_stream():
                    torch.cuda.current_stream().wait_stream(qs)
            buf = buf[:m]
            return TrajHits(buf[:, 0], buf[:, 1], buf[:, 2].view(torch.float64), buf[:, 3].view(torch.float64))
        arr = np.empty((max(m, 1), 4), dtype=np.int64)
        if m:
            L.check(L.lib().tds_fetch_trajectories(self._h, None, qmem,
                                                   C.c_void_p(arr.ctypes.data), m, L.TDS_MEM_HOST,
                                                   C.byref(n)))
        arr = arr[:m]
        return TrajHits(arr[:, 0].copy(), arr[:, 1].copy(), arr[:, 2].copy().view(np.float64),
                        arr[:, 3].copy().view(np.float64))

    def stats(self) -> dict:
        s = L.tds_stats()
        L.check(L.lib().tds_query_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in L.tds_stats._fields_}

    def device_bytes(self) -> int:
        """Device memory the handle holds now (tds_query_device_bytes)."""
        n = C.c_int64()
        L.check(L.lib().tds_query_device_bytes(self._h, C.byref(n)))
        return int(n.value)

    def tiles(self):
        """Tiles of the last fetched batch and the caller indices in tile order.

        Returns (tiles, members): tiles is a structured array with fields
        q_first, n_query, e_first, n_entry (q_first indexes members).
        """
        nt, nm = C.c_int64(), C.c_int64()
        L.check(L.lib().tds_query_tiles(self._h, None, 0, None, 0, C.byref(nt), C.byref(nm)))
        dt = np.dtype([("q_first", np.int32), ("n_query", np.int32), ("e_first", np.int32),
                       ("n_entry", np.int32)])
        tiles = np.zeros(max(nt.value, 1), dtype=dt)
        members = np.zeros(max(nm.value, 1), dtype=np.int32)
        L.check(L.lib().tds_query_tiles(self._h, tiles.ctypes.data, nt.value, members.ctypes.data,
                                        nm.value, C.byref(nt), C.byref(nm)))
        return tiles[: nt.value], members[: nm.value]

    def ranges(self):
        first = np.empty(max(self._nq, 1), np.int64)
        last = np.empty(max(self._nq, 1), np.int64)
        L.check(L.lib().tds_query_ranges(self._h, first.ctypes.data, last.ctypes.data, self._nq))
        return first[: self._nq], last[: self._nq]

    def close(self):
        if self._h:
            L.lib().tds_query_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ flat names
def build_index(db, num_bins: int, stream=None) -> Index:
    return Index(db, num_bins, stream=stream)


def query_batch(target, q, d, **opts) -> Query:
    qh = target if isinstance(target, Query) else Query(target)
    return qh.batch(q, d, **opts)


def fetch_results(qh: Query, out: str = "host", cap: Optional[int] = None) -> Hits:
    return qh.fetch(out=out, cap=cap)


def search(index: Index, q, d, **opts) -> Hits:
    qh = Query(index)
    try:
        qh.batch(q, d, **opts)
        return qh.fetch()
    finally:
        qh.close()


def search_noalloc(index: Index, q, d, out, mode="fp64", tiling="range", batch_size=0, block_size=0,
                   grid=0, stream=None) -> int:
    """tds_search_noalloc: one search whose buffers all live in the library's
    fixed device scratch (no allocation). q: device segments (float64 CUDA
    tensors), d: thresholds, out: a (cap, 5) int64 CUDA tensor receiving
    tds_hit records. Returns the number of hits (records beyond cap are
    counted, not written)."""
    p = q if isinstance(q, Prepared) else Prepared(q, d)
    if p.mem != L.TDS_MEM_DEVICE:
        raise TypeError("search_noalloc takes device segments")
    o = L.tds_query_opts(MODES[mode], TILINGS[tiling], int(batch_size), int(block_size), 0, -1, 0,
                         int(grid), 0)
    n = C.c_int64()
    cap = int(out.shape[0]) if out is not None else 0
    L.check(L.lib().tds_search_noalloc(index.handle, C.byref(p.segments), p.dptr, C.byref(o),
                                       C.c_void_p(out.data_ptr() if cap else 0), cap, C.byref(n),
                                       _stream_handle(stream)))
    return int(n.value)


def plan_bins(t0_sorted, t1_sorted, num_bins: int) -> np.ndarray:
    """Host-side bin table of entries already sorted by t_start (no GPU)."""
    t0 = np.ascontiguousarray(t0_sorted, dtype=np.float64)
    t1 = np.ascontiguousarray(t1_sorted, dtype=np.float64)
    n = C.c_int64()
    L.check(L.lib().tds_plan_bins(t0.ctypes.data, t1.ctypes.data, t0.size, int(num_bins), None, 0,
                                  C.byref(n)))
    out = (L.tds_bin * max(n.value, 1))()
    L.check(L.lib().tds_plan_bins(t0.ctypes.data, t1.ctypes.data, t0.size, int(num_bins), out,
                                  n.value, C.byref(n)))
    return _bins_array(out, n.value)


def plan_ranges(bins: np.ndarray, t0, t1):
    """Host-side candidate range per (t0, t1) span from a bin table."""
    b = np.ascontiguousarray(bins, dtype=BIN_DTYPE)
    t0 = np.ascontiguousarray(t0, dtype=np.float64)
    t1 = np.ascontiguousarray(t1, dtype=np.float64)
    first = np.empty(max(t0.size, 1), np.int64)
    last = np.empty(max(t0.size, 1), np.int64)
    L.check(L.lib().tds_plan_ranges(b.ctypes.data_as(C.POINTER(L.tds_bin)), b.size, t0.ctypes.data,
                                    t1.ctypes.data, t0.size, first.ctypes.data, last.ctypes.data))
    return first[: t0.size], last[: t0.size]


_torch_hooks = None  # the callbacks must outlive their registration


def use_torch_allocator(enable: bool = True) -> None:
    """Serve the library's device buffers from PyTorch's caching allocator.

    Buffers allocated after the call come from torch (and show up in
    torch.cuda.memory_allocated()); buffers already allocated go back to the
    allocator that made them. enable=False restores hipMalloc / hipFree.
    """
    global _torch_hooks
    if not enable:
        L.check(L.lib().tds_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None))
        return
    import torch

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      int(stream or 0))
        except Exception:  # reported to the caller as TDS_ENOMEM
            return None

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    hooks = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
    L.check(L.lib().tds_set_allocator(hooks[0], hooks[1], None))
    # keep every registered pair: buffers made by an earlier one free through it
    _torch_hooks = (_torch_hooks or ()) + (hooks,)


class NativeServer:
    """The library's serving runtime (tds_server_*): a scheduler thread and
    `streams` executors in native code. Requests are host arrays; each is
    submitted with its arrival time on the server's clock (seconds), and
    the arrays are kept referenced here until the request is released."""

    def __init__(self, index: Index, streams=4, max_batch_segments=65536, max_waiting=0,
                 pool_bytes=256 * (1 << 20), k_safety=4.0, epochs=50, reserve_segments=0,
                 alpha_prior=1e-4, mode="fp32_refine", tiling="range", batch_size=0, block_size=0):
        q = L.tds_query_opts(MODES[mode], TILINGS[tiling], int(batch_size), int(block_size), 0, -1, 0, 0, 0)
        o = L.tds_server_opts(int(streams), int(max_batch_segments), int(max_waiting), float(pool_bytes),
                              float(k_safety), int(epochs), int(reserve_segments), float(alpha_prior), q)
        h = C.c_void_p()
        L.check(L.lib().tds_server_create(index.handle, C.byref(o), C.byref(h)))
        self.index = index
        self._h = h
        self._keep = {}

    def now(self) -> float:
        return float(L.lib().tds_server_now(self._h))

    def submit(self, q, d, arrival: float = 0.0) -> int:
        """Submit host segments q with thresholds d (scalar or per segment);
        raises TdsError (code TDS_EBUSY) when the waiting queue is full."""
        s, keep, mem = _segments(q, with_traj=False)
        if mem != L.TDS_MEM_HOST:
            raise TypeError("server requests are host arrays")
        dd = np.ascontiguousarray(np.broadcast_to(np.asarray(d, dtype=np.float64), (int(s.n),)))
        rid = C.c_int64()
        L.check(L.lib().tds_server_submit(self._h, C.byref(s), dd.ctypes.data_as(C.c_void_p),
                                          float(arrival), C.byref(rid)))
        self._keep[rid.value] = (keep, dd)
        return rid.value

    def wait(self, rid: int, timeout: float = -1.0) -> dict:
        info = L.tds_request_info()
        L.check(L.lib().tds_server_wait(self._h, int(rid), float(timeout), C.byref(info)))
        return {f: getattr(info, f) for f, _ in L.tds_request_info._fields_}

    def results(self, rid: int) -> Hits:
        n = C.c_int64()
        L.check(L.lib().tds_server_results(self._h, int(rid), None, 0, C.byref(n)))
        buf = np.empty((max(n.value, 1), 5), dtype=np.int64)
        L.check(L.lib().tds_server_results(self._h, int(rid), buf.ctypes.data_as(C.c_void_p), n.value,
                                           C.byref(n)))
        buf = buf[:n.value]
        return Hits(buf[:, 0].copy(), buf[:, 1].copy(), buf[:, 2].copy(), buf[:, 3].view(np.float64).copy(),
                    buf[:, 4].view(np.float64).copy())

    def release(self, rid: int) -> None:
        L.check(L.lib().tds_server_release(self._h, int(rid)))
        self._keep.pop(int(rid), None)

    def stats(self) -> dict:
        st = L.tds_server_stats()
        L.check(L.lib().tds_server_stats_get(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in L.tds_server_stats._fields_}

    def alpha(self) -> np.ndarray:
        n = C.c_int32()
        L.check(L.lib().tds_server_alpha(self._h, None, 0, C.byref(n)))
        a = np.empty(n.value, dtype=np.float64)
        L.check(L.lib().tds_server_alpha(self._h, a.ctypes.data_as(C.c_void_p), n.value, C.byref(n)))
        return a

    def close(self):
        if self._h:
            L.lib().tds_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
