"""FP64 brute-force oracle for the distance-threshold search.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. It shares no
code with the GPU library: ``oracle.c`` (compiled with gcc) does the
arithmetic, ``exact.py`` re-decides tiny cases in exact rational arithmetic.

What is computed: paper Sec. 3 (problem definition) and Sec. 5, Alg. 1
(temporal intersection, then the time interval within d from a degree-two
polynomial), over all query/entry pairs. The readings taken where the paper
is silent are listed at the top of ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from pathlib import Path
from typing import Optional

import numpy as np

from .build import build as _build

_LIB = None
_LIB_PATH: Optional[Path] = None


def _configure(lib):
    lib.oracle_search.restype = C.c_int64
    lib.oracle_search.argtypes = [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                  C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_int64), C.c_int]
    lib.oracle_pair.restype = C.c_int
    lib.oracle_pair.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
    return lib


def load(path: Optional[Path] = None):
    """The oracle library as a ctypes CDLL.

    With no ``path`` the real oracle is built (if needed) and cached; a
    ``path`` loads that build (e.g. a modified copy in a test) uncached.
    """
    global _LIB, _LIB_PATH
    if path is None:
        if _LIB is None:
            _LIB_PATH = _build()
            _LIB = _configure(C.CDLL(str(_LIB_PATH)))
        return _LIB
    return _configure(C.CDLL(str(path)))


def _ptrs(arrs):
    keep = [np.ascontiguousarray(a, dtype=np.float64) for a in arrs]
    p = (C.c_void_p * 8)(*[a.ctypes.data for a in keep])
    return p, keep


@dataclass
class Hits:
    q: np.ndarray      # query index (caller order)
    e: np.ndarray      # entry index (caller order)
    ta: np.ndarray
    tb: np.ndarray
    n_overlap: int     # pairs with a non-empty common time span

    def __len__(self):
        return int(self.q.shape[0])


def search(db, q, d=None, nthreads: int = 0, lib=None) -> Hits:
    """All hits of query segments ``q`` against database ``db`` (gen.Segments).

    ``d``: per-query thresholds (defaults to ``q.d``). Hits come sorted by
    (query, entry).
    """
    lib = load() if lib is None else lib
    dq = np.ascontiguousarray(q.d if d is None else np.broadcast_to(d, (len(q),)), dtype=np.float64)
    ep, ek = _ptrs(db.arrays())
    qp, qk = _ptrs(q.arrays())
    novl = C.c_int64(0)
    cap = 1 << 16
    while True:
        oq = np.empty(cap, np.int64)
        oe = np.empty(cap, np.int64)
        ota = np.empty(cap, np.float64)
        otb = np.empty(cap, np.float64)
        n = lib.oracle_search(len(db), ep, len(q), qp, dq.ctypes.data, cap,
                              oq.ctypes.data, oe.ctypes.data, ota.ctypes.data, otb.ctypes.data,
                              C.byref(novl), int(nthreads))
        if n == -1:
            raise ValueError("oracle: invalid input")
        if n < 0:
            raise MemoryError("oracle: out of memory")
        if n <= cap:
            del ek, qk
            return Hits(oq[:n].copy(), oe[:n].copy(), ota[:n].copy(), otb[:n].copy(), int(novl.value))
        cap = int(n)


def pair(qrow, erow, d, lib=None):
    """Evaluate one pair from 8-value rows; returns (code, t_a, t_b)."""
    lib = load() if lib is None else lib
    qa = np.ascontiguousarray(qrow, dtype=np.float64)
    ea = np.ascontiguousarray(erow, dtype=np.float64)
    out = np.zeros(2, np.float64)
    r = lib.oracle_pair(qa.ctypes.data, ea.ctypes.data, float(d), out.ctypes.data)
    return int(r), float(out[0]), float(out[1])


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
