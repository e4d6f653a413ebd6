"""Query batches of the paper's Sec. 6 (oracle side).

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``): nothing in
the library imports this module.

Written from the paper:

* Sec. 4, the temporal bins: entries sorted by non-decreasing t_start are cut
  into m bins of equal width (t_last - t_first) / m; a bin records its
  temporal extent and the index range of its members. Readings: the bin of
  an entry is clamp(floor((t_start - t_first) / width), 0, m - 1), t_first is
  the smallest t_start and t_last the largest t_end; a bin starts at its
  smallest member t_start; empty bins are not kept.
* Sec. 4, the candidate range of a time interval (a, b): over the set of bins
  whose temporal extent [start, end] overlaps (a, b) with positive length
  (start < b and end > a), first = the smallest first member index and
  last = the largest last member index; the candidates are the entries
  first..last of the sorted order (contiguous, and it may take in entries of
  bins between them that do not overlap (a, b) themselves).
* Sec. 4, interactions of a batch: the number of its query segments times
  the number of entries in the candidate range of the batch's temporal
  extent [smallest t_start, largest t_end].
* Sec. 6, Periodic: consecutive runs of s query segments in t_start order.
* Sec. 6, Alg. 4, GreedySetSplit-Min: starting from one batch per query
  segment in t_start order, first merge each batch with its successor
  while the merge adds no interactions (a "free" merge); then, in a second
  pass, merge a batch with its successor while the batch holds fewer than
  `bound` segments. GreedySetSplit-Max: the second pass merges a batch with
  its successor while the merged batch would hold at most `bound` segments
  (the reading of the paper's one-line description of the Max variant; see
  the readings of the design notes).

Readings: query segments whose own candidate range is empty (they overlap no
bin and can produce no hit) take no part in batching; ties in t_start keep
the caller order.

The two passes are written as the paper's loops over a list with a cursor i:
"merge B[i] and B[i+1], remove B[i+1]" keeps i, "i <- i + 1" moves on. Here
the batch at the cursor is held as ``cur`` and the list after the cursor is
consumed in order, which performs the same merges without list deletions.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Bins:
    start: np.ndarray   # smallest member t_start
    end: np.ndarray     # largest member t_end
    first: np.ndarray   # first member (sorted entry index)
    last: np.ndarray    # last member
    memo: dict = field(default_factory=dict)  # (a, b) -> candidate range, filled on use


def entry_order(t0) -> np.ndarray:
    """Entries sorted by non-decreasing t_start, ties in caller order."""
    return np.argsort(np.asarray(t0, dtype=np.float64), kind="stable")


def bin_table(t0_sorted, t1_sorted, m: int) -> Bins:
    t0 = np.asarray(t0_sorted, dtype=np.float64)
    t1 = np.asarray(t1_sorted, dtype=np.float64)
    n = t0.size
    if n == 0:
        z = np.zeros(0)
        return Bins(z, z, z.astype(np.int64), z.astype(np.int64))
    t_first, t_last = t0[0], t1.max()
    width = (t_last - t_first) / m
    start, end, first, last = [], [], [], []
    cur = None
    for p in range(n):
        u = np.floor((t0[p] - t_first) / width)
        j = 0 if u <= 0 else (m - 1 if u >= m - 1 else int(u))
        if j != cur:
            start.append(t0[p]), end.append(t1[p]), first.append(p), last.append(p)
            cur = j
        else:
            end[-1] = max(end[-1], t1[p])
            last[-1] = p
    return Bins(np.array(start), np.array(end), np.array(first, dtype=np.int64),
                np.array(last, dtype=np.int64))


def candidate_range(bins: Bins, a: float, b: float) -> Optional[Tuple[int, int]]:
    """(first, last) sorted entry indices of the bins overlapping (a, b), or None.

    Sec. 4 written out: every bin is tested, the overlapping ones give
    first = min of their first members and last = max of their last members.
    """
    key = (float(a), float(b))
    memo = bins.memo
    if key in memo:
        return memo[key]
    hit = (bins.start < b) & (bins.end > a)
    if not hit.any():
        r = None
    else:
        r = (int(bins.first[hit].min()), int(bins.last[hit].max()))
    memo[key] = r
    return r


def _range_size(r) -> int:
    return 0 if r is None else r[1] - r[0] + 1


@dataclass
class Batch:
    order: np.ndarray       # the ordered query segments (caller indices), shared
    pos: int                # the batch is order[pos : pos + n]
    n: int
    t_lo: float             # temporal extent of the batch
    t_hi: float

    @property
    def members(self) -> np.ndarray:
        return self.order[self.pos:self.pos + self.n]

    def merged(self, other: "Batch") -> "Batch":
        assert other.pos == self.pos + self.n  # only adjacent batches merge
        return Batch(self.order, self.pos, self.n + other.n, min(self.t_lo, other.t_lo),
                     max(self.t_hi, other.t_hi))


def num_ints(bins: Bins, batch: Batch) -> int:
    """Interactions of a batch (Sec. 4): segments x entries in its candidate range."""
    return batch.n * _range_size(candidate_range(bins, batch.t_lo, batch.t_hi))


def batch_range(bins: Bins, batch: Batch):
    return candidate_range(bins, batch.t_lo, batch.t_hi)


def singletons(bins: Bins, q_t0, q_t1) -> List[Batch]:
    """One batch per query segment with a non-empty candidate range, t_start order."""
    q_t0 = np.asarray(q_t0, dtype=np.float64)
    q_t1 = np.asarray(q_t1, dtype=np.float64)
    keep = [int(i) for i in np.argsort(q_t0, kind="stable")
            if candidate_range(bins, q_t0[i], q_t1[i]) is not None]
    order = np.array(keep, dtype=np.int64)
    return [Batch(order, k, 1, float(q_t0[i]), float(q_t1[i])) for k, i in enumerate(keep)]


def periodic(bins: Bins, q_t0, q_t1, s: int) -> List[Batch]:
    """Sec. 6 Periodic over the same ordered list."""
    one = singletons(bins, q_t0, q_t1)
    out = []
    for k in range(0, len(one), s):
        b = one[k]
        for x in one[k + 1:k + s]:
            b = b.merged(x)
        out.append(b)
    return out


def free_merges(bins: Bins, batches: List[Batch]) -> List[Batch]:
    """First pass of Alg. 4: merge with the successor while it adds no interactions."""
    out: List[Batch] = []
    if not batches:
        return out
    cur = batches[0]
    for nxt in batches[1:]:
        m = cur.merged(nxt)
        if num_ints(bins, m) == num_ints(bins, cur) + num_ints(bins, nxt):
            cur = m
        else:
            out.append(cur)
            cur = nxt
    out.append(cur)
    return out


def greedy_set_split(bins: Bins, q_t0, q_t1, bound: int, variant: str = "min") -> List[Batch]:
    """Alg. 4, GreedySetSplit-Min (variant "min") or -Max ("max")."""
    if variant not in ("min", "max"):
        raise ValueError(variant)
    groups = free_merges(bins, singletons(bins, q_t0, q_t1))
    out: List[Batch] = []
    if not groups:
        return out
    cur = groups[0]
    for nxt in groups[1:]:
        if variant == "min":
            take = cur.n < bound
        else:
            take = cur.n + nxt.n <= bound
        if take:
            cur = cur.merged(nxt)
        else:
            out.append(cur)
            cur = nxt
    out.append(cur)
    return out


def total_interactions(bins: Bins, batches: List[Batch]) -> int:
    return sum(num_ints(bins, b) for b in batches)
