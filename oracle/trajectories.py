"""Trajectory-level answers from segment-level hits (oracle side).

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``).

Definition (paper Sec. 3: the query asks, per query trajectory, for the
entry trajectories within d and the times at which they are): for each pair
(query trajectory, entry trajectory), the set of times at which some query
segment of the first is within d of some entry segment of the second is the
union of the segment-pair intervals of that pair. Written out as the sorted
list of its maximal closed intervals: sort the pair's intervals by start,
then sweep, extending the current interval while the next one starts at or
before its end (closed intervals that touch belong to one maximal interval).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class TrajHits:
    qtraj: np.ndarray  # int64
    etraj: np.ndarray  # int64
    ta: np.ndarray
    tb: np.ndarray

    def __len__(self):
        return int(self.qtraj.shape[0])


def union_by_trajectory(q_idx, e_idx, ta, tb, q_traj, e_traj) -> TrajHits:
    """Maximal intervals per (query trajectory, entry trajectory).

    q_idx, e_idx, ta, tb: segment-level hits (any order); q_traj, e_traj:
    trajectory id of each query / entry segment. Result sorted by
    (query trajectory, entry trajectory, start).
    """
    qt = np.asarray(q_traj, dtype=np.int64)[np.asarray(q_idx, dtype=np.int64)]
    et = np.asarray(e_traj, dtype=np.int64)[np.asarray(e_idx, dtype=np.int64)]
    a = np.asarray(ta, dtype=np.float64)
    b = np.asarray(tb, dtype=np.float64)
    order = np.lexsort((a, et, qt))
    out_q, out_e, out_a, out_b = [], [], [], []
    cur = None  # [qt, et, start, end]
    for k in order:
        key = (int(qt[k]), int(et[k]))
        if cur is not None and (cur[0], cur[1]) == key and a[k] <= cur[3]:
            cur[3] = max(cur[3], b[k])
            continue
        if cur is not None:
            out_q.append(cur[0]), out_e.append(cur[1]), out_a.append(cur[2]), out_b.append(cur[3])
        cur = [key[0], key[1], float(a[k]), float(b[k])]
    if cur is not None:
        out_q.append(cur[0]), out_e.append(cur[1]), out_a.append(cur[2]), out_b.append(cur[3])
    return TrajHits(np.array(out_q, dtype=np.int64), np.array(out_e, dtype=np.int64),
                    np.array(out_a, dtype=np.float64), np.array(out_b, dtype=np.float64))
