"""Readers of the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                tag, *vals = line.split()
                yield tag, vals


def fig1():
    segs, bins, lookup = [], [], None
    for tag, v in _rows("fig1_index.txt"):
        if tag == "seg":
            segs.append((int(v[0]), float(v[1]), float(v[2])))
        elif tag == "bin":
            bins.append((int(v[0]), float(v[1]), float(v[2]), int(v[3]), int(v[4])))
        elif tag == "lookup":
            lookup = dict(t0=float(v[0]), t1=float(v[1]), first=int(v[2]), last=int(v[3]),
                          overlap=[int(x) for x in v[4:]])
    t0 = np.array([s[1] for s in segs])
    t1 = np.array([s[2] for s in segs])
    return t0, t1, bins, lookup


def fig2():
    batches, totals = [], {}
    for tag, v in _rows("fig2_batches.txt"):
        if tag == "batch":
            batches.append((int(v[0]), float(v[1]), float(v[2])))
        elif tag == "total":
            totals[int(v[0])] = (int(v[1]), int(v[2]))
    return batches, totals


def fig2_greedy():
    rows = []
    for tag, v in _rows("fig2_greedy.txt"):
        if tag == "greedy":
            rows.append((v[0], int(v[1]), [int(x) for x in v[2].split(",")], int(v[3])))
    return rows


def fig1_sec4():
    """Hand-worked ranges and two-segment GreedySetSplit cases on Fig. 1's bins."""
    ranges, greedy = [], []
    for tag, v in _rows("fig1_sec4_ranges.txt"):
        if tag == "range":
            ranges.append((float(v[0]), float(v[1]), int(v[2]), int(v[3])))
        elif tag == "greedy":
            segs = [tuple(float(x) for x in p.split(":")) for p in v[2].split(";")]
            greedy.append((v[0], int(v[1]), segs, [int(x) for x in v[3].split(",")], int(v[4])))
    return ranges, greedy


def r8_collapse():
    """Query/entry rows (8 values each) and d of the R8 collapse fixture."""
    out = []
    for tag, v in _rows("r8_collapse.txt"):
        if tag == "pair":
            x = [float.fromhex(t) for t in v]
            out.append((x[0:8], x[8:16], x[16]))
    return out
