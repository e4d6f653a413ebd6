"""Writes r8_collapse.txt: query/entry pairs whose interval roots cross.

Reading R8 of the interval computation (Sec. 5, Alg. 1's time interval
from the degree-two polynomial): when rounding puts the computed entry time
after the computed exit time, the interval collapses to the point of
closest approach clamped to the common span. This script finds pairs that
take that branch: a straight pass by an entry at rest whose distance reaches
d within a few ulps of the end of the common span, the closest approach
lying after it. A copy of the oracle whose collapse writes NaN marks the
branch; only the oracle package is used. Run from the repository root:

    python tests/golden/make_r8_collapse.py
"""
from __future__ import annotations

import os
import sys
import tempfile
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from oracle.build import SRC, build  # noqa: E402

COLLAPSE = ("        double tv = dmin(dmax(-B / a, 0.0), T);\n"
            "        a_ = tlo + tv;\n"
            "        b_ = a_;")
OUT = Path(__file__).resolve().parent / "r8_collapse.txt"


def candidates(rng):
    """Straight passes reaching distance d near the end of the common span."""
    while True:
        T = float(rng.uniform(0.1, 12.0))
        d = float(rng.uniform(0.05, 5.0))
        s = float(rng.uniform(0.05, 4.0))
        t0 = float(rng.choice([0.0, float(rng.integers(-50, 50)), rng.uniform(-100.0, 100.0)]))
        h = d * float(rng.uniform(0.0, 0.99))           # miss distance of the pass
        w = np.sqrt(d * d - h * h) / s                 # half-time within d
        tc = T + w * (1.0 + float(rng.choice([0, 1, -1])) * 2.0 ** -int(rng.integers(30, 53)))
        ex, ey, ez = (float(v) for v in rng.uniform(-50.0, 50.0, 3))
        ang = float(rng.uniform(0.0, 2.0 * np.pi))
        c, sn = np.cos(ang), np.sin(ang)

        def at(t):
            x = s * (t - tc)
            return ex + c * x - sn * h, ey + sn * x + c * h, ez

        a0, a1 = at(0.0), at(T)
        q = [a0[0], a0[1], a0[2], t0, a1[0], a1[1], a1[2], t0 + T]
        e = [ex, ey, ez, t0 - float(rng.uniform(0.0, 1.0)), ex, ey, ez,
             t0 + T + float(rng.uniform(0.0, 1.0))]
        yield [float(v) for v in q], [float(v) for v in e], d


def main(count: int = 8, seed: int = 14057461):
    with tempfile.TemporaryDirectory() as tmp:
        text = SRC.read_text()
        assert text.count(COLLAPSE) == 1, "collapse branch not found in oracle.c"
        marked = oracle.load(build(out=Path(tmp), src_text=text.replace(COLLAPSE, "        a_ = b_ = NAN;")))
        found = []
        for q, e, d in candidates(np.random.default_rng(seed)):
            code, ta, _ = oracle.pair(q, e, d, lib=marked)
            if code == 1 and np.isnan(ta):
                found.append((q, e, d))
                if len(found) == count:
                    break
    with open(OUT, "w") as f:
        f.write("# Pairs that take the interval collapse of reading R8 (Sec. 5, Alg. 1's time\n"
                "# interval): written by make_r8_collapse.py with the oracle only.\n"
                "# Values are binary64 in hexadecimal (float.fromhex).\n"
                "# pair qx0 qy0 qz0 qt0 qx1 qy1 qz1 qt1 ex0 ey0 ez0 et0 ex1 ey1 ez1 et1 d\n")
        for q, e, d in found:
            f.write("pair " + " ".join(float(v).hex() for v in q + e + [d]) + "\n")
    print(f"{len(found)} pairs -> {OUT}")


if __name__ == "__main__":
    main()
