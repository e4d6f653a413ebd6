"""Measured autotuner for the search's launch parameters.

Replaces the paper's offline performance model for choosing the batch size
(Sec. 8, Table 3) with measurement on the device: every candidate
configuration runs the same query batch, the fastest wins, and all of them
must report the same number of hits (the hit set does not depend on launch
shape, so a mismatch is an error, not a tuning result).

Searched: bin count m (rebuilds the index), tiling (range buckets, the
paper's Periodic batches, or its GreedySetSplit-Min / -Max batches of
Alg. 4), the batch size s of Periodic or the bound of GreedySetSplit, and
the workgroup size.
Results are cached in a JSON file keyed by the workload's shape.
"""
from __future__ import annotations

import itertools
import json
import os
import time
from dataclasses import dataclass, field
from pathlib import Path
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import api

DEFAULT_CACHE = Path(os.environ.get("TDS_TUNE_CACHE", Path.home() / ".cache" / "tds_autotune.json"))


@dataclass
class Trial:
    num_bins: int
    opts: Dict
    ms: float
    pair_ms: float
    n_hit: int
    n_eval: int
    prep_ms: float = 0.0   # query preparation, sort and tiling (HIP events)
    n_tiles: int = 0


@dataclass
class TuneResult:
    num_bins: int
    opts: Dict
    ms: float
    trials: List[Trial] = field(default_factory=list)

    def as_dict(self):
        return {"num_bins": self.num_bins, "opts": self.opts, "ms": self.ms}


def workload_key(n_entries: int, n_queries: int, d, mode: str) -> str:
    """Cache key: sizes rounded to powers of two, d by decade."""
    dd = np.asarray(d, dtype=np.float64)
    dmed = float(np.median(dd)) if dd.size else 0.0
    dcls = int(np.floor(np.log10(dmed))) if dmed > 0 else -99
    return f"n{int(np.log2(max(n_entries, 1)))}_q{int(np.log2(max(n_queries, 1)))}_d{dcls}_{mode}"


def _time_config(qh, q, d, opts, reps, stream):
    import torch
    best_ms, best_pair, best_prep, hits, n_eval, n_tiles = np.inf, np.inf, np.inf, None, None, 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qh.batch(q, d, timing=True, stream=stream, **opts)
        h = qh.fetch(out="device")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        st = qh.stats()
        best_ms = min(best_ms, ms)
        best_pair = min(best_pair, st["ms_pair"])
        best_prep = min(best_prep, st["ms_prep"])
        hits, n_eval, n_tiles = len(h), st["n_eval"], st["n_tiles"]
    return best_ms, best_pair, best_prep, hits, n_eval, n_tiles


def tune(db, q, d, mode: str = "fp32_refine", num_bins: Sequence[int] = (250, 500, 1000, 2000, 4000),
         tilings: Sequence[str] = ("range", "periodic", "greedy_min", "greedy_max"),
         batch_sizes: Sequence[int] = (64, 128, 256),
         blocks: Sequence[int] = (64, 256, 1024),
         reps: int = 3, cache: Optional[Path] = DEFAULT_CACHE, use_cache: bool = True,
         log=None) -> TuneResult:
    """Search the grid on (db, q, d) and return the fastest configuration.

    ``q`` may hold host (numpy) or device (torch) arrays; device arrays give
    timings without host transfers, as the search is used in practice.
    """
    import torch
    n_q = int(q.t0.shape[0])
    key = workload_key(len(db.t0) if hasattr(db, "t0") else 0, n_q, d if not hasattr(d, "cpu") else d.cpu().numpy(), mode)
    if use_cache and cache is not None and Path(cache).exists():
        try:
            hit = json.loads(Path(cache).read_text()).get(key)
            if hit:
                return TuneResult(hit["num_bins"], hit["opts"], hit["ms"])
        except (OSError, ValueError):
            pass
    stream = torch.cuda.current_stream()
    trials: List[Trial] = []
    ref_hits = None
    for m in num_bins:
        ix = api.build_index(db, m)
        qh = api.Query(ix)
        try:
            for tiling, blk in itertools.product(tilings, blocks):
                for bs in (batch_sizes if tiling != "range" else (0,)):
                    opts = dict(mode=mode, tiling=tiling, block_size=blk)
                    if bs:
                        opts["batch_size"] = bs
                    ms, pair_ms, prep_ms, hits, n_eval, n_tiles = _time_config(qh, q, d, opts, reps,
                                                                                stream)
                    if ref_hits is None:
                        ref_hits = hits
                    if hits != ref_hits:
                        raise RuntimeError(f"hit count {hits} != {ref_hits} for m={m} {opts}")
                    trials.append(Trial(m, opts, ms, pair_ms, hits, n_eval, prep_ms, n_tiles))
                    if log:
                        log(f"m={m} {opts}: {ms:.3f} ms (pair {pair_ms:.3f}, prep {prep_ms:.3f}), "
                            f"N_eval {n_eval}, tiles {n_tiles}")
        finally:
            qh.close()
            ix.close()
    best = min(trials, key=lambda t: t.ms)
    res = TuneResult(best.num_bins, best.opts, best.ms, trials)
    if cache is not None:
        try:
            Path(cache).parent.mkdir(parents=True, exist_ok=True)
            data = json.loads(Path(cache).read_text()) if Path(cache).exists() else {}
            data[key] = res.as_dict()
            Path(cache).write_text(json.dumps(data, indent=1, sort_keys=True))
        except (OSError, ValueError):
            pass
    return res
