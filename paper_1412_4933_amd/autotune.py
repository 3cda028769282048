"""Autotuner for the launch shape of the tile engine.

Results never depend on the tiling (regions of 64*nw columns x rows, steps
per launch, workgroup size) or on the number of persistent workgroups per
compute unit, so the tuner only measures: it runs every candidate for a few
steps on a throwaway copy of the workload and keeps the fastest. Results are
cached per workload signature (grid-size bucket, mode mix, scenario count),
in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import pedsim

# (nw, rows, steps per launch, threads); nw = 0 is the row-lane engine. Shapes
# the library rejects for a workload (the tour variant and the eight-neighbour
# set take nw = 0 only) are skipped.
PLAIN_CANDIDATES = [
    (1, 32, 1, 256), (1, 32, 2, 512), (1, 48, 2, 512), (1, 64, 2, 512), (1, 64, 3, 512),
    (1, 96, 2, 1024), (1, 128, 3, 1024), (2, 32, 2, 512), (2, 64, 2, 1024), (2, 64, 3, 1024),
    (0, 64, 2, 256), (0, 64, 3, 256), (0, 64, 4, 256), (0, 48, 2, 256), (0, 64, 3, 512),
    (0, 56, 4, 512), (0, 52, 4, 512), (0, 48, 6, 512), (3, 48, 2, 256), (3, 48, 3, 256),
    (3, 64, 2, 256), (3, 50, 2, 256),
]
# (nw, rows, steps per launch, threads, workgroups per CU)
BATCH_CANDIDATES = [
    (1, 32, 1, 256, 4), (1, 32, 2, 512, 2), (1, 32, 2, 512, 4), (1, 48, 2, 512, 2), (1, 64, 2, 512, 2),
    (1, 64, 3, 512, 2), (1, 64, 2, 1024, 1), (1, 96, 3, 1024, 1), (2, 48, 2, 1024, 1),
    (0, 64, 2, 256, 2), (0, 64, 3, 256, 2), (0, 48, 2, 256, 3), (0, 64, 2, 128, 4),
    (0, 48, 3, 512, 2), (3, 48, 2, 256, 4), (3, 48, 3, 256, 4), (3, 56, 3, 256, 4), (3, 60, 3, 256, 4),
    (3, 62, 3, 256, 4),
]

_cache: Dict[str, tuple] = {}


def _bucket(v: float) -> int:
    return int(round(math.log2(max(v, 1.0)) * 2))


def signature(scns: Sequence, kind: str) -> str:
    cells = sum(s.W * s.H for s in scns)
    aco = sum(1 for s in scns if s.mode != 0)
    tour = sum(1 for s in scns if s.mode == 2)
    nb = max(getattr(s, "neighbours", 5) for s in scns)
    return f"{kind}:n{len(scns)}:c{_bucket(cells)}:a{_bucket(aco + 1)}:t{_bucket(tour + 1)}:nb{nb}"


def load(path: Optional[str]) -> None:
    if path and os.path.exists(path):
        with open(path) as f:
            _cache.update({k: tuple(v) for k, v in json.load(f).items()})


def save(path: Optional[str]) -> None:
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump({k: list(v) for k, v in _cache.items()}, f, indent=1)


def _time(fn, sync) -> float:
    sync()
    t0 = time.perf_counter()
    fn()
    sync()
    return time.perf_counter() - t0


def tune_plain(scn, mode: int, steps: int = 40, candidates: Iterable = PLAIN_CANDIDATES,
               device: str = "cuda") -> Tuple[tuple, List[tuple]]:
    """Fastest tiling for one scenario run alone; returns (best, [(seconds, tiling)])."""
    import torch
    key = signature([scn], f"plain{mode}")
    timings = []
    for tl in candidates:
        sim = pedsim.Sim(scn, device=device)
        try:
            sim.set_tiling(mode, *tl)
        except pedsim.SimError:
            sim.close()
            continue
        sim.step(2 * tl[2], mode)
        dt = _time(lambda: sim.step(steps, mode), torch.cuda.synchronize)
        sim.close()
        timings.append((dt, tl))
    timings.sort()
    _cache[key] = timings[0][1]
    return timings[0][1], timings


def cached_plain(scn, mode: int) -> Optional[tuple]:
    return _cache.get(signature([scn], f"plain{mode}"))


def tune_batch(scns: Sequence, steps: int = 20, candidates: Iterable = BATCH_CANDIDATES,
               device: str = "cuda") -> Tuple[tuple, List[tuple]]:
    """Fastest batch tuning for a set of scenarios advanced together; returns
    (best (nw, rows, k, threads, wgs_per_cu), [(seconds, tuning)])."""
    import torch
    key = signature(scns, "batch")
    timings = []
    batch = pedsim.Batch(len(scns), device=device)
    try:
        nb = getattr(scns[0], "neighbours", 5) if scns else 5
        if nb != 5:
            batch.set_neighbours(nb)
        elif any(s.mode == 2 for s in scns):
            batch.set_tuning(0, 48, 3, 512, 2)  # tour scenarios need the LDS form before they are added
        for s in scns:
            batch.add(s)
        for tu in candidates:
            try:
                batch.set_tuning(*tu, 1)
            except pedsim.SimError:
                continue
            batch.step(steps)  # instantiate this launch count's graph outside the timed region
            dt = _time(lambda: batch.step(steps), torch.cuda.synchronize)
            timings.append((dt, tu))
    finally:
        batch.close()
    timings.sort()
    _cache[key] = timings[0][1]
    return timings[0][1], timings


def cached_batch(scns: Sequence) -> Optional[tuple]:
    return _cache.get(signature(scns, "batch"))
