"""Autotuner for the launch shape of the tile engine.

Results never depend on the tiling (regions of 64*nw columns x rows, steps
per launch, workgroup size) or on the number of persistent workgroups per
compute unit, so the tuner only measures. Every candidate is timed from the
same initial state over the same steps (a fresh scenario or batch per
candidate, built from one device copy of the initial planes), after a
throwaway run that loads its kernel. The fastest candidate is cached per
workload signature (grid-size bucket, mode mix, scenario count, candidate
set).

The cache committed beside this module (tunings.json) is what `pedsim.Sim`
and `pedsim.Batch` read when they are created / first stepped: the launch
shapes of the benchmark workloads come from here, and a workload without an
entry keeps the library's built-in default. Regenerate it on the GPU with

    python -m paper_1412_4933_amd.autotune --out tunings.json [--workloads ...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import pedsim

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tunings.json")

# (nw, rows, steps per launch, threads); nw = 0 is the row-lane engine. Shapes
# the library rejects for a workload (the tour variant and the eight-neighbour
# set take nw = 0 only) are skipped.
PLAIN_CANDIDATES = [
    (1, 32, 1, 256), (1, 32, 2, 512), (1, 48, 2, 512), (1, 64, 2, 512), (1, 64, 3, 512),
    (1, 96, 2, 1024), (1, 128, 3, 1024), (2, 32, 2, 512), (2, 64, 2, 1024), (2, 64, 3, 1024),
    (0, 64, 2, 256), (0, 64, 3, 256), (0, 64, 4, 256), (0, 48, 2, 256), (0, 64, 3, 512),
    (0, 56, 4, 512), (0, 52, 4, 512), (0, 48, 6, 512), (0, 56, 2, 512), (0, 64, 2, 512),
    (3, 48, 2, 256), (3, 48, 3, 256), (3, 64, 2, 256), (3, 50, 2, 256), (3, 56, 3, 256), (3, 58, 3, 256),
    (3, 60, 3, 256), (3, 62, 3, 256), (3, 56, 4, 256), (3, 60, 4, 256), (3, 60, 2, 256),
    (0, 50, 5, 512), (0, 52, 5, 512), (0, 54, 5, 512), (0, 56, 5, 512), (0, 62, 5, 512), (0, 52, 6, 512),
    (0, 56, 6, 512), (0, 48, 5, 512),
]
# (nw, rows, steps per launch, threads, workgroups per CU)
BATCH_CANDIDATES = [
    (1, 32, 1, 256, 4), (1, 32, 2, 512, 2), (1, 32, 2, 512, 4), (1, 48, 2, 512, 2), (1, 64, 2, 512, 2),
    (1, 64, 3, 512, 2), (1, 64, 2, 1024, 1), (1, 96, 3, 1024, 1), (2, 48, 2, 1024, 1),
    (0, 64, 2, 256, 2), (0, 64, 3, 256, 2), (0, 48, 2, 256, 3), (0, 64, 2, 128, 4),
    (0, 48, 3, 512, 2), (3, 48, 2, 256, 4), (3, 48, 3, 256, 4), (3, 56, 3, 256, 4), (3, 60, 3, 256, 4),
    (3, 62, 3, 256, 4), (3, 62, 4, 256, 4), (3, 62, 3, 256, 5), (3, 56, 4, 256, 4), (0, 52, 5, 512, 2),
    (0, 52, 4, 512, 2), (3, 62, 2, 256, 4),
]

# (cols, rows, steps per launch, threads) of the range kernel (larger scanning
# and moving ranges); shapes that do not fit a workload's ranges are skipped
RANGE_CANDIDATES = [
    (64, 32, 1, 512), (64, 16, 1, 512), (64, 32, 1, 256), (64, 16, 1, 256), (128, 16, 1, 512),
    (32, 32, 1, 512), (64, 24, 1, 512), (64, 32, 2, 512), (64, 16, 2, 512), (64, 24, 2, 512),
    (32, 32, 2, 512), (48, 32, 2, 512), (64, 16, 3, 512), (32, 16, 3, 512), (64, 32, 2, 256),
    (96, 16, 2, 512), (32, 32, 3, 512), (64, 8, 4, 512), (64, 28, 2, 512), (56, 32, 2, 512), (80, 24, 2, 512),
    (64, 32, 2, 448), (48, 24, 3, 512), (64, 16, 3, 256),
]

_cache: Dict[str, tuple] = {}
_loaded = False


def _bucket(v: float) -> int:
    return int(round(math.log2(max(v, 1.0)) * 2))


def signature(scns: Sequence, kind: str) -> str:
    cells = sum(s.W * s.H for s in scns)
    aco = sum(1 for s in scns if s.mode != 0)
    tour = sum(1 for s in scns if s.mode == 2)
    nb = max(getattr(s, "neighbours", 5) for s in scns)
    key = f"{kind}:n{len(scns)}:c{_bucket(cells)}:a{_bucket(aco + 1)}:t{_bucket(tour + 1)}:nb{nb}"
    ranges = getattr(scns[0], "ranges", None) if len(scns) == 1 else None
    return key + (f":r{ranges[0]}x{ranges[1]}" if ranges else "")


def load(path: Optional[str] = None) -> None:
    """Merge a cache file (default: the committed one) into the cache."""
    path = path or CACHE_PATH
    if os.path.exists(path):
        with open(path) as f:
            _cache.update({k: tuple(v) for k, v in json.load(f).items()})


def save(path: Optional[str] = None) -> None:
    path = path or CACHE_PATH
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump({k: list(v) for k, v in sorted(_cache.items())}, f, indent=1)
        f.write("\n")


def _ensure_loaded() -> None:
    global _loaded
    if not _loaded:
        load(CACHE_PATH)
        _loaded = True


def cached_plain(scn, mode: int) -> Optional[tuple]:
    """The cached tiling of `scn` run alone in `mode`, if any."""
    _ensure_loaded()
    return _cache.get(signature([scn], f"plain{mode}"))


def cached_batch(scns: Sequence) -> Optional[tuple]:
    """The cached (nw, rows, k, threads, wgs_per_cu) of a batch of `scns`."""
    _ensure_loaded()
    return _cache.get(signature(scns, "batch")) if scns else None


def cached_range(scn, mode: int) -> Optional[tuple]:
    """The cached (cols, rows, steps per launch, threads) of the range kernel for `scn`, if any."""
    _ensure_loaded()
    if getattr(scn, "ranges", None) is None:
        return None
    return _cache.get(signature([scn], f"range{mode}"))


def _timed(fn) -> float:
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def tune_plain(scn, mode: int, steps: Optional[int] = None, candidates: Iterable = PLAIN_CANDIDATES,
               device: str = "cuda") -> Tuple[tuple, List[tuple]]:
    """Fastest tiling for one scenario run alone in `mode`, each candidate
    timed over the same `steps` (default: the scenario's own step count) from
    the initial state. Returns (best, [(seconds, tiling)]) and caches best."""
    steps = steps or scn.steps or 100
    key = signature([scn], f"plain{mode}")
    timings = []
    for tl in candidates:
        warm = pedsim.Sim(scn, device=device, autotune=False)
        try:
            warm.set_tiling(mode, *tl)
        except pedsim.SimError:
            warm.close()
            continue
        warm.step(tl[2], mode)  # loads this kernel variant
        warm.close()
        sim = pedsim.Sim(scn, device=device, autotune=False)
        sim.set_tiling(mode, *tl)
        dt = _timed(lambda: sim.step(steps, mode))
        sim.close()
        timings.append((dt, tuple(tl)))
    timings.sort()
    _cache[key] = timings[0][1]
    return timings[0][1], timings


def tune_range(scn, mode: int, steps: Optional[int] = None, candidates: Iterable = RANGE_CANDIDATES,
               device: str = "cuda") -> Tuple[tuple, List[tuple]]:
    """Fastest range-kernel tiling (cols, rows, steps per launch, threads) for one scenario with
    ranges, each candidate timed over the same `steps` from the initial
    state. Returns (best, [(seconds, tiling)]) and caches best."""
    steps = steps or scn.steps or 100
    key = signature([scn], f"range{mode}")
    timings = []
    for tl in candidates:
        warm = pedsim.Sim(scn, device=device, autotune=False)
        try:
            warm.set_range_tiling(*tl)
        except pedsim.SimError:
            warm.close()
            continue
        warm.step(tl[2], mode)  # loads the kernel
        warm.close()
        sim = pedsim.Sim(scn, device=device, autotune=False)
        sim.set_range_tiling(*tl)
        dt = _timed(lambda: sim.step(steps, mode))
        sim.close()
        timings.append((dt, tuple(tl)))
    timings.sort()
    _cache[key] = timings[0][1]
    return timings[0][1], timings


def _prepare(batch, scns) -> None:
    nb = getattr(scns[0], "neighbours", 5) if scns else 5
    if nb != 5:
        batch.set_neighbours(nb)


def tune_batch(scns: Sequence, steps: Optional[int] = None, candidates: Iterable = BATCH_CANDIDATES,
               device: str = "cuda") -> Tuple[tuple, List[tuple]]:
    """Fastest batch tuning for a set of scenarios advanced together, each
    candidate timed over the same `steps` (default: the scenarios' largest
    step count) from the initial state, with direct launches (no graph to
    instantiate inside the timed region; the launches are much longer than
    their host cost). Returns (best (nw, rows, k, threads, wgs_per_cu),
    [(seconds, tuning)]) and caches best."""
    steps = steps or max(s.steps for s in scns) or 100
    key = signature(scns, "batch")
    initial = [pedsim._Resident(s, device) for s in scns]  # one upload; each candidate clones it
    timings = []
    for tu in candidates:
        warm = pedsim.Batch(1, device=device, autotune=False)
        try:
            _prepare(warm, scns)
            warm.set_tuning(*tu, 0)
            warm.add_resident(initial[0].clone())
            warm.step(tu[2])  # loads this kernel variant
        except pedsim.SimError:
            continue
        finally:
            warm.close()
        batch = pedsim.Batch(len(scns), device=device, autotune=False)
        try:
            _prepare(batch, scns)
            batch.set_tuning(*tu, 0)
            for res in initial:
                batch.add_resident(res.clone())
            dt = _timed(lambda: batch.step(steps))
        except pedsim.SimError:
            continue
        finally:
            batch.close()
        timings.append((dt, tuple(tu)))
    del initial
    timings.sort()
    _cache[key] = timings[0][1]
    return timings[0][1], timings


# Workloads whose tunings the committed cache holds: name -> (kind, builder, mode).
def _workloads():
    from . import scenarios as S
    return {
        "lem_200x100": ("plain", S.lem_200x100, S.MODE_LEM),
        "aco_1024x512": ("plain", S.aco_1024x512, S.MODE_ACO),
        "aco_tour_1024x512": ("plain", S.aco_tour_1024x512, S.MODE_ACO_TOUR),
        "aco_nb8_1024x512": ("plain", S.aco_nb8_1024x512, S.MODE_ACO),
        "stress_aco_4096x2048": ("plain", lambda: S.stress_4096x2048(S.MODE_ACO), S.MODE_ACO),
        "stress_lem_4096x2048": ("plain", lambda: S.stress_4096x2048(S.MODE_LEM), S.MODE_LEM),
        "aco_range_1024x512": ("range", lambda: S.range_1024x512(S.MODE_ACO), S.MODE_ACO),
        "lem_range_1024x512": ("range", lambda: S.range_1024x512(S.MODE_LEM), S.MODE_LEM),
        "batched_256": ("batch", S.batched_256, None),
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="tune the launch shapes of the named workloads")
    ap.add_argument("--workloads", default=",".join(_workloads()))
    ap.add_argument("--out", default=CACHE_PATH, help="cache file to merge into and write")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's)")
    args = ap.parse_args(argv)
    load(args.out)
    table = _workloads()
    for name in args.workloads.split(","):
        kind, build, mode = table[name]
        t0 = time.perf_counter()
        if kind == "plain":
            scn = build()
            best, timings = tune_plain(scn, mode, args.steps)
        elif kind == "range":
            scn = build()
            best, timings = tune_range(scn, mode, args.steps)
        else:
            scns = build()
            best, timings = tune_batch(scns, args.steps)
        print(f"{name}: best {best}; " + ", ".join(f"{tu} {dt * 1e3:.2f} ms" for dt, tu in timings[:6])
              + f" ({time.perf_counter() - t0:.1f} s)", flush=True)
        save(args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
