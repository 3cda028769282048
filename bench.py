"""Benchmark: agent-steps/s of the ACO step at 100K agents on one MI355X.

A step is one pass of the whole hot path (request, resolve, commit,
evaporation + deposit, counters) over the 1024x512 grid with 50,000 agents
per group (seeded synthetic input, inputs resident in HBM before timing).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

WORKLOADS = {
    "aco_1024x512": ("aco_1024x512", "ACO 1024x512, 50,000 agents per group (100K), 2,000 steps"),
    "batched_256": ("batched_256", "256 independent scenarios, widths log-uniform 64-2048, H=W/2, "
                    "500-100K agents, half LEM half ACO, seeds 0..255, in one batch"),
    "served": ("served_requests", "Poisson stream of scenarios drawn like the batch, 200-2000 steps each, "
               "continuous batching under an HBM budget"),
    "lem_200x100": ("lem_200x100", "LEM 200x100, 1,000 agents per group, 500 steps"),
    "aco_tour_1024x512": ("aco_tour_1024x512", "ACO tour variant (eq. 5 deposits, tour matrix) 1024x512, "
                          "50,000 agents per group (100K), 2,000 steps"),
    "aco_nb8_1024x512": ("aco_nb8_1024x512", "ACO with all eight neighbours as candidates 1024x512, "
                         "50,000 agents per group (100K), 2,000 steps"),
    "aco_range_1024x512": ("range_1024x512", "ACO 1024x512, 50,000 agents per group (100K), scanning range 4, "
                           "moving range 2, 2,000 steps"),
    "lem_range_1024x512": ("range_1024x512", "LEM 1024x512, 50,000 agents per group (100K), scanning range 4, "
                           "moving range 2, 2,000 steps"),
    "stress_aco_4096x2048": ("stress_4096x2048", "ACO 4096x2048, 5% obstacles, 1M agents"),
    "stress_lem_4096x2048": ("stress_4096x2048", "LEM 4096x2048, 5% obstacles, 1M agents"),
}
# workloads run by the single-scenario path
PLAIN = ("aco_1024x512", "aco_tour_1024x512", "aco_nb8_1024x512", "lem_200x100", "stress_aco_4096x2048",
         "stress_lem_4096x2048", "aco_range_1024x512", "lem_range_1024x512")
MODE_NAMES = {0: "LEM", 1: "ACO", 2: "ACO tour variant"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make(workload):
    from paper_1412_4933_amd import scenarios as S
    if workload == "stress_lem_4096x2048":
        return S.stress_4096x2048(S.MODE_LEM)
    if workload == "lem_range_1024x512":
        return S.range_1024x512(S.MODE_LEM)
    return getattr(S, WORKLOADS[workload][0])()


def algorithmic_bytes_per_step(mode: int, cells: int, agents: int) -> int:
    """Bytes one step of the method must move (lower bound; the few bytes of
    the agents that actually move are left out): every code byte is read,
    every agent's id is read, and for ACO both pheromone planes are read and
    written (8 B read + 8 B write per cell); the tour variant also reads and
    writes every agent's tour length (4 B + 4 B per agent)."""
    return cells * (1 + (16 if mode != 0 else 0)) + agents * (4 + (8 if mode == 2 else 0))


# The sources that define each traced kernel's device code.
KERNEL_SOURCES = {
    "tile_rows_kernel": ("tile_rows.hpp", "tile_engine.hpp", "rules.hpp", "step_plain.hip"),
    "tile_kernel": ("tile_engine.hpp", "rules.hpp", "step_plain.hip"),
    "range_kernel": ("range_step.hip", "range_step.hpp", "rules.hpp"),
}


def kernel_source_digest(kernel: str = "") -> str:
    """Digest of the sources of `kernel` (all kernel sources if unknown)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1412_4933_amd", "csrc")
    names = KERNEL_SOURCES.get(kernel) or tuple(n for n in os.listdir(csrc) if n.endswith((".hip", ".hpp")))
    for name in sorted(names):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str, tiling=None):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only
    if they were taken on the current kernel sources (and the same tiling)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_src_digest") != kernel_source_digest(kernel):
        return None
    if tiling is not None and rec.get("tiling") is not None and list(rec["tiling"]) != list(tiling):
        return None
    return rec.get("bytes_per_launch")


def _oracle_leg(scn, mode, threads, budget_s):
    """Time the oracle on a sample of roughly budget_s seconds: steps
    5..5+n of the workload (the first 5 size the sample)."""
    import oracle
    st = oracle.State.from_scenario(scn, threads=threads)
    t0 = time.perf_counter()
    st.run(mode, 5)
    per = (time.perf_counter() - t0) / 5
    n = max(5, min(scn.steps - 5, int(budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    st.run(mode, n)
    dt = time.perf_counter() - t0
    return scn.agents * n / dt, n, dt


def cpu_baseline(workload: str, budget_s: float):
    """The oracle as it stands, on this host: the plain build on one thread
    (the paper's CPU baseline is one thread) and the OpenMP build of the same
    source on all the cores this process may use (at most 16), each on a
    bounded sample of the workload. `value` and `cores` are the all-core
    leg's."""
    import oracle
    scn = make(workload)
    mode = 1 if workload == "stress_aco_4096x2048" else scn.mode
    threads = oracle.cpu_threads()
    v1, n1, dt1 = _oracle_leg(scn, mode, None, budget_s)
    vn, nn, dtn = _oracle_leg(scn, mode, threads, budget_s)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": vn, "unit": "agent-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"steps 5..{5 + nn} of the {WORKLOADS[workload][1]} workload, "
                      f"C oracle (OpenMP build), {threads} threads, {dtn:.1f} s",
            "one_thread": {"value": v1, "cores": 1,
                           "sample": f"steps 5..{5 + n1}, C oracle (plain build), one thread, "
                                     f"{dt1:.1f} s"},
            "nproc": os.cpu_count(), "affinity_cpus": affinity}


def stress_run(first: int = 300) -> dict:
    """The 4096x2048 ACO workload (5% obstacles, 1M agents) beside the default
    line: the grid whose state does not fit the caches. Its first `first`
    steps and all of its steps, each timed from the initial state with HIP
    events at the tiling the autotuner cache gives it, with the algorithmic
    roofline fraction of each."""
    import torch
    from paper_1412_4933_amd import pedsim
    scn = make("stress_aco_4096x2048")
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    alg = algorithmic_bytes_per_step(1, scn.W * scn.H, scn.agents)
    w = pedsim.Sim(scn, stream=stream)
    w.step(3, 1)
    w.stats()
    tiling = pedsim.sim_get_tiling(w.h, 1)
    source = "autotuner cache" if 1 in w.tuned else "library default"
    w.close()
    out = {"workload": WORKLOADS["stress_aco_4096x2048"][1], "tiling": list(tiling), "tiling_source": source}
    for name, K in ((f"steps_0_{first - 1}", first), ("all_steps", scn.steps)):
        sim = pedsim.Sim(scn, stream=stream)
        torch.cuda.synchronize(dev)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(K, 1)
        b.record(stream)
        torch.cuda.synchronize(dev)
        ms = a.elapsed_time(b)
        sim.close()
        gbs = alg * K / (ms / 1e3) / 1e9
        out[name] = {"steps": K, "ms_per_step": ms / K, "agent_steps_per_s": scn.agents * K / (ms / 1e3),
                     "alg_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def batched_run(K: int, warmup: int, autotune_first: bool = False) -> dict:
    """All 256 scenarios advanced together (one batch, captured launch
    sequences) vs the same scenarios one after another through the plain
    path; K steps each from the initial state. The batch first runs the same
    K-step call untimed (it instantiates that call's graphs and applies the
    autotuner's cached tuning), then every slot is refilled with the initial
    state and the call is timed."""
    import torch
    from paper_1412_4933_amd import autotune, pedsim, scenarios
    scns = scenarios.batched_256(steps=K)
    agents = sum(s.agents for s in scns)
    if autotune_first:
        log("autotuning the batch ...")
        best, timings = autotune.tune_batch(scns, steps=min(K, 200))
        log("autotune:", [(round(t * 1e3, 2), tu) for t, tu in timings[:5]])
    initial = [pedsim._Resident(sc, "cuda") for sc in scns]  # one upload
    batch = pedsim.Batch(len(scns))
    for res in initial:
        batch.add_resident(res.clone())
    batch.step(K)
    torch.cuda.synchronize()
    for slot in list(batch.members):
        batch.remove(slot)
    for res in initial:
        batch.add_resident(res.clone())
    log(f"batch of {len(scns)} scenarios, {agents} agents")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tuning, source = batch.tuning(), batch.tuning_source
    batch.close()
    del initial
    value = agents * K / wall
    log(f"batched: {K} steps in {wall * 1e3:.1f} ms -> {value:.4g} agent-steps/s, "
        f"tuning {tuning} ({source})")
    # back-to-back plain launches of the same scenarios (step calls only)
    plain = 0.0
    for sc in scns:
        if warmup > 0:  # a throwaway run loads the scenario's kernel variant
            sim = pedsim.Sim(sc)
            sim.step(min(warmup, 4), sc.mode)
            sim.close()
        sim = pedsim.Sim(sc)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim.step(K, sc.mode)
        torch.cuda.synchronize()
        plain += time.perf_counter() - t1
        sim.close()
    log(f"back-to-back plain: {plain * 1e3:.1f} ms -> {agents * K / plain:.4g} agent-steps/s")
    return {"scenarios": len(scns), "agents": agents, "steps": K, "wall_s": wall,
            "agent_steps_per_s": value, "tuning": list(tuning), "tuning_source": source,
            "back_to_back_plain": {"agent_steps_per_s": agents * K / plain, "wall_s": plain},
            "speedup_vs_back_to_back": plain / wall}


def run_batched(args):
    K = args.steps if args.steps is not None else 1000
    b = batched_run(K, args.warmup, args.autotune)
    line = {
        "metric": "agent-steps/s (batched, 256 scenarios)", "value": b["agent_steps_per_s"],
        "unit": "agent-steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": b["wall_s"] * 1e3 / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+u32", "data": "synthetic",
        "config": {"workload": WORKLOADS["batched_256"][1], "scenarios": b["scenarios"],
                   "agents": b["agents"], "tuning": b["tuning"], "tuning_source": b["tuning_source"]},
        "back_to_back_plain": b["back_to_back_plain"],
        "speedup_vs_back_to_back": b["speedup_vs_back_to_back"],
    }
    print(json.dumps(line), flush=True)


def served_run(n_requests: int, rate: float, budget: int, quantum: int, seed: int = 1):
    """Continuous batching of a Poisson request stream, and the same requests
    back to back through the plain path. Each request carries its initial
    state (built on the host before the run); serving uploads, validates,
    advances and harvests it."""
    from paper_1412_4933_amd import scenarios, serve
    specs = scenarios.served_requests(n_requests, rng_seed=seed)
    reqs = serve.poisson_requests(specs, rate=rate, seed=seed)
    serve.prebuild(reqs)  # requests arrive with their initial state
    srv = serve.Server(capacity=256, budget_bytes=budget, quantum=quantum)
    t0 = time.perf_counter()
    results = srv.run(reqs)
    wall = time.perf_counter() - t0
    srv.close()
    summary = serve.summarize(results, wall)
    b2b = serve.run_back_to_back(reqs)
    summary.update({"rate_per_s": rate, "budget_bytes": budget, "quantum": quantum,
                    "back_to_back_agent_steps_per_s": b2b["agent_steps_per_s"],
                    "back_to_back_wall_s": b2b["wall_s"],
                    "speedup_vs_back_to_back": b2b["wall_s"] / wall})
    return summary


def calibrate_copy():
    """A plain device copy of known size, for scaling rocprofv3's FETCH_SIZE
    and WRITE_SIZE counters to bytes: 1 GiB read and 1 GiB written per
    dispatch."""
    import torch
    n = 256 * 1024 * 1024
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": n * 4, "dispatches": 4}), flush=True)


def _counter_per_dispatch(run_dir: str, kernel: str, counter: str):
    """Mean value of `counter` per dispatch of kernels whose name contains
    `kernel`, from a rocprofv3 --pmc run's CSV output (summed over the rows of
    one dispatch), and the number of dispatches."""
    import csv
    import glob
    per = {}
    for path in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if kernel not in row.get("Kernel_Name", "") or row.get("Counter_Name") != counter:
                    continue
                key = (path, row.get("Dispatch_Id") or row.get("Correlation_Id"))
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for {kernel} under {run_dir}")
    return sum(per.values()) / len(per), len(per)


def record_traffic(kernel: str, workload: str, fetch_dir: str, write_dir: str, copy_fetch_dir: str,
                   copy_write_dir: str, tiling: str, steps_per_launch: int) -> None:
    """Write profiles/traffic_<kernel>_<workload>.json from four rocprofv3
    --pmc runs (FETCH_SIZE and WRITE_SIZE of the kernel, and of the 1 GiB copy
    of --calibrate-copy, which scales each counter to bytes)."""
    copy_bytes = 1 << 30
    cf, _ = _counter_per_dispatch(copy_fetch_dir, "copyBuffer", "FETCH_SIZE")
    cw, _ = _counter_per_dispatch(copy_write_dir, "copyBuffer", "WRITE_SIZE")
    fetch_scale = copy_bytes / 1024.0 / cf
    write_scale = copy_bytes / 1024.0 / cw
    kf, nf = _counter_per_dispatch(fetch_dir, kernel, "FETCH_SIZE")
    kw, nw = _counter_per_dispatch(write_dir, kernel, "WRITE_SIZE")
    rec = {"kernel": kernel, "workload": workload, "kernel_src_digest": kernel_source_digest(kernel),
           "tiling": [int(v) for v in tiling.split(",")], "steps_per_launch": steps_per_launch,
           "fetch_kib_per_dispatch": round(kf, 1), "write_kib_per_dispatch": round(kw, 1),
           "dispatches": [nf, nw],
           "copy_fetch_kib": round(cf, 1), "copy_write_kib": round(cw, 1),
           "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
           "bytes_per_launch": int(round((kf * fetch_scale + kw * write_scale) * 1024))}
    out = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec), flush=True)


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 8) -> float:
    """Achievable HBM bandwidth on this machine: a plain device-to-device copy of
    nbytes (read nbytes + write nbytes per copy), best of `reps`, in GB/s."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        b.copy_(a)
        e.record()
        torch.cuda.synchronize()
        best = min(best, s.elapsed_time(e) / 1e3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * n * 4 / best / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="aco_1024x512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--autotune", action="store_true", help="autotune the batch launch shape first")
    ap.add_argument("--requests", type=int, default=512, help="requests in the served run")
    ap.add_argument("--rate", type=float, default=540.0,
                    help="request arrival rate (1/s); default 0.8 x the batched throughput "
                         "(9.1e9 agent-steps/s) over the mean request work (13.4M agent-steps)")
    ap.add_argument("--budget-gib", type=float, default=2.0, help="HBM budget for resident scenarios")
    ap.add_argument("--quantum", type=int, default=200, help="steps per serving quantum")
    ap.add_argument("--no-serve", action="store_true", help="skip the served run of the default line")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched run of the default line")
    ap.add_argument("--no-stress", action="store_true", help="skip the 4096x2048 run of the default line")
    ap.add_argument("--batched-steps", type=int, default=1000,
                    help="steps of the default line's batched run (the batched workload's own)")
    ap.add_argument("--tiling", default=None,
                    help="nw,rows,steps_per_launch,threads for the step kernel (default: the library's)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration for profiles)")
    ap.add_argument("--record-traffic", nargs=8,
                    metavar=("KERNEL", "WORKLOAD", "FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR",
                             "TILING", "STEPS_PER_LAUNCH"),
                    help="write profiles/traffic_<kernel>_<workload>.json from rocprofv3 --pmc runs "
                         "(no GPU work)")
    args = ap.parse_args()
    if args.record_traffic:
        k, w, fd, wd, cfd, cwd, tl, spl = args.record_traffic
        return record_traffic(k, w, fd, wd, cfd, cwd, tl, int(spl))
    if args.calibrate_copy:
        return calibrate_copy()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched_256":
        return run_batched(args)
    if args.workload == "served":
        summary = served_run(args.requests, args.rate, int(args.budget_gib * (1 << 30)), args.quantum)
        log("served:", summary)
        print(json.dumps({"metric": "batched p50/p99 scenario latency (served)", "value": summary["p99_latency_s"],
                          "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
                          "config": {"workload": WORKLOADS["served"][1]}, "served": summary}), flush=True)
        return

    import torch
    from paper_1412_4933_amd import pedsim

    # The served leg runs first: after the single-scenario timing (and its
    # streams) in the same process its latencies came out ~1.5-2x higher
    # than in a process of its own; first, they match.
    served = None
    if not args.no_serve:
        log(f"served run: {args.requests} requests at {args.rate}/s ...")
        served = served_run(args.requests, args.rate, int(args.budget_gib * (1 << 30)), args.quantum)
        log("served:", served)

    batched = None
    if not args.no_batched and args.workload == "aco_1024x512":
        log(f"batched run: 256 scenarios x {args.batched_steps} steps ...")
        batched = batched_run(args.batched_steps, min(args.warmup, 20))

    stress = None
    if not args.no_stress and not args.no_batched and args.workload == "aco_1024x512":
        log("4096x2048 ACO run ...")
        stress = stress_run()
        log("4096x2048:", stress)

    scn = make(args.workload)
    mode = scn.mode if args.workload != "stress_aco_4096x2048" else 1
    K = args.steps if args.steps is not None else scn.steps
    cells, agents = scn.W * scn.H, scn.agents
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)

    # warmup on a throwaway copy, then time K steps from the initial state
    log(f"workload {args.workload}: {scn.W}x{scn.H}, {agents} agents, mode {mode}, K={K}")
    tiling_arg = tuple(int(v) for v in args.tiling.split(",")) if args.tiling else None

    def make_sim():
        sim = pedsim.Sim(scn, stream=stream)
        if tiling_arg is not None:
            if getattr(scn, "ranges", None) is not None:  # cols,rows,steps,threads for the range kernel
                sim.set_range_tiling(*tiling_arg)
            else:
                sim.set_tiling(mode, *tiling_arg)
        return sim

    if args.warmup > 0:
        w = make_sim()
        w.step(args.warmup, mode)
        w.stats()
        w.close()
    sim = make_sim()
    torch.cuda.synchronize(dev)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(K, mode)
    end.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    stats = sim.stats()
    sim.close()
    sec = ms / 1e3
    value = agents * K / sec
    log(f"timed {K} steps: {ms:.3f} ms (wall {wall * 1e3:.3f} ms), stats {stats}")

    # the whole workload (all its steps from the initial state), beside the
    # K timed steps of the line
    full = None
    if K != scn.steps and scn.steps:
        fs = make_sim()
        torch.cuda.synchronize(dev)
        fa, fb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fa.record(stream)
        fs.step(scn.steps, mode)
        fb.record(stream)
        torch.cuda.synchronize(dev)
        fms = fa.elapsed_time(fb)
        fs.close()
        full = {"steps": scn.steps, "ms": fms, "ms_per_step": fms / scn.steps,
                "agent_steps_per_s": agents * scn.steps / (fms / 1e3)}
        log(f"full run: {scn.steps} steps in {fms:.3f} ms -> {full['agent_steps_per_s']:.4g} agent-steps/s")

    # per-launch durations of the step kernel with HIP events on the launch stream
    prof = make_sim()
    ranged = getattr(scn, "ranges", None) is not None
    if ranged:  # range kernel: one step per launch, tiles of cols x rows cells
        tiling = pedsim.sim_get_range_tiling(prof.h)  # (cols, rows, steps per launch, threads)
        tiling_source = ("--tiling" if tiling_arg is not None else "library default") + \
            " (range kernel: cols, rows, steps per launch, threads)"
    else:
        tiling = pedsim.sim_get_tiling(prof.h, mode)
        tiling_source = ("--tiling" if tiling_arg is not None
                         else "autotuner cache" if mode in prof.tuned else "library default")
    per_kernel = pedsim.sim_step_timed(prof.h, mode, K, stream)
    prof.close()
    log("tiling (nw, rows, steps/launch, threads):", tiling)
    log("per-kernel:", {k: (round(v[0], 3), v[1]) for k, v in per_kernel.items()})
    # The timed region above ran exactly these launches back to back on
    # `stream`: the step kernel's average duration is the region's event time
    # (minus the copy-back launches, if any) over its launch count.
    dom_n = per_kernel["tile_kernel"][1]
    dom = ("range_kernel" if ranged else
           "tile_rows_kernel" if tiling[0] in (0, 3) else "tile_kernel")  # kernel symbol in traces
    copy_ms = per_kernel["copy_back"][0]
    dom_avg_ms = (ms - copy_ms) / dom_n
    alg_step = algorithmic_bytes_per_step(mode, cells, agents)
    alg_launch = alg_step * K / dom_n
    achieved = alg_launch / (dom_avg_ms / 1e3) / 1e9
    traffic = measured_traffic(args.workload, dom, tiling)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "avg_launch_us": round(dom_avg_ms * 1e3, 3),
                "alg_bytes_per_launch": int(alg_launch),
                "steps_per_launch": tiling[2],
                "tiling": list(tiling),
                "isolated_launch_events": {k: {"avg_us": round(v[0] / v[1] * 1e3, 3) if v[1] else 0.0,
                                               "launches": v[1]} for k, v in per_kernel.items()}}
    if traffic is not None:
        roofline["traffic_gbs"] = round(traffic / (dom_avg_ms / 1e3) / 1e9, 1)
        roofline["traffic_frac"] = round(roofline["traffic_gbs"] / HBM_PEAK_GBS, 4)
    # the achievable bandwidth of a plain copy on this machine, beside the published peak
    roofline["copy_gbs"] = round(copy_bandwidth(), 1)


    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle ...")
        cpu = cpu_baseline(args.workload, args.cpu_budget)
        log(f"cpu oracle: {cpu['value']:.4g} agent-steps/s")

    line = {
        "metric": "agent-steps/s (ACO, 100K agents)" if args.workload == "aco_1024x512"
        else f"agent-steps/s ({args.workload})",
        "value": value, "unit": "agent-steps/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+u32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload][1], "grid": f"{scn.W}x{scn.H}",
                   "agents": agents, "mode": MODE_NAMES[mode], "seed": scn.seed,
                   "neighbours": getattr(scn, "neighbours", 5),
                   "ranges": list(scn.ranges) if getattr(scn, "ranges", None) else None,
                   "timed_steps": f"steps 0..{K - 1} of the workload's {scn.steps}, from its initial state",
                   "tiling": list(tiling), "tiling_source": tiling_source},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "full_run": full,
        "batched": batched,
        "served": served,
        "stress_4096x2048": stress,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
