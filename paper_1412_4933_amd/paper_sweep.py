"""Population sweep of the paper's results section (Sec. VI) on one GPU.

For each density k (2,560 k agents on a 480 x 480 grid), `repeats` seeded
placements are run for 25,000 steps with the LEM rule and with the ACO rule,
all scenarios resident together in one batch, and the agents that reached the
opposite band are counted. The paper reports that both rules let nearly
everyone cross at low density, that ACO lets more agents cross at medium
density, and that both jam at high density; it quotes an overall gain of
39.6% for ACO over the first 20 densities. Its exact counts come from its own
random placements and generator, so only the qualitative shape can be
compared.

  python -m paper_1412_4933_amd.paper_sweep [--densities 1-20] [--repeats 10]
                                             [--steps 25000] [--neighbours 5|8]
                                             [--aco constant|tour] [--out FILE]

Prints one JSON document (per-density means, the overall ACO/LEM ratio and
the run's throughput).
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def parse_range(text: str):
    if "-" in text:
        a, b = text.split("-")
        return list(range(int(a), int(b) + 1))
    return [int(v) for v in text.split(",")]


def run(densities, repeats: int, steps: int, neighbours: int = 5, aco: str = "constant", log=print):
    import torch
    from . import pedsim
    from . import scenarios as S

    aco_mode = S.MODE_ACO_TOUR if aco == "tour" else S.MODE_ACO
    scns = S.paper_sweep(densities, repeats, steps, modes=(S.MODE_LEM, aco_mode), neighbours=neighbours)
    batch = pedsim.Batch(len(scns))
    if neighbours != 5:
        batch.set_neighbours(neighbours)
    elif aco_mode == S.MODE_ACO_TOUR:
        batch.set_tuning(0, 48, 3, 512, 2)  # the tour variant runs on the LDS form
    slots = []
    for s in scns:
        slots.append(batch.add(s))
    log(f"{len(scns)} scenarios resident; stepping {steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chunk = 1000
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        batch.step(n)
        torch.cuda.synchronize()
        done += n
        log(f"  {done}/{steps} steps, {time.perf_counter() - t0:.1f} s")
    wall = time.perf_counter() - t0
    rows = {}
    for s, slot in zip(scns, slots):
        st = batch.stats(slot)
        k = s.n_a // 1280
        r = rows.setdefault(k, {"k": k, "agents": s.agents, "band": s.band_a, "lem": [], "aco": []})
        r["lem" if s.mode == S.MODE_LEM else "aco"].append(st["crossed_a"] + st["crossed_b"])
    batch.close()
    table = []
    for k in sorted(rows):
        r = rows[k]
        table.append({"k": k, "agents": r["agents"], "band": r["band"],
                      "lem_crossed_mean": sum(r["lem"]) / max(1, len(r["lem"])),
                      "aco_crossed_mean": sum(r["aco"]) / max(1, len(r["aco"])),
                      "lem_crossed": r["lem"], "aco_crossed": r["aco"]})
    tot_lem = sum(t["lem_crossed_mean"] for t in table)
    tot_aco = sum(t["aco_crossed_mean"] for t in table)
    agent_steps = sum(s.agents for s in scns) * steps
    return {"grid": "480x480", "steps": steps, "repeats": repeats, "densities": list(densities),
            "neighbours": neighbours, "aco_deposit": aco,
            "table": table, "aco_over_lem": (tot_aco / tot_lem) if tot_lem else None,
            "wall_s": wall, "agent_steps_per_s": agent_steps / wall}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--densities", default="1-20")
    ap.add_argument("--repeats", type=int, default=10)
    ap.add_argument("--steps", type=int, default=25000)
    ap.add_argument("--neighbours", type=int, default=5, choices=(5, 8),
                    help="candidate set: 5 (no backward cells) or the paper's full 8")
    ap.add_argument("--aco", default="constant", choices=("constant", "tour"),
                    help="ACO deposit: constant dtau on occupied cells, or eq. 5's dtau / L_k "
                         "on entered cells (the tour variant)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    res = run(parse_range(args.densities), args.repeats, args.steps, args.neighbours, args.aco,
              log=lambda *a: print(*a, file=sys.stderr, flush=True))
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
