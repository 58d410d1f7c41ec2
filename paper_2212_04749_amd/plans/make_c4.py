"""Writes c4_cap32.json: a contraction tree and sliced set for the 53-qubit
workload (6x9 grid minus one corner, depth 14, 1024 bitstrings) at rank cap
32 and at most 2^33 elements per multi-amplitude tensor, with at least 9
sliced indices so that one slice is a unit of work that can be timed on its
own (the per-slice time of complex64 against complex-half).  Found by the
planner with the time objective under the complex-half time model (the
workload's headline precision) from bisection candidates, the only family
that reaches a total cost near 10^16-10^17 CMAC here (the greedy families
stay above 10^21).  The result depends strongly on the seed: of seeds 0-35,
seed 7 reached 2.07e16 CMAC over 2^12 slices and every other seed stayed
between 8.4e16 and 1.1e20; seed 7's plan is the stored one.  One seed takes
a few minutes of host time, so the bench loads the stored plan; any tree is
valid input to the library.

    python -m paper_2212_04749_amd.plans.make_c4 [--seeds 7,8,...] [--jobs N]
"""

from __future__ import annotations

import json
import os

from ..circuit_tn import build_network
from .. import planner

CAP = 32
MEM_CAP = 33
MIN_SLICED = 9
HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, f"c4_cap{CAP}.json")


def _plan_seed(seed: int):
    from workload import CONFIGS
    w = CONFIGS["C4"]
    net = build_network(w.circuit())
    with planner.time_model("chalf"):
        pl = planner.find_plan(net, w.bitstrings(), (), CAP, seed=seed, trials=0, include_greedy=False,
                               partition_trials=8, refine_top=2, min_slices=MIN_SLICED, max_sliced=60,
                               objective="time", mem_cap=MEM_CAP)
    return seed, pl


def main() -> None:
    import argparse
    import sys
    from multiprocessing import Pool
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", default="7")
    ap.add_argument("--jobs", type=int, default=max(1, min(6, os.cpu_count() or 1)))
    args = ap.parse_args()
    seeds = [int(x) for x in args.seeds.split(",")]
    best = None
    with Pool(min(args.jobs, len(seeds))) as pool:
        for seed, pl in pool.imap_unordered(_plan_seed, seeds):
            print(seed, len(pl.sliced), f"{pl.costs.total:.3e} CMAC", f"{pl.costs.time:.0f} s", pl.method, flush=True)
            if best is None or pl.costs.time < best.costs.time:
                best = pl
    out = {"pairs": [list(p) for p in best.pairs], "sliced": list(best.sliced), "cap": CAP, "mem_cap": MEM_CAP,
           "est_seconds": best.costs.time, "cmac_total": best.costs.total, "method": best.method,
           "time_model": "chalf"}
    with open(PATH, "w") as f:
        json.dump(out, f, separators=(",", ":"))


def load() -> dict:
    with open(PATH) as f:
        return json.load(f)


if __name__ == "__main__":
    main()
