"""Writes c2_cap28.json: the contraction tree and sliced set of the 5x6
depth-12 workload (4096 uniform bitstrings, rank cap 28), found by the
planner with the time objective from the deterministic greedy order and 32
greedy-family candidates (seed 0), refined by subtree reconfiguration; with
the cost figures of that plan and of the plain greedy order sliced to the
same cap, for comparison.  The search takes about 20 s of host time, so the
bench loads the stored plan; any tree is valid input to the library.

    python -m paper_2212_04749_amd.plans.make_c2
"""

from __future__ import annotations

import json
import os

from ..circuit_tn import build_network
from .. import planner

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "c2_cap28.json")


def main() -> None:
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from workload import CONFIGS
    w = CONFIGS["C2"]
    net = build_network(w.circuit())
    words = w.bitstrings()
    pl = planner.find_plan(net, words, (), w.cap, seed=0, trials=32, objective="time",
                           progress=lambda m: print(m, flush=True))
    greedy = planner.greedy_plan(net, words, (), w.cap)
    out = {"pairs": [list(p) for p in pl.pairs], "sliced": list(pl.sliced), "cap": w.cap,
           "est_seconds": pl.costs.time, "cmac_total": pl.costs.total, "method": pl.method,
           "report": planner.report(pl, words), "greedy_report": planner.report(greedy, words)}
    with open(PATH, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(len(pl.sliced), f"{pl.costs.total:.3e} CMAC", f"{pl.costs.time:.3f} s", pl.method,
          f"greedy {greedy.costs.total:.3e} CMAC")


def load() -> dict:
    with open(PATH) as f:
        return json.load(f)


if __name__ == "__main__":
    main()
