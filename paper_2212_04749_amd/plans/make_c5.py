"""Writes c5_cap30.json: contraction trees and sliced sets of the 32 uneven
circuits (workload.configs.uneven_batch_c5) at rank cap 30, found by the
planner with the time objective (8 greedy and 8 bisection candidates, 2
refined).  Planning all 32 takes about an hour on one host core, so the
uneven-batch runs load the
stored plans; any tree is valid input to the library (the contraction tree
is given, main text), and the file only saves the search.

    python -m paper_2212_04749_amd.plans.make_c5
"""

from __future__ import annotations

import json
import os

from ..circuit_tn import build_network
from .. import planner

CAP = 30
HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, f"c5_cap{CAP}.json")


def main() -> None:
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from workload.configs import uneven_batch_c5
    out = {}
    for w in uneven_batch_c5():
        net = build_network(w.circuit())
        pl = planner.find_plan(net, w.bitstrings(), (), CAP, trials=8, partition_trials=8, objective="time",
                               refine_top=2)
        out[w.name] = {"pairs": [list(p) for p in pl.pairs], "sliced": list(pl.sliced), "cap": CAP,
                       "est_seconds": pl.costs.time, "cmac_total": pl.costs.total}
        print(w.name, len(pl.sliced), f"{pl.costs.time:.2f}s", flush=True)
    with open(PATH, "w") as f:
        json.dump(out, f, separators=(",", ":"))


def load() -> dict:
    with open(PATH) as f:
        return json.load(f)


if __name__ == "__main__":
    main()
