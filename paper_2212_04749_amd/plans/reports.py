"""Adds cost reports to the stored plans: for each workload (and each
circuit of the uneven batch) the figures of the stored, searched plan and of
the deterministic greedy order sliced to the same caps (S, S_k, the ideal
multi-amplitude speedup k S / S_k, total CMAC over all slices, slice count),
so that every reported number names how far the search moved from the
greedy order.

    python -m paper_2212_04749_amd.plans.reports [c3] [c4] [c5]
"""

from __future__ import annotations

import json
import os
import sys

from ..circuit_tn import build_network
from .. import planner

HERE = os.path.dirname(os.path.abspath(__file__))


def _annotate(e: dict, net, words, open_qubits=(), min_slices: int = 0) -> dict:
    # time estimates under the model the plan was searched with
    with planner.time_model(e.get("time_model", "c64")):
        stored = planner.plan_from(net, words, open_qubits, e["pairs"], e["sliced"], e.get("method", "stored"))
        e["report"] = planner.report(stored, words)
        try:
            g = planner.greedy_plan(net, words, open_qubits, e["cap"], min_slices=min_slices,
                                    mem_cap=e.get("mem_cap"))
            e["greedy_report"] = planner.report(g, words)
        except ValueError as err:  # the greedy order cannot meet the caps
            e["greedy_report"] = {"method": "greedy", "error": str(err)}
    return e


def annotate(name: str) -> None:
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from workload import CONFIGS
    from workload.configs import uneven_batch_c5
    if name in ("c3", "c4"):
        path = os.path.join(HERE, {"c3": "c3_cap30.json", "c4": "c4_cap32.json"}[name])
        e = json.load(open(path))
        w = CONFIGS[name.upper()]
        min_sl = (w.n_slices_target.bit_length() - 1) if w.n_slices_target else 0
        _annotate(e, build_network(w.circuit()), w.bitstrings(), w.open_qubits, min_sl)
        print(name, e["report"]["cmac_total"], e["greedy_report"].get("cmac_total"), flush=True)
    elif name == "c5":
        path = os.path.join(HERE, "c5_cap30.json")
        e = json.load(open(path))
        for w in uneven_batch_c5():
            _annotate(e[w.name], build_network(w.circuit()), w.bitstrings())
            print(w.name, e[w.name]["report"]["cmac_total"], e[w.name]["greedy_report"].get("cmac_total"),
                  flush=True)
    else:
        raise ValueError(name)
    with open(path, "w") as f:
        json.dump(e, f, separators=(",", ":"))


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c3", "c4", "c5"]:
        annotate(n)
