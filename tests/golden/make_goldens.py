"""Write the stored reference amplitudes of tests/golden/ (calls only oracle/).

Every value here is the FP64 state-vector amplitude <b|psi> of a seeded
workload circuit (Supplementary Information, Sec. II), computed by
oracle.sv_native, the plain-C dense simulation of the oracle, which is
itself pinned against the numpy state vector and brute force.

    python tests/golden/make_goldens.py [name ...]

Outputs (JSON text, amplitudes as [re, im] pairs):
  c2_subset.json   5x6 grid, depth 12: a seeded 256-bitstring subset of the
                   4096-bitstring batch
  c4_sub.json      4x5 grid, depth 14 (the 20-qubit error instance): all 1024
                   bitstrings of its batch
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import sv_native  # noqa: E402
from workload import CONFIGS, sub_instance_c4  # noqa: E402
from workload.bitstrings import subset  # noqa: E402

SUBSET_SEED_C2 = 2256


def write(name: str, payload: dict) -> None:
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(payload, f, indent=0)
    print("wrote", path, flush=True)


def c2_subset():
    w = CONFIGS["C2"]
    circ, words = w.circuit(), w.bitstrings()
    idx = subset(words, 256, SUBSET_SEED_C2)
    t = time.time()
    amps = sv_native.amplitudes(circ, words[idx])
    write("c2_subset.json", {
        "what": "FP64 state-vector amplitudes <b|psi> (oracle.sv_native) of the 5x6 depth-12 circuit "
                "(circuit seed 2) for a 256-bitstring subset of its 4096 uniform bitstrings (seed 1002)",
        "source": "Supplementary Information Sec. II (amplitude = <b|psi>); workload.configs C2",
        "subset_seed": SUBSET_SEED_C2,
        "indices": [int(i) for i in idx],
        "words": [str(int(x)) for x in words[idx]],
        "amps": [[float(a.real), float(a.imag)] for a in amps],
        "oracle_seconds": time.time() - t,
    })


def c4_sub():
    w = sub_instance_c4()
    circ, words = w.circuit(), w.bitstrings()
    amps = sv_native.amplitudes(circ, words)
    write("c4_sub.json", {
        "what": "FP64 state-vector amplitudes of the 4x5 depth-14 sub-instance (circuit seed 40) for its "
                "1024 uniform bitstrings (seed 1040)",
        "source": "Supplementary Information Sec. II; workload.configs sub_instance_c4",
        "words": [str(int(x)) for x in words],
        "amps": [[float(a.real), float(a.imag)] for a in amps],
    })


JOBS = {"c2_subset": c2_subset, "c4_sub": c4_sub}

if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for n in names:
        JOBS[n]()
