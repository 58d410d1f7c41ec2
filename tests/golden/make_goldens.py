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
  c5_sv.json       the circuits of the seeded uneven batch with 26..30 qubits
                   (six of the 32): all bitstrings of each circuit's batch
  c1_all.json      4x4 grid, depth 8: all 64 bitstrings of its batch
  pt_samples.json  4x5 grid, depth 12 (seed 4501): bitstrings sampled from
                   the mixture of its exact output distribution (weight F)
                   and the uniform one, for F = 1 and F = 0.2, with the exact
                   x = 2^n |<b|psi>|^2 of each (the fidelity workload)
  c3_permutation.json
                   the permutation circuit (seed 303) on the 6x6 depth-14
                   grid of the batching workload: exact amplitudes
                   (oracle.closed_forms) of every open-leg entry of a seeded
                   subset of 4 of its 64 bitstring groups
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

from oracle import closed_forms, statevector, sv_native  # noqa: E402
from workload import CONFIGS, GridSpec, permutation_circuit, random_circuit, sample_mixture, sub_instance_c4  # noqa: E402
from workload.configs import uneven_batch_c5  # noqa: E402
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


def c5_sv():
    out = {
        "what": "FP64 state-vector amplitudes (oracle.sv_native) of every uneven-batch circuit with 26..30 "
                "qubits, for all bitstrings of its batch",
        "source": "Supplementary Information Sec. II; workload.configs uneven_batch_c5 (master seed 5)",
        "circuits": {},
    }
    for w in uneven_batch_c5():
        if not 26 <= w.n_qubits <= 30:
            continue
        words = w.bitstrings()
        t = time.time()
        amps = sv_native.amplitudes(w.circuit(), words)
        print(f"{w.name}: {w.n_qubits} qubits, depth {w.depth}, {len(words)} bitstrings, "
              f"{time.time() - t:.1f} s", flush=True)
        out["circuits"][w.name] = {
            "n_qubits": w.n_qubits, "depth": w.depth,
            "words": [str(int(x)) for x in words],
            "amps": [[float(a.real), float(a.imag)] for a in amps],
        }
    write("c5_sv.json", out)


def c1_all():
    w = CONFIGS["C1"]
    words = w.bitstrings()
    amps = sv_native.amplitudes(w.circuit(), words)
    write("c1_all.json", {
        "what": "FP64 state-vector amplitudes (oracle.sv_native) of the 4x4 depth-8 circuit (circuit seed 1) "
                "for its 64 uniform bitstrings (seed 1001)",
        "source": "Supplementary Information Sec. II; workload.configs C1",
        "words": [str(int(x)) for x in words],
        "amps": [[float(a.real), float(a.imag)] for a in amps],
    })


PERM_SEED_C3 = 303
GROUP_SUBSET_SEED_C3 = 2303


def c3_permutation():
    w = CONFIGS["C3"]
    circ = permutation_circuit(w.grid, w.depth, PERM_SEED_C3)
    groups = w.bitstrings()
    gidx = subset(groups, 4, GROUP_SUBSET_SEED_C3)
    opens = list(w.open_qubits)
    words = []
    for g in groups[gidx]:
        for j in range(1 << len(opens)):
            word = int(g)
            for t, q in enumerate(opens):
                word |= ((j >> t) & 1) << q
            words.append(word)
    amps = closed_forms.permutation_amplitudes(circ, np.array(words, dtype=np.uint64))
    write("c3_permutation.json", {
        "what": "exact amplitudes (oracle.closed_forms) of the permutation circuit of the 6x6 depth-14 grid "
                f"(permutation seed {PERM_SEED_C3}) for every open-leg entry (qubits 28..35; entry j sets the "
                "t-th open qubit to bit t of j) of 4 of the 64 bitstring groups of the batching workload",
        "source": "Supplementary Information Sec. II (amplitude); a permutation circuit keeps one basis "
                  "state up to a phase until its last single-qubit layer",
        "permutation_seed": PERM_SEED_C3,
        "group_subset_seed": GROUP_SUBSET_SEED_C3,
        "groups": [int(i) for i in gidx],
        "amps": [[float(a.real), float(a.imag)] for a in amps],
    })


PT_CIRCUIT_SEED = 4501
PT_K = 4096


def pt_samples():
    circ = random_circuit(GridSpec(4, 5), 12, PT_CIRCUIT_SEED)
    p = statevector.probabilities(circ)
    out = {
        "what": "bitstrings sampled from the mixture of the exact output distribution (weight F) and the uniform "
                "one, for the 4x5 depth-12 circuit (seed 4501), with x = 2^n p(b) of each from the oracle's "
                "state vector",
        "source": "main text Eq. (2) (density of x for samples of fidelity F) and Fig. 4",
        "grid": [4, 5], "depth": 12, "circuit_seed": PT_CIRCUIT_SEED, "n_qubits": 20,
        "ideal_linear_xeb": float(np.ldexp(np.sum(p * p), 20) - 1.0),
        "sets": [],
    }
    for f, seed in ((1.0, 4602), (0.2, 4622)):
        words = sample_mixture(p, PT_K, f, seed)
        out["sets"].append({"fidelity": f, "sample_seed": seed, "words": [str(int(x)) for x in words],
                            "x": [float(v) for v in np.ldexp(p[words.astype(np.int64)], 20)]})
    write("pt_samples.json", out)


JOBS = {"c2_subset": c2_subset, "c4_sub": c4_sub, "c5_sv": c5_sv, "c1_all": c1_all,
        "c3_permutation": c3_permutation, "pt_samples": pt_samples}

if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for n in names:
        JOBS[n]()
