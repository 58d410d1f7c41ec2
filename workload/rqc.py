"""Seeded random quantum circuits on rectangular qubit grids.

Structure (Supplementary Information, Sec. I "Random quantum circuits"):
a circuit of depth d is d cycles, each a layer of single-qubit gates followed
by a layer of two-qubit gates; the single-qubit gates come from
{sqrt(X), sqrt(Y), sqrt(W)} and the two-qubit gate is fSim.  Two-qubit layers
follow four coupler patterns A, B, C, D such that each nearest-neighbour pair
gets exactly one gate in any four cycles that contain all four patterns; the
depth-8 sequence is ABCDCDAB and the depth-12 one ABCDCDABABCD.

Readings taken where the paper is silent (its figure of the patterns is not
available):
  * patterns on an R x C grid are staggered matchings of qubit (r, c):
    A = horizontal (r,c)-(r,c+1) with r+c even, B = horizontal with r+c odd,
    C = vertical (r,c)-(r+1,c) with r+c even, D = vertical with r+c odd;
    couplers touching a removed site are dropped;
  * the pattern of depth d is the first d letters of ABCDCDAB repeated, which
    gives back both printed sequences;
  * cycle 0 draws each single-qubit gate uniformly from the three; later
    cycles draw uniformly from the two gates that differ from the previous
    gate on that qubit ("no repeat on a qubit");
  * one more single-qubit layer follows the last two-qubit layer, before
    measurement;
  * qubit ids are row-major over the sites that are kept; bit q of a
    bitstring is the measured value of qubit q.

Nothing here computes a gate matrix: gates are names plus fSim angles.
"""

from __future__ import annotations

import json
import math
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

ONE_Q_RANDOM = ("sqrtX", "sqrtY", "sqrtW")
FSIM_THETA = math.pi / 2
FSIM_PHI = math.pi / 6
PATTERN_CYCLE = "ABCDCDAB"


@dataclass(frozen=True)
class GridSpec:
    rows: int
    cols: int
    removed: Tuple[Tuple[int, int], ...] = field(default_factory=tuple)


def grid_qubits(spec: GridSpec) -> Dict[Tuple[int, int], int]:
    """Row-major qubit ids over the kept sites of the grid."""
    removed = set(map(tuple, spec.removed))
    ids: Dict[Tuple[int, int], int] = {}
    for r in range(spec.rows):
        for c in range(spec.cols):
            if (r, c) not in removed:
                ids[(r, c)] = len(ids)
    return ids


def pattern_edges(spec: GridSpec, letter: str) -> List[Tuple[int, int]]:
    """Coupler list of pattern A/B/C/D as (qubit_a, qubit_b), qubit_a < qubit_b."""
    ids = grid_qubits(spec)
    horizontal = letter in "AB"
    parity = 0 if letter in "AC" else 1
    edges = []
    for (r, c), qa in ids.items():
        if (r + c) % 2 != parity:
            continue
        other = (r, c + 1) if horizontal else (r + 1, c)
        if other in ids:
            edges.append((qa, ids[other]))
    edges.sort()
    return edges


def pattern_sequence(depth: int) -> str:
    reps = depth // len(PATTERN_CYCLE) + 1
    return (PATTERN_CYCLE * reps)[:depth]


def _one_qubit_layers(rng: np.random.Generator, n: int, n_layers: int) -> List[List[str]]:
    layers: List[List[str]] = []
    prev = [None] * n
    for t in range(n_layers):
        layer = []
        for q in range(n):
            if prev[q] is None:
                g = ONE_Q_RANDOM[int(rng.integers(0, 3))]
            else:
                choices = [x for x in ONE_Q_RANDOM if x != prev[q]]
                g = choices[int(rng.integers(0, 2))]
            prev[q] = g
            layer.append(g)
        layers.append(layer)
    return layers


def _assemble(spec: GridSpec, depth: int, seed: int, one_q: List[List[str]],
              theta: float, phi: float, kind: str) -> dict:
    n = len(grid_qubits(spec))
    seq = pattern_sequence(depth)
    layers = []
    for t in range(depth):
        layers.append({"kind": "1q", "gates": [[q, one_q[t][q]] for q in range(n)]})
        layers.append({
            "kind": "2q",
            "pattern": seq[t],
            "gates": [[a, b, theta, phi] for a, b in pattern_edges(spec, seq[t])],
        })
    layers.append({"kind": "1q", "gates": [[q, one_q[depth][q]] for q in range(n)]})
    return {
        "format": "grid-rqc-v1",
        "kind": kind,
        "rows": spec.rows,
        "cols": spec.cols,
        "removed": [list(x) for x in spec.removed],
        "n_qubits": n,
        "depth": depth,
        "seed": seed,
        "layers": layers,
    }


def random_circuit(spec: GridSpec, depth: int, seed: int,
                   theta: float = FSIM_THETA, phi: float = FSIM_PHI) -> dict:
    """Seeded grid RQC: depth x (1q layer, 2q layer) + final 1q layer."""
    n = len(grid_qubits(spec))
    rng = np.random.default_rng(seed)
    one_q = _one_qubit_layers(rng, n, depth + 1)
    return _assemble(spec, depth, seed, one_q, theta, phi, "random")


def permutation_circuit(spec: GridSpec, depth: int, seed: int,
                        theta: float = FSIM_THETA, phi: float = FSIM_PHI) -> dict:
    """Same two-qubit structure as random_circuit, but the state before the final
    layer is a phased basis state: layer 0 applies X to a seeded subset of the
    qubits (identity elsewhere), the middle single-qubit layers are identity,
    and the last layer is a seeded choice of sqrt(X)/sqrt(Y)/sqrt(W).  With
    fSim(pi/2, phi) every two-qubit gate maps basis states to phased basis
    states, so every amplitude has modulus 2^(-n/2)."""
    n = len(grid_qubits(spec))
    rng = np.random.default_rng(seed)
    flips = rng.integers(0, 2, n)
    one_q = [["X" if flips[q] else "I" for q in range(n)]]
    for _ in range(1, depth):
        one_q.append(["I"] * n)
    last = [ONE_Q_RANDOM[int(x)] for x in rng.integers(0, 3, n)]
    if depth == 0:
        # a single layer: the flip is merged into nothing; keep the X layer out
        one_q = [last]
    else:
        one_q.append(last)
    return _assemble(spec, depth, seed, one_q, theta, phi, "permutation")


def product_circuit(spec: GridSpec, seed: int) -> dict:
    """Depth 0: one seeded single-qubit layer on |0...0>."""
    return random_circuit(spec, 0, seed)


def circuit_to_json(circ: dict) -> str:
    return json.dumps(circ, separators=(",", ":"))


def circuit_from_json(text: str) -> dict:
    circ = json.loads(text)
    if circ.get("format") != "grid-rqc-v1":
        raise ValueError("unknown circuit format")
    return circ


def count_two_qubit_gates(circ: dict) -> int:
    return sum(len(L["gates"]) for L in circ["layers"] if L["kind"] == "2q")


def edges_of_grid(spec: GridSpec) -> Sequence[Tuple[int, int]]:
    """All nearest-neighbour couplers of the grid (union of the four patterns)."""
    out = []
    for letter in "ABCD":
        out.extend(pattern_edges(spec, letter))
    return sorted(out)
