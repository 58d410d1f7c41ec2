"""Circuit -> fused tensor network (host side of the library).

Mapping (Supplementary Information, Sec. II): |0> is a rank-1 tensor, a
single-qubit gate rank 2 and a two-qubit gate rank 4; the rank-1 and rank-2
tensors are absorbed into the rank-4 ones ("gate fusion"), leaving one tensor
per fSim gate.  The output index of each qubit is its last wire; fixing it to
b_q selects an amplitude, leaving it open gives correlated amplitudes.

Fusion rule used here: the single-qubit gates on a wire between two fSim
gates, and the |0> at the start of a wire, are absorbed into the input leg of
the next fSim on that qubit; the single-qubit gates after the last fSim on a
qubit are absorbed into that fSim's output leg.  A qubit that no fSim touches
becomes a rank-1 tensor holding only its output index.

The gate matrices are transcribed here from Sec. I independently of any other
copy in the repository (Delta parameters zero; fSim on |q_a q_b> with q_a the
more significant bit).

Tensor data layout handed to the library: complex128, row-major over the
tensor's index list, first index most significant.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_H = 1.0 / math.sqrt(2.0)

# single-qubit gates [row = output, column = input]
_ONE_Q = {
    "sqrtX": _H * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128),
    "sqrtY": _H * np.array([[1, -1], [1, 1]], dtype=np.complex128),
    "sqrtW": _H * np.array([[1, -_H * (1 + 1j)], [_H * (1 - 1j), 1]], dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "I": np.array([[1, 0], [0, 1]], dtype=np.complex128),
}


def one_qubit_matrix(name: str) -> np.ndarray:
    if name not in _ONE_Q:
        raise ValueError(f"unknown single-qubit gate {name!r}")
    return _ONE_Q[name].copy()


def fsim_matrix(theta: float, phi: float) -> np.ndarray:
    """fSim(theta, phi) with zero Delta parameters, basis |q_a q_b>."""
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1.0
    m[1, 1] = m[2, 2] = math.cos(theta)
    m[1, 2] = m[2, 1] = -1j * math.sin(theta)
    m[3, 3] = complex(math.cos(phi), -math.sin(phi))
    return m


@dataclass
class TensorNetwork:
    """Fused network.  Index ids are ints; every index has dimension 2."""
    n_qubits: int
    tensors: List[np.ndarray]            # complex128, shape (2,)*rank
    indices: List[Tuple[int, ...]]       # axis ids of each tensor
    output_index: List[int]              # output index id of each qubit
    n_index: int

    @property
    def n_tensors(self) -> int:
        return len(self.tensors)

    def ranks(self) -> List[int]:
        return [len(ix) for ix in self.indices]


def build_network(circ: dict) -> TensorNetwork:
    if circ.get("format") != "grid-rqc-v1":
        raise ValueError("unknown circuit format")
    n = int(circ["n_qubits"])
    # pending[q]: 2x2 operator accumulated on qubit q since its last fSim
    # (starting from the |0> state, kept as a 2x1 column while no fSim has come)
    pending: List[np.ndarray] = [np.array([[1.0], [0.0]], dtype=np.complex128) for _ in range(n)]
    has_gate = [False] * n
    wire: List[Optional[int]] = [None] * n   # current index id of each qubit's wire
    last_fsim: List[Optional[int]] = [None] * n  # tensor holding the wire as output
    tensors: List[np.ndarray] = []
    indices: List[Tuple[int, ...]] = []
    next_id = 0

    for layer in circ["layers"]:
        if layer["kind"] == "1q":
            for q, name in layer["gates"]:
                pending[q] = one_qubit_matrix(name) @ pending[q]
        elif layer["kind"] == "2q":
            for qa, qb, theta, phi in layer["gates"]:
                g = fsim_matrix(float(theta), float(phi)).reshape(2, 2, 2, 2)  # [oa, ob, ia, ib]
                legs: List[int] = []
                # absorb the pending operators into the input legs
                for pos, q in ((2, qa), (3, qb)):
                    g = np.moveaxis(np.tensordot(g, pending[q], axes=([pos], [0])), -1, pos)
                # g now [oa, ob, ia', ib'] where ia' is the previous wire (dim 2) or
                # the collapsed |0> start (dim 1)
                oa, ob = next_id, next_id + 1
                next_id += 2
                shape = [2, 2]
                legs = [oa, ob]
                for q in (qa, qb):
                    if has_gate[q]:
                        legs.append(wire[q])
                        shape.append(2)
                    else:
                        shape.append(1)
                g = g.reshape(2, 2, *[s for s in shape[2:]])
                squeeze = tuple(i for i, s in enumerate(g.shape) if s == 1)
                g = np.squeeze(g, axis=squeeze) if squeeze else g
                t = len(tensors)
                tensors.append(np.ascontiguousarray(g))
                indices.append(tuple(legs))
                for q, new in ((qa, oa), (qb, ob)):
                    wire[q] = new
                    has_gate[q] = True
                    last_fsim[q] = t
                    pending[q] = np.eye(2, dtype=np.complex128)
        else:
            raise ValueError(f"unknown layer kind {layer['kind']!r}")

    output_index = [0] * n
    for q in range(n):
        if has_gate[q]:
            t = last_fsim[q]
            pos = indices[t].index(wire[q])
            tensors[t] = np.ascontiguousarray(
                np.moveaxis(np.tensordot(pending[q], tensors[t], axes=([1], [pos])), 0, pos))
            output_index[q] = wire[q]
        else:
            vec = pending[q][:, 0]
            tensors.append(np.ascontiguousarray(vec))
            indices.append((next_id,))
            output_index[q] = next_id
            next_id += 1
    return TensorNetwork(n, tensors, indices, output_index, next_id)
