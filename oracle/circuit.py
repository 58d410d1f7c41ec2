"""Reading of the grid-rqc-v1 circuit description into a flat gate list.

A circuit is a time-ordered list of layers; a single-qubit layer lists
(qubit, gate name) and a two-qubit layer lists (qubit_a, qubit_b, theta, phi)
for fSim.  Qubit q is bit q of a bitstring.
"""

from __future__ import annotations

from typing import List, Tuple, Union

import numpy as np

from . import gates

# (qubits, matrix): a 2x2 matrix on (q,) or a 4x4 matrix on (q_a, q_b)
Gate = Tuple[Tuple[int, ...], np.ndarray]


def gate_list(circ: dict) -> Tuple[int, List[Gate]]:
    if circ.get("format") != "grid-rqc-v1":
        raise ValueError("oracle: unknown circuit format")
    n = int(circ["n_qubits"])
    out: List[Gate] = []
    for layer in circ["layers"]:
        if layer["kind"] == "1q":
            for q, name in layer["gates"]:
                if not 0 <= q < n:
                    raise ValueError("oracle: qubit out of range")
                out.append(((int(q),), gates.one_qubit(name)))
        elif layer["kind"] == "2q":
            for qa, qb, theta, phi in layer["gates"]:
                if qa == qb or not (0 <= qa < n and 0 <= qb < n):
                    raise ValueError("oracle: bad two-qubit gate")
                out.append(((int(qa), int(qb)), gates.fsim(float(theta), float(phi))))
        else:
            raise ValueError(f"oracle: unknown layer kind {layer['kind']!r}")
    return n, out


def words_to_bits(words: Union[np.ndarray, list], n: int) -> np.ndarray:
    """uint64 words (bit q = qubit q) to an int array of shape (k, n)."""
    w = np.asarray(words, dtype=np.uint64).reshape(-1)
    return np.array([[(int(x) >> q) & 1 for q in range(n)] for x in w], dtype=np.int64).reshape(len(w), n)
