"""Dense state-vector simulation in complex128 (the plain definition of an amplitude).

psi = U_last ... U_1 |0...0>, and the amplitude of bitstring b is <b|psi>
(Supplementary Information, Sec. II).  The state is an n-axis array with axis
q holding qubit q, so psi[b_0, ..., b_{n-1}] is the amplitude of b.
Each gate is applied with numpy.tensordot over the axes it acts on.
Memory is 16 * 2^n bytes: n <= 30.
"""

from __future__ import annotations

import numpy as np

from .circuit import gate_list, words_to_bits


def final_state(circ: dict) -> np.ndarray:
    n, glist = gate_list(circ)
    if n > 30:
        raise ValueError("oracle state vector: n > 30 does not fit")
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for qubits, mat in glist:
        if len(qubits) == 1:
            (q,) = qubits
            # new[o, ...] = sum_i U[o, i] psi[..., i at axis q, ...]
            psi = np.moveaxis(np.tensordot(mat, psi, axes=([1], [q])), 0, q)
        else:
            qa, qb = qubits
            g = mat.reshape(2, 2, 2, 2)  # [out_a, out_b, in_a, in_b]
            psi = np.moveaxis(np.tensordot(g, psi, axes=([2, 3], [qa, qb])), [0, 1], [qa, qb])
    return psi


def amplitudes_from_state(psi: np.ndarray, words) -> np.ndarray:
    n = psi.ndim
    bits = words_to_bits(words, n)
    return psi[tuple(bits[:, q] for q in range(n))]


def amplitudes(circ: dict, words) -> np.ndarray:
    return amplitudes_from_state(final_state(circ), words)


def probabilities(circ: dict) -> np.ndarray:
    """|<b|psi>|^2 for every bitstring b, indexed by the packed word
    (bit q = qubit q, so qubit n-1 is the most significant)."""
    psi = final_state(circ)
    n = psi.ndim
    flat = np.transpose(psi, tuple(range(n - 1, -1, -1))).reshape(-1)
    return (flat.real * flat.real + flat.imag * flat.imag).astype(np.float64)
