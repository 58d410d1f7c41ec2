"""Gate matrices, complex128 (Supplementary Information, Sec. I).

The three single-qubit gates sqrt(X), sqrt(Y), sqrt(W) and the five-parameter
fSim gate are written out as the section gives them.  The angle parameters
Delta_+, Delta_-, Delta_-,off are taken as zero (the workloads only fix theta
and phi), which removes the duplicated phase of the two middle diagonal
entries.  fSim acts on |q_a q_b> with q_a the more significant bit of the
row/column index.  X and I are the Pauli X and identity, used by the
permutation circuits.
"""

from __future__ import annotations

import numpy as np

_S2 = np.sqrt(2.0) / 2.0


def sqrt_x() -> np.ndarray:
    return _S2 * np.array([[1.0, -1.0j], [-1.0j, 1.0]], dtype=np.complex128)


def sqrt_y() -> np.ndarray:
    return _S2 * np.array([[1.0, -1.0], [1.0, 1.0]], dtype=np.complex128)


def sqrt_w() -> np.ndarray:
    return _S2 * np.array([[1.0, -_S2 * (1.0 + 1.0j)],
                           [_S2 * (1.0 - 1.0j), 1.0]], dtype=np.complex128)


def pauli_x() -> np.ndarray:
    return np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)


def identity() -> np.ndarray:
    return np.eye(2, dtype=np.complex128)


def fsim(theta: float, phi: float, d_plus: float = 0.0, d_minus: float = 0.0,
         d_minus_off: float = 0.0) -> np.ndarray:
    """Five-parameter fSim on |q_a q_b>.  With all Deltas zero this is
    [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],[0,0,0,e^{-i phi}]]."""
    c, s = np.cos(theta), np.sin(theta)
    g = np.zeros((4, 4), dtype=np.complex128)
    g[0, 0] = 1.0
    g[1, 1] = np.exp(1j * (d_plus + d_minus)) * c
    g[1, 2] = -1j * np.exp(1j * (d_plus - d_minus_off)) * s
    g[2, 1] = -1j * np.exp(1j * (d_plus + d_minus_off)) * s
    # the printed matrix repeats the [1,1] phase here; with zero Deltas the two
    # readings coincide
    g[2, 2] = np.exp(1j * (d_plus + d_minus)) * c
    g[3, 3] = np.exp(1j * (2.0 * d_plus - phi))
    return g


ONE_QUBIT = {
    "sqrtX": sqrt_x,
    "sqrtY": sqrt_y,
    "sqrtW": sqrt_w,
    "X": pauli_x,
    "I": identity,
}


def one_qubit(name: str) -> np.ndarray:
    try:
        return ONE_QUBIT[name]()
    except KeyError:
        raise ValueError(f"unknown single-qubit gate {name!r}") from None
