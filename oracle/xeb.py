"""Linear cross-entropy benchmarking fidelity, in float64.

Eq. (2) models the distribution of x = N p (N = 2^n, p the ideal probability
of a measured bitstring) as (F x + 1 - F) e^{-x}.  Its mean is
integral x (F x + 1 - F) e^{-x} dx = 2F + (1 - F) = 1 + F, so the estimate of
F from a batch of k bitstrings is F = (N / k) sum_i |a_i|^2 - 1.
"""

from __future__ import annotations

import numpy as np


def linear_xeb(amps: np.ndarray, n_qubits: int) -> float:
    a = np.asarray(amps, dtype=np.complex128).reshape(-1)
    if a.size == 0:
        raise ValueError("oracle xeb: empty batch")
    p = a.real * a.real + a.imag * a.imag
    return float(np.ldexp(np.sum(p) / a.size, n_qubits) - 1.0)
