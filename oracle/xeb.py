"""Linear cross-entropy benchmarking fidelity, in float64.

Eq. (2) models the distribution of x = N p (N = 2^n, p the ideal probability
of a measured bitstring) as (F x + 1 - F) e^{-x}.  Its mean is
integral x (F x + 1 - F) e^{-x} dx = 2F + (1 - F) = 1 + F, so the estimate of
F from a batch of k bitstrings is F = (N / k) sum_i |a_i|^2 - 1.

The maximum-likelihood estimate of F under the same density maximises
L(F) = sum_i log(F x_i + 1 - F) (the factor e^{-x} does not depend on F) over
[0, 1]; L is concave, so the maximiser is the root of
L'(F) = sum_i (x_i - 1) / (F (x_i - 1) + 1), or an end of the interval.
Here it is found by bisection on L'.

This module is test infrastructure (the oracle): only the tests, the smoke
check and the bench's CPU baseline use it.
"""

from __future__ import annotations

import numpy as np


def linear_xeb(amps: np.ndarray, n_qubits: int) -> float:
    a = np.asarray(amps, dtype=np.complex128).reshape(-1)
    if a.size == 0:
        raise ValueError("oracle xeb: empty batch")
    p = a.real * a.real + a.imag * a.imag
    return float(np.ldexp(np.sum(p) / a.size, n_qubits) - 1.0)


def porter_thomas_density(x, fidelity: float) -> np.ndarray:
    """Eq. (2): the density of x = N p for samples of fidelity F."""
    x = np.asarray(x, dtype=np.float64)
    return (fidelity * x + 1.0 - fidelity) * np.exp(-x)


def mle_fidelity(x, iterations: int = 200) -> float:
    """Maximum-likelihood F in [0, 1] of the samples x = N p under Eq. (2),
    by bisection on the derivative of the log-likelihood."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    if x.size == 0:
        raise ValueError("oracle mle: empty batch")

    def slope(f: float) -> float:
        return float(np.sum((x - 1.0) / (f * (x - 1.0) + 1.0)))

    if slope(0.0) <= 0.0:
        return 0.0
    if slope(1.0) >= 0.0:
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(iterations):
        mid = 0.5 * (lo + hi)
        if slope(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
