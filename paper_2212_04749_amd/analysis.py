"""Fidelity analysis of a batch of amplitudes (main text Eq. (2), Fig. 4).

For a bitstring b sampled by a device of fidelity F, x = 2^n |<b|psi>|^2
follows (F x + 1 - F) e^{-x} (Porter-Thomas for F = 0, its x-weighted form
for F = 1).  Two estimates of F from the amplitudes of k sampled bitstrings:

* linear XEB: the mean of x is 1 + F, so F = <x> - 1 (the library's
  matnc_xeb computes the same sum on the GPU in FP64);
* maximum likelihood: F maximises sum_i log(F x_i + 1 - F) over [0, 1];
  that function is concave in F, and its maximiser is found here by Newton's
  method on the derivative, kept inside [0, 1].

The histogram of x against the density at the fitted F is the data of
Fig. 4.  Host-side post-processing of the library's output; the amplitudes
themselves come from the GPU.
"""

from __future__ import annotations

import numpy as np


def x_values(amps, n_qubits: int) -> np.ndarray:
    a = np.asarray(amps, dtype=np.complex128).reshape(-1)
    return np.ldexp(a.real * a.real + a.imag * a.imag, n_qubits)


def linear_fidelity(x) -> float:
    return float(np.mean(np.asarray(x, dtype=np.float64)) - 1.0)


def fit_fidelity(x, tol: float = 1e-13, max_iter: int = 100) -> float:
    """Maximum-likelihood F in [0, 1] under Eq. (2)."""
    y = np.asarray(x, dtype=np.float64).reshape(-1) - 1.0
    if y.size == 0:
        raise ValueError("empty batch")

    def d1(f):
        return float(np.sum(y / (1.0 + f * y)))

    if d1(0.0) <= 0.0:
        return 0.0
    if d1(1.0) >= 0.0:
        return 1.0
    # the derivative falls monotonically from > 0 at 0 to < 0 at 1; Newton
    # steps from the linear estimate, with a bracket as a guard
    lo, hi = 0.0, 1.0
    f = min(max(float(np.mean(y)), 0.0), 1.0)
    for _ in range(max_iter):
        g = d1(f)
        if g > 0.0:
            lo = f
        else:
            hi = f
        h = -float(np.sum((y / (1.0 + f * y)) ** 2))
        step = -g / h if h < 0.0 else 0.0
        nf = f + step
        if not lo < nf < hi:
            nf = 0.5 * (lo + hi)
        if abs(nf - f) <= tol:
            return nf
        f = nf
    return f


def porter_thomas_histogram(x, fidelity: float, bins: int = 40, x_max: float = 8.0) -> dict:
    """Normalised histogram of x on [0, x_max) and Eq. (2)'s density at the
    bin centres for the given F."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    edges = np.linspace(0.0, x_max, bins + 1)
    counts, _ = np.histogram(x, bins=edges)
    width = edges[1] - edges[0]
    centres = 0.5 * (edges[1:] + edges[:-1])
    return {"edges": edges.tolist(), "density": (counts / (x.size * width)).tolist(),
            "model": ((fidelity * centres + 1.0 - fidelity) * np.exp(-centres)).tolist(),
            "fidelity": fidelity, "samples": int(x.size), "beyond_range": int(np.sum(x >= x_max))}
