"""Seeded bitstring batches.  Bit q of a packed uint64 is the value of qubit q."""

from __future__ import annotations

import numpy as np


def uniform_bitstrings(n_qubits: int, k: int, seed: int) -> np.ndarray:
    """k uniform-random bitstrings over n qubits, packed as uint64 (bit q = qubit q).

    Drawn as ``default_rng(seed).integers(0, 2, (k, n))`` so that every reader
    of the same seed sees the same batch.  Duplicates are kept."""
    if not 0 < n_qubits <= 64:
        raise ValueError("n_qubits must be in 1..64")
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, (k, n_qubits))
    return bits_to_u64(bits)


def bits_to_u64(bits: np.ndarray) -> np.ndarray:
    bits = np.asarray(bits, dtype=np.uint64)
    if bits.ndim != 2:
        raise ValueError("bits must be (k, n)")
    weights = np.left_shift(np.uint64(1), np.arange(bits.shape[1], dtype=np.uint64))
    return (bits * weights[None, :]).sum(axis=1, dtype=np.uint64)


def u64_to_bits(words: np.ndarray, n_qubits: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint64)
    shifts = np.arange(n_qubits, dtype=np.uint64)
    return ((words[:, None] >> shifts[None, :]) & np.uint64(1)).astype(np.int64)


def subset(words: np.ndarray, m: int, seed: int) -> np.ndarray:
    """A seeded subset of m positions (sorted) of a batch, for oracle checks."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(words), size=min(m, len(words)), replace=False))
    return idx


def sample_mixture(probs: np.ndarray, k: int, fidelity: float, seed: int) -> np.ndarray:
    """k bitstrings (packed uint64, bit q = qubit q) from the mixture that
    draws each one, independently, from the distribution ``probs`` (indexed
    by the packed bitstring) with probability ``fidelity`` and uniformly
    otherwise -- the model of a noisy device's samples behind Eq. (2)."""
    probs = np.asarray(probs, dtype=np.float64).reshape(-1)
    size = probs.size
    if size & (size - 1) or not 0.0 <= fidelity <= 1.0:
        raise ValueError("probs must have 2^n entries and fidelity must be in [0, 1]")
    rng = np.random.default_rng(seed)
    from_p = rng.random(k) < fidelity
    out = rng.integers(0, size, size=k, dtype=np.uint64)
    n_p = int(from_p.sum())
    if n_p:
        out[from_p] = rng.choice(size, size=n_p, p=probs / probs.sum()).astype(np.uint64)
    return out
