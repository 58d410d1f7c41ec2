"""Helpers shared by the GPU tests (no method arithmetic here)."""

import sys

import numpy as np
import pytest

# elementwise bar, relative to the batch bar: max_i |a_i - ref_i| / rms(ref)
# may be at most this many times the tolerance on the batch-norm ratio
ELEMENT_FACTOR = 10.0


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg: str) -> None:
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def rel_err(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_2 / ||ref||_2 over the whole batch."""
    a = np.asarray(a).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def max_err_over_rms(a: np.ndarray, ref: np.ndarray) -> float:
    """max_i |a_i - ref_i| / rms(|ref|): one bad amplitude cannot hide in the
    batch norm."""
    a = np.asarray(a).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    return float(np.max(np.abs(a - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2)))


def assert_close(a, ref, tol: float, what: str = "") -> float:
    """Batch-norm ratio <= tol and every element within ELEMENT_FACTOR * tol
    of the rms amplitude; returns the batch-norm ratio."""
    e = rel_err(a, ref)
    m = max_err_over_rms(a, ref)
    assert e <= tol, f"{what} rel err {e:.3e} > {tol:.1e}"
    assert m <= ELEMENT_FACTOR * tol, f"{what} max |err| / rms {m:.3e} > {ELEMENT_FACTOR * tol:.1e}"
    return e


def bit_positions_to_index(positions, n_coords):
    """offset of every coordinate value: sum_t bit_t(x) << positions[t]."""
    x = np.arange(1 << len(positions), dtype=np.int64)
    off = np.zeros_like(x)
    for t, p in enumerate(positions):
        off |= ((x >> t) & 1) << p
    return off
