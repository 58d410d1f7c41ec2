"""Helpers shared by the GPU tests (no method arithmetic here)."""

import sys

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg: str) -> None:
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def rel_err(a: np.ndarray, ref: np.ndarray) -> float:
    a = np.asarray(a).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def bit_positions_to_index(positions, n_coords):
    """offset of every coordinate value: sum_t bit_t(x) << positions[t]."""
    x = np.arange(1 << len(positions), dtype=np.int64)
    off = np.zeros_like(x)
    for t, p in enumerate(positions):
        off |= ((x >> t) & 1) << p
    return off
