"""The five workloads, with their seeds.

C1  4x4 grid, depth 8, no slicing, 64 bitstrings (complex128 check against the
    full state vector).
C2  5x6 grid, depth 12, rank cap 28, 4096 bitstrings (complex64), oracle on a
    256-bitstring subset.
C3  6x6 grid, depth 14, rank cap 30 with 2^8 slices, 2^14 amplitudes as 8 open
    output legs (qubits 28..35) x 64 seeded assignments of qubits 0..27.
C4  53 qubits (6x9 grid without site (5,8)), depth 14, rank cap 32; 64 seeded
    slice ids timed with 1024 bitstrings; error measured on a 4x5, depth-14
    sub-instance sliced to 64 slices.
C5  32 seeded circuits of 20..36 qubits, depth 10..16, 256..4096 bitstrings
    each, rank cap 28.

Seeds: circuit seed of C1..C4 is 1..4, bitstring seed is 1000 + circuit seed;
the C4 slice subset uses seed 2004; C5 uses master seed 5 and circuit seed
500 + i (bitstrings 1500 + i); the C4 sub-instance uses circuit seed 40 and
bitstring seed 1040.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from .rqc import GridSpec, random_circuit
from .bitstrings import uniform_bitstrings


@dataclass
class Workload:
    name: str
    grid: GridSpec
    depth: int
    circuit_seed: int
    k: int
    bitstring_seed: int
    cap: Optional[int]
    precision: str
    open_qubits: Tuple[int, ...] = field(default_factory=tuple)
    n_slices_target: Optional[int] = None
    oracle_subset: Optional[int] = None
    slice_subset: Optional[int] = None
    slice_subset_seed: Optional[int] = None

    @property
    def n_qubits(self) -> int:
        return self.grid.rows * self.grid.cols - len(self.grid.removed)

    def circuit(self) -> dict:
        return random_circuit(self.grid, self.depth, self.circuit_seed)

    def bitstrings(self) -> np.ndarray:
        """The closed part of the batch.  With open qubits, those bits are zero
        and each row is one group (a closed-prefix assignment)."""
        words = uniform_bitstrings(self.n_qubits, self.k, self.bitstring_seed)
        if self.open_qubits:
            mask = np.uint64(0)
            for q in self.open_qubits:
                mask |= np.uint64(1) << np.uint64(q)
            words = words & ~mask
        return words


CONFIGS = {
    "C1": Workload("C1", GridSpec(4, 4), 8, 1, 64, 1001, None, "c128"),
    "C2": Workload("C2", GridSpec(5, 6), 12, 2, 4096, 1002, 28, "c64", oracle_subset=256),
    "C3": Workload("C3", GridSpec(6, 6), 14, 3, 64, 1003, 30, "c64",
                   open_qubits=tuple(range(28, 36)), n_slices_target=256),
    "C4": Workload("C4", GridSpec(6, 9, ((5, 8),)), 14, 4, 1024, 1004, 32, "c64",
                   slice_subset=64, slice_subset_seed=2004),
}


def sub_instance_c4() -> Workload:
    """4x5, depth 14: the 20-qubit instance on which C4's precision error is
    measured (sliced to 64 slices by lowering its cap)."""
    return Workload("C4sub", GridSpec(4, 5), 14, 40, 1024, 1040, None, "c64")


C5_GRIDS = ((4, 5), (4, 6), (4, 7), (4, 8), (4, 9), (5, 5), (5, 6), (5, 7), (6, 6))


def uneven_batch_c5(n_circuits: int = 32, master_seed: int = 5) -> List[Workload]:
    rng = np.random.default_rng(master_seed)
    out = []
    for i in range(n_circuits):
        r, c = C5_GRIDS[int(rng.integers(0, len(C5_GRIDS)))]
        depth = int(rng.integers(10, 17))
        k = 1 << int(rng.integers(8, 13))
        out.append(Workload(f"C5.{i}", GridSpec(r, c), depth, 500 + i, k, 1500 + i, 28, "chalf"))
    return out
