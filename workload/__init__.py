"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only draws random structure: which gate sits on which qubit in
which cycle, and which bitstrings are asked for.  It holds none of the
method's arithmetic (no gate matrices, no tensor network, no contraction).
Both the oracle and the library read what it produces, each with its own
gate transcription.
"""

from .rqc import (  # noqa: F401
    GridSpec,
    grid_qubits,
    pattern_edges,
    pattern_sequence,
    random_circuit,
    permutation_circuit,
    product_circuit,
    circuit_to_json,
    circuit_from_json,
)
from .bitstrings import uniform_bitstrings, bits_to_u64, u64_to_bits, sample_mixture  # noqa: F401
from .configs import CONFIGS, sub_instance_c4, uneven_batch_c5  # noqa: F401
