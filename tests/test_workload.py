"""Seeded workload generator: coupler patterns, sequences, gate-choice rule."""

import numpy as np
import pytest

from workload import (CONFIGS, GridSpec, pattern_edges, pattern_sequence, random_circuit,
                      sub_instance_c4, uneven_batch_c5, uniform_bitstrings, u64_to_bits)
from workload.rqc import count_two_qubit_gates, grid_qubits


def all_grid_edges(spec):
    ids = grid_qubits(spec)
    out = set()
    for (r, c), q in ids.items():
        for other in ((r, c + 1), (r + 1, c)):
            if other in ids:
                out.add(tuple(sorted((q, ids[other]))))
    return out


@pytest.mark.parametrize("spec", [GridSpec(4, 4), GridSpec(5, 6), GridSpec(6, 9, ((5, 8),)),
                                  GridSpec(3, 7), GridSpec(1, 5)])
def test_patterns_are_matchings_that_partition_the_edges(spec):
    # Supplementary Sec. I: each neighbouring pair gets one gate in any ABCD window
    seen = []
    for letter in "ABCD":
        e = pattern_edges(spec, letter)
        qs = [q for pair in e for q in pair]
        assert len(qs) == len(set(qs)), f"pattern {letter} is not a matching"
        seen.extend(e)
    assert len(seen) == len(set(seen))
    assert set(seen) == all_grid_edges(spec)


def test_printed_sequences():
    # Supplementary Sec. I prints the depth-8 and depth-12 sequences
    assert pattern_sequence(8) == "ABCDCDAB"
    assert pattern_sequence(12) == "ABCDCDABABCD"
    assert pattern_sequence(14) == "ABCDCDABABCDCD"


def test_corner_removed_keeps_ids_contiguous():
    ids = grid_qubits(GridSpec(6, 9, ((5, 8),)))
    assert sorted(ids.values()) == list(range(53))
    assert (5, 8) not in ids


def test_single_qubit_rule():
    circ = random_circuit(GridSpec(3, 3), 6, 11)
    one = [L for L in circ["layers"] if L["kind"] == "1q"]
    assert len(one) == 7
    for t in range(1, 7):
        for (q, g), (_, h) in zip(one[t - 1]["gates"], one[t]["gates"]):
            assert g != h
    names = {g for L in one for _, g in L["gates"]}
    assert names <= {"sqrtX", "sqrtY", "sqrtW"}


def test_fsim_counts_of_configs():
    counts = {k: count_two_qubit_gates(w.circuit()) for k, w in CONFIGS.items()}
    assert counts == {"C1": 48, "C2": 147, "C3": 210, "C4": 317}
    assert count_two_qubit_gates(sub_instance_c4().circuit()) == 108


def test_seeded_determinism_and_bits():
    a = uniform_bitstrings(30, 100, 5)
    b = uniform_bitstrings(30, 100, 5)
    assert np.array_equal(a, b)
    bits = u64_to_bits(a, 30)
    rng = np.random.default_rng(5)
    assert np.array_equal(bits, rng.integers(0, 2, (100, 30)))


def test_open_qubits_zeroed_in_groups():
    w = CONFIGS["C3"]
    words = w.bitstrings()
    assert len(words) == 64
    mask = sum(1 << q for q in w.open_qubits)
    assert all(int(x) & mask == 0 for x in words)


def test_c5_ranges():
    ws = uneven_batch_c5()
    assert len(ws) == 32
    for w in ws:
        assert 20 <= w.n_qubits <= 36
        assert 10 <= w.depth <= 16
        assert 256 <= w.k <= 4096
