"""Pins of the oracle's gate matrices (Supplementary Sec. I).

Each check is against a property fixed by the mathematics, not against the
matrices retyped: unitarity, sqrt(P)^2 = -i P for the Pauli-type P, the
action of fSim(pi/2, phi) on basis states, and agreement with the library's
independent transcription.
"""

import math

import numpy as np
import pytest

from oracle import gates
from paper_2212_04749_amd import circuit_tn

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
W = (X + Y) / math.sqrt(2)


@pytest.mark.parametrize("name", ["sqrtX", "sqrtY", "sqrtW", "X", "I"])
def test_unitary(name):
    u = gates.one_qubit(name)
    assert np.allclose(u.conj().T @ u, np.eye(2), atol=1e-15)


@pytest.mark.parametrize("name,P", [("sqrtX", X), ("sqrtY", Y), ("sqrtW", W)])
def test_square_roots(name, P):
    u = gates.one_qubit(name)
    assert np.allclose(u @ u, -1j * P, atol=1e-15)


def test_fsim_unitary_and_closed_form():
    phi = math.pi / 6
    g = gates.fsim(math.pi / 2, phi)
    assert np.allclose(g.conj().T @ g, np.eye(4), atol=1e-15)
    e = np.eye(4)
    # basis |q_a q_b>, index = 2 q_a + q_b
    assert np.allclose(g @ e[0], e[0], atol=1e-15)
    assert np.allclose(g @ e[1], -1j * e[2], atol=1e-15)
    assert np.allclose(g @ e[2], -1j * e[1], atol=1e-15)
    assert np.allclose(g @ e[3], np.exp(-1j * phi) * e[3], atol=1e-15)


def test_fsim_special_cases():
    assert np.allclose(gates.fsim(0.0, 0.0), np.eye(4), atol=1e-15)
    # theta = pi/2, phi = 0 is iSWAP^dagger (SWAP with -i on the swapped pair)
    swap = np.eye(4)[[0, 2, 1, 3]]
    g = gates.fsim(math.pi / 2, 0.0)
    assert np.allclose(np.abs(g), swap, atol=1e-15)


def test_fsim_swap_symmetric_at_zero_deltas():
    swap = np.eye(4)[[0, 2, 1, 3]]
    g = gates.fsim(math.pi / 2, math.pi / 6)
    assert np.allclose(swap @ g @ swap, g, atol=1e-15)


def test_two_transcriptions_agree():
    for name in ["sqrtX", "sqrtY", "sqrtW", "X", "I"]:
        assert np.allclose(gates.one_qubit(name), circuit_tn.one_qubit_matrix(name), atol=1e-15)
    for th, ph in [(math.pi / 2, math.pi / 6), (0.3, 1.1)]:
        assert np.allclose(gates.fsim(th, ph), circuit_tn.fsim_matrix(th, ph), atol=1e-15)
