"""Amplitudes with closed forms, usable at any qubit count.

Product state (depth 0): a single layer of one-qubit gates U_q on |0...0>
gives a(b) = prod_q U_q[b_q, 0].

Permutation circuits: when every gate before the last single-qubit layer maps
computational basis states to phased basis states, the state before that
layer is c |y> for one bitstring y and one phase c, and
a(b) = c prod_q U_q[b_q, y_q].  X flips a bit, I does nothing, and fSim with
theta = pi/2 and zero Deltas (Supplementary Sec. I) acts on |q_a q_b> as
|00> -> |00>, |01> -> -i |10>, |10> -> -i |01>, |11> -> e^{-i phi} |11>.
Every such amplitude has modulus 2^(-n/2) when each U_q is one of
sqrt(X), sqrt(Y), sqrt(W) (all their entries have modulus 1/sqrt(2)).

Slicing (Supplementary Sec. IV.B) fixes a wire of the network to one value;
on a permutation circuit every wire between gates carries a single basis
value (the trajectory), so exactly one assignment of a sliced set -- the
trajectory's -- contributes, and every other slice is exactly zero.
"""

from __future__ import annotations

import math

import numpy as np

from . import gates
from .circuit import words_to_bits


def _last_layer(circ: dict):
    layers = circ["layers"]
    if not layers or layers[-1]["kind"] != "1q":
        raise ValueError("closed form: circuit must end with a single-qubit layer")
    n = int(circ["n_qubits"])
    U = [gates.identity() for _ in range(n)]
    for q, name in layers[-1]["gates"]:
        U[q] = gates.one_qubit(name) @ U[q]
    return layers[:-1], U


def permutation_state(circ: dict):
    """(y bits, phase) of the basis state before the last single-qubit layer."""
    n = int(circ["n_qubits"])
    body, _ = _last_layer(circ)
    y = [0] * n
    phase = complex(1.0)
    for layer in body:
        if layer["kind"] == "1q":
            for q, name in layer["gates"]:
                if name == "X":
                    y[q] ^= 1
                elif name != "I":
                    raise ValueError("closed form: not a permutation circuit")
        else:
            for qa, qb, theta, phi in layer["gates"]:
                if abs(math.cos(theta)) > 1e-12 or math.sin(theta) < 0:
                    raise ValueError("closed form: fSim must have theta = pi/2")
                a, b = y[qa], y[qb]
                if a != b:
                    y[qa], y[qb] = b, a
                    phase *= -1j
                elif a == 1:
                    phase *= complex(math.cos(phi), -math.sin(phi))
    return y, phase


def permutation_trajectory(circ: dict):
    """Basis values along a permutation circuit: entry g lists, for the g-th
    two-qubit gate in circuit order, ((qubit_a, bit after the gate),
    (qubit_b, bit after the gate))."""
    n = int(circ["n_qubits"])
    body, _ = _last_layer(circ)
    y = [0] * n
    out = []
    for layer in body:
        if layer["kind"] == "1q":
            for q, name in layer["gates"]:
                if name == "X":
                    y[q] ^= 1
                elif name != "I":
                    raise ValueError("closed form: not a permutation circuit")
        else:
            for qa, qb, theta, phi in layer["gates"]:
                if abs(math.cos(theta)) > 1e-12 or math.sin(theta) < 0:
                    raise ValueError("closed form: fSim must have theta = pi/2")
                if y[qa] != y[qb]:
                    y[qa], y[qb] = y[qb], y[qa]
                out.append(((int(qa), y[qa]), (int(qb), y[qb])))
    return out


def permutation_amplitudes(circ: dict, words) -> np.ndarray:
    n = int(circ["n_qubits"])
    y, phase = permutation_state(circ)
    _, U = _last_layer(circ)
    bits = words_to_bits(words, n)
    out = np.empty(len(bits), dtype=np.complex128)
    for i, b in enumerate(bits):
        a = phase
        for q in range(n):
            a *= U[q][b[q], y[q]]
        out[i] = a
    return out


def product_amplitudes(circ: dict, words) -> np.ndarray:
    if any(L["kind"] == "2q" and L["gates"] for L in circ["layers"]):
        raise ValueError("closed form: product state needs no two-qubit gates")
    n = int(circ["n_qubits"])
    U = [gates.identity() for _ in range(n)]
    for layer in circ["layers"]:
        for q, name in layer["gates"]:
            U[q] = gates.one_qubit(name) @ U[q]
    bits = words_to_bits(words, n)
    out = np.empty(len(bits), dtype=np.complex128)
    for i, b in enumerate(bits):
        a = complex(1.0)
        for q in range(n):
            a *= U[q][b[q], 0]
        out[i] = a
    return out
