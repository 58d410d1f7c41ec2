"""Plain-C state vector (oracle/sv.c) for circuits up to 30+ qubits.

Same definition as ``statevector`` (amplitude = <b|U|0...0>, gates applied in
circuit order), written as in-place loops in C so that 30-qubit references
(16 GiB of complex128) finish in minutes on the host cores.  The gate
matrices come from ``oracle.gates`` through ``oracle.circuit``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .circuit import gate_list

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sv.c")
LIB = os.path.join(HERE, "libsv.so")


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _lib():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    L = ctypes.CDLL(LIB)
    L.sv_amplitudes.restype = ctypes.c_int
    L.sv_amplitudes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    return L


def amplitudes(circ: dict, words, max_gates=None) -> np.ndarray:
    """Amplitudes of the bitstrings in ``words``.  ``max_gates`` stops after
    the first gates of the circuit (used only to time a bounded sample)."""
    n, glist = gate_list(circ)
    if max_gates is not None:
        glist = glist[:max_gates]
    G = len(glist)
    kind = np.zeros(G, dtype=np.int32)
    qa = np.zeros(G, dtype=np.int32)
    qb = np.zeros(G, dtype=np.int32)
    mats = np.zeros((G, 32), dtype=np.float64)
    for g, (qubits, mat) in enumerate(glist):
        kind[g] = len(qubits)
        qa[g] = qubits[0]
        qb[g] = qubits[-1]
        flat = np.ascontiguousarray(mat).reshape(-1)
        mats[g, : 2 * flat.size] = np.stack([flat.real, flat.imag], axis=1).reshape(-1)
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64).reshape(-1))
    out = np.zeros(2 * len(w), dtype=np.float64)
    rc = _lib().sv_amplitudes(n, G, kind.ctypes.data, qa.ctypes.data, qb.ctypes.data, mats.ctypes.data,
                              len(w), w.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle sv: state does not fit in host memory")
    return out[0::2] + 1j * out[1::2]
