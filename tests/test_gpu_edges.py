"""Degenerate batches through the C ABI, against the oracle's state vector:
one bitstring; a batch of one bitstring repeated; every qubit open (one
group whose block is the whole state); an empty slice range (nothing
added).  Both precisions, each at its bar."""

import numpy as np
import pytest

from gpu_util import assert_close, require_gpu, say
from oracle import statevector
from workload import GridSpec, random_circuit, uniform_bitstrings

pytestmark = pytest.mark.gpu

BARS = [("c64", 1e-5), ("chalf", 3e-3)]


@pytest.mark.parametrize("precision,tol", BARS)
def test_single_and_repeated_bitstring(precision, tol):
    require_gpu()
    from paper_2212_04749_amd import api
    circ = random_circuit(GridSpec(3, 4), 8, 71)
    one = uniform_bitstrings(12, 1, 72)
    ref = statevector.amplitudes(circ, one)
    run = api.Contraction.from_circuit(circ, one, cap=8, precision=precision, slice_batch=2, trials=2)
    say(f"{precision}: k = 1, {run.n_slices} slices")
    assert_close(run.amplitudes(), ref, tol, "k = 1")
    run.close()
    rep = np.repeat(one, 7)
    run = api.Contraction.from_circuit(circ, rep, cap=8, precision=precision, slice_batch=2, trials=2)
    assert run.info.n_unique == 1
    got = run.amplitudes()
    run.close()
    assert np.all(got == got[0])
    assert_close(got, np.repeat(ref, 7), tol, "one bitstring repeated")


@pytest.mark.parametrize("precision,tol", BARS)
def test_every_qubit_open(precision, tol):
    # one group with all 12 output indices open: its block is the whole
    # final state, entry j = amplitude of the bitstring j (bit t = qubit t)
    require_gpu()
    from paper_2212_04749_amd import api
    circ = random_circuit(GridSpec(3, 4), 7, 73)
    psi = statevector.final_state(circ)
    words = np.zeros(1, dtype=np.uint64)
    run = api.Contraction.from_circuit(circ, words, open_qubits=tuple(range(12)), cap=12, precision=precision,
                                       trials=2)
    got = run.amplitudes()[0]
    run.close()
    ref = statevector.amplitudes_from_state(psi, np.arange(4096, dtype=np.uint64))
    say(f"{precision}: every qubit open, {got.size} entries")
    assert_close(got, ref, tol, "whole state")
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) <= 2 * tol


def test_empty_slice_range_adds_nothing():
    require_gpu()
    from paper_2212_04749_amd import api
    circ = random_circuit(GridSpec(3, 4), 8, 74)
    words = uniform_bitstrings(12, 20, 75)
    run = api.Contraction.from_circuit(circ, words, cap=7, slice_batch=4, trials=2)
    amps = run.new_amplitudes()
    run.execute(amps, 3, 3)
    run.synchronize()
    assert not amps.any().item()
    run.close()
