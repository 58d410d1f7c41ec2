"""Pins of the oracle's state vector, tensor network and XEB.

* brute force: a dense 2^n x 2^n matrix built entry by entry from each gate's
  action on basis states (no tensordot), for n <= 6;
* product states and permutation circuits have closed forms at any n;
* normalisation: the probabilities of all 2^n bitstrings sum to 1, and XEB
  over all of them is 0;
* the tensor network (its own unfused network and order) matches the state
  vector to 1e-12 on the 4x4 depth-8 circuit, with and without slicing, with
  open legs;
* XEB: the mean of x under Eq. (2) is 1 + F, checked by quadrature;
* planted mistakes in the oracle are caught by these pins.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import closed_forms, gates, statevector, tn, xeb
from oracle.circuit import gate_list
from workload import (CONFIGS, GridSpec, permutation_circuit, product_circuit, random_circuit,
                      uniform_bitstrings)


def dense_unitary(circ):
    """Brute force: every gate as a 2^n x 2^n matrix filled entry by entry."""
    n, glist = gate_list(circ)
    N = 1 << n
    total = np.eye(N, dtype=complex)
    for qubits, mat in glist:
        M = np.zeros((N, N), dtype=complex)
        for col in range(N):
            if len(qubits) == 1:
                (q,) = qubits
                bi = (col >> q) & 1
                for bo in (0, 1):
                    row = (col & ~(1 << q)) | (bo << q)
                    M[row, col] += mat[bo, bi]
            else:
                qa, qb = qubits
                ia, ib = (col >> qa) & 1, (col >> qb) & 1
                for oa, ob in itertools.product((0, 1), repeat=2):
                    row = (col & ~(1 << qa) & ~(1 << qb)) | (oa << qa) | (ob << qb)
                    M[row, col] += mat[2 * oa + ob, 2 * ia + ib]
        total = M @ total
    return total


@pytest.mark.parametrize("spec,depth,seed", [(GridSpec(2, 2), 4, 3), (GridSpec(2, 3), 5, 4),
                                              (GridSpec(1, 5), 6, 5)])
def test_statevector_vs_brute_force(spec, depth, seed):
    circ = random_circuit(spec, depth, seed)
    n = circ["n_qubits"]
    U = dense_unitary(circ)
    words = np.arange(1 << n, dtype=np.uint64)  # word index = bit pattern, bit q = qubit q
    ref = U[:, 0]
    got = statevector.amplitudes(circ, words)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_product_state_closed_form():
    circ = product_circuit(GridSpec(3, 4), 9)
    words = np.arange(1 << 12, dtype=np.uint64)
    a = statevector.amplitudes(circ, words)
    b = closed_forms.product_amplitudes(circ, words)
    assert np.max(np.abs(a - b)) < 1e-14


@pytest.mark.parametrize("spec,depth,seed", [(GridSpec(3, 3), 6, 1), (GridSpec(4, 4), 8, 2)])
def test_permutation_circuit_closed_form(spec, depth, seed):
    circ = permutation_circuit(spec, depth, seed)
    n = circ["n_qubits"]
    words = uniform_bitstrings(n, 64, 77)
    a = statevector.amplitudes(circ, words)
    b = closed_forms.permutation_amplitudes(circ, words)
    assert np.max(np.abs(a - b)) < 1e-13
    assert np.allclose(np.abs(b), 2.0 ** (-n / 2), atol=1e-15)
    t = tn.amplitudes(circ, words[:16])
    assert np.max(np.abs(t - b[:16])) < 1e-13


def test_normalisation_and_xeb_of_all_bitstrings():
    circ = CONFIGS["C1"].circuit()
    psi = statevector.final_state(circ)
    p = np.abs(psi.reshape(-1)) ** 2
    assert abs(p.sum() - 1.0) < 1e-12
    assert abs(xeb.linear_xeb(psi.reshape(-1), 16)) < 1e-11


def test_tn_matches_statevector_c1():
    w = CONFIGS["C1"]
    circ = w.circuit()
    words = w.bitstrings()
    ref = statevector.amplitudes(circ, words)
    got = tn.amplitudes(circ, words)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_sliced_sum_equals_unsliced():
    circ = random_circuit(GridSpec(3, 4), 8, 21)
    words = uniform_bitstrings(12, 6, 22)
    plain = tn.Plan(circ)
    sliced = tn.Plan(circ, cap=plain.max_rank - 3)
    assert len(sliced.sliced) >= 3 and sliced.max_rank <= plain.max_rank - 3
    a = tn.amplitudes(circ, words, plan=plain)
    b = tn.amplitudes(circ, words, plan=sliced)
    assert np.max(np.abs(a - b)) < 1e-13
    # the individual slices are not the answer (slicing really splits the sum)
    bits = np.array([(int(words[0]) >> q) & 1 for q in range(12)])
    part = sliced.slice_partial(bits, [0] * len(sliced.sliced))
    assert abs(part[0] - a[0]) > 1e-6


def test_open_legs_match_statevector():
    circ = random_circuit(GridSpec(3, 4), 6, 31)
    psi = statevector.final_state(circ)
    opens = (2, 5, 11)
    words = uniform_bitstrings(12, 5, 32)
    plan = tn.Plan(circ, open_qubits=opens)
    got = tn.amplitudes(circ, words, plan=plan)
    for i, w0 in enumerate(words):
        for j in range(8):
            word = int(w0)
            for t, q in enumerate(opens):
                word = (word & ~(1 << q)) | (((j >> t) & 1) << q)
            ref = statevector.amplitudes_from_state(psi, [word])[0]
            assert abs(got[i, j] - ref) < 1e-13


def test_xeb_reading_of_eq2():
    from scipy.integrate import quad
    for F in (0.0, 0.002, 0.3, 1.0):
        mean, _ = quad(lambda x: x * (F * x + 1 - F) * math.exp(-x), 0, np.inf)
        assert abs(mean - (1 + F)) < 1e-9
    # uniform amplitudes of modulus 2^{-n/2} give F = 0 exactly
    n = 10
    a = np.full(37, 2.0 ** (-n / 2), dtype=complex)
    assert abs(xeb.linear_xeb(a, n)) < 1e-15


def test_xeb_of_exact_samples_near_one():
    # Eq. (2) at F = 1: bitstrings drawn from p give F close to 1
    circ = random_circuit(GridSpec(3, 4), 10, 41)
    psi = statevector.final_state(circ)
    p = (np.abs(np.moveaxis(psi, range(12), range(11, -1, -1)).reshape(-1)) ** 2)
    rng = np.random.default_rng(42)
    idx = rng.choice(1 << 12, size=20000, p=p / p.sum())
    words = idx.astype(np.uint64)
    f = xeb.linear_xeb(statevector.amplitudes_from_state(psi, words), 12)
    assert abs(f - 1.0) < 0.1
    u = uniform_bitstrings(12, 20000, 43)
    f0 = xeb.linear_xeb(statevector.amplitudes_from_state(psi, u), 12)
    assert abs(f0) < 0.1


# --- planted mistakes: each plausible error in the oracle trips a pin --------

def _fsim_transposed(theta, phi, *a):
    g = np.zeros((4, 4), dtype=complex)
    g[0, 0] = 1
    g[1, 1] = g[2, 2] = math.cos(theta)
    g[1, 2] = g[2, 1] = -1j * math.sin(theta)
    g[3, 3] = np.exp(+1j * phi)  # wrong sign of the phase
    return g


def test_planted_phase_sign_is_caught(monkeypatch):
    circ = permutation_circuit(GridSpec(3, 3), 6, 1)
    words = uniform_bitstrings(9, 32, 5)
    good = closed_forms.permutation_amplitudes(circ, words)
    monkeypatch.setattr(gates, "fsim", _fsim_transposed)
    bad = statevector.amplitudes(circ, words)
    assert np.max(np.abs(bad - good)) > 1e-3


def test_planted_axis_order_is_caught(monkeypatch):
    circ = random_circuit(GridSpec(2, 3), 5, 4)
    n = 6
    ref = dense_unitary(circ)[:, 0]
    orig = statevector.final_state

    def wrong(c):
        psi = orig(c)
        return np.transpose(psi, list(range(n))[::-1])  # qubit order reversed
    monkeypatch.setattr(statevector, "final_state", wrong)
    got = statevector.amplitudes(circ, np.arange(1 << n, dtype=np.uint64))
    assert np.max(np.abs(got - ref)) > 1e-3


def test_planted_dropped_slice_is_caught():
    circ = random_circuit(GridSpec(3, 4), 8, 21)
    words = uniform_bitstrings(12, 3, 22)
    plain = tn.Plan(circ)
    sliced = tn.Plan(circ, cap=plain.max_rank - 2)
    bits = np.array([(int(words[0]) >> q) & 1 for q in range(12)])
    full = plain.amplitude_block(bits)[0]
    # sum over all but one slice assignment
    parts = [sliced.slice_partial(bits, a)[0]
             for a in itertools.product((0, 1), repeat=len(sliced.sliced))]
    assert abs(sum(parts) - full) < 1e-13
    assert abs(sum(parts[:-1]) - full) > 1e-8


def test_permutation_trajectory_selects_one_slice():
    # the oracle TN sliced on every wire after the first two-qubit gate of
    # each of two qubits: only the trajectory's values contribute
    circ = permutation_circuit(GridSpec(3, 3), 6, 4)
    traj = closed_forms.permutation_trajectory(circ)
    words = uniform_bitstrings(9, 4, 9)
    ref = closed_forms.permutation_amplitudes(circ, words)
    net = tn.Network(circ)
    # the oracle network's tensor of the g-th two-qubit gate holds that
    # gate's output wires as its first two indices
    two_q = [ix for ix in net.indices if len(ix) == 4]
    (qa, va), (qb, vb) = traj[0]
    wires = [two_q[0][0], two_q[0][1]]
    plan = tn.Plan(circ, sliced=wires)
    for i, w0 in enumerate(words):
        bits = np.array([(int(w0) >> q) & 1 for q in range(9)])
        for x in range(2):
            for y in range(2):
                part = plan.slice_partial(bits, [x, y])[0]
                if (x, y) == (va, vb):
                    assert abs(part - ref[i]) < 1e-14
                else:
                    assert abs(part) < 1e-15


# --- Eq. (2) fidelity estimates (the oracle's maximum likelihood and the
# library's analysis, two independent methods) ---------------------------

def _eq2_samples(fidelity, k, seed):
    # Eq. (2) is the mixture (1 - F) e^{-x} + F x e^{-x}: Exp(1) with
    # probability 1 - F, Gamma(2, 1) with probability F
    rng = np.random.default_rng(seed)
    pick = rng.random(k) < fidelity
    return np.where(pick, rng.gamma(2.0, 1.0, k), rng.exponential(1.0, k))


@pytest.mark.parametrize("fidelity", [0.0, 0.3, 1.0])
def test_mle_fidelity_recovers_eq2_mixtures(fidelity):
    from oracle import xeb as oxeb
    k = 200_000
    x = _eq2_samples(fidelity, k, 91)
    f = oxeb.mle_fidelity(x)
    sigma = np.sqrt((1 + 2 * fidelity - fidelity ** 2) / k)  # of the linear estimate, larger than the MLE's
    assert abs(f - fidelity) <= 5 * sigma
    assert abs((x.mean() - 1) - fidelity) <= 5 * sigma


def test_mle_fidelity_is_the_likelihood_argmax():
    # brute force: the maximiser of sum log(F x + 1 - F) on a fine grid
    from oracle import xeb as oxeb
    x = _eq2_samples(0.4, 3000, 92)
    grid = np.linspace(0.0, 1.0, 20001)
    ll = [np.sum(np.log(f * x + 1 - f)) for f in grid]
    assert abs(oxeb.mle_fidelity(x) - grid[int(np.argmax(ll))]) <= 1e-4
    # the boundaries: all x below 1 pulls F to 0, all above 1 to 1
    assert oxeb.mle_fidelity(np.full(10, 0.5)) == 0.0
    assert oxeb.mle_fidelity(np.full(10, 3.0)) == 1.0


def test_density_of_eq2_integrates_to_one_with_mean_one_plus_f():
    from oracle import xeb as oxeb
    x = np.linspace(0, 60, 600001)
    for f in (0.0, 0.25, 1.0):
        p = oxeb.porter_thomas_density(x, f)
        assert abs(np.trapezoid(p, x) - 1) < 1e-8
        assert abs(np.trapezoid(x * p, x) - (1 + f)) < 1e-8


def test_library_fit_matches_oracle_fit():
    # the library's Newton fit against the oracle's bisection, same samples
    from oracle import xeb as oxeb
    from paper_2212_04749_amd import analysis
    for f, seed in ((0.0, 93), (0.05, 94), (0.5, 95), (1.0, 96)):
        x = _eq2_samples(f, 5000, seed)
        assert abs(analysis.fit_fidelity(x) - oxeb.mle_fidelity(x)) <= 1e-9


def test_probabilities_match_amplitudes_and_sum_to_one():
    from oracle import statevector
    from workload import GridSpec, random_circuit, uniform_bitstrings
    circ = random_circuit(GridSpec(2, 3), 6, 97)
    p = statevector.probabilities(circ)
    assert abs(p.sum() - 1) < 1e-12
    words = uniform_bitstrings(6, 20, 98)
    a = statevector.amplitudes(circ, words)
    assert np.allclose(p[words.astype(np.int64)], np.abs(a) ** 2, atol=1e-15)


def test_mixture_sampler_follows_its_distribution():
    from workload import sample_mixture
    p = np.array([0.5, 0.25, 0.125, 0.125])
    w = sample_mixture(p, 100_000, 1.0, 99)
    freq = np.bincount(w.astype(np.int64), minlength=4) / w.size
    assert np.allclose(freq, p, atol=0.01)
    w0 = sample_mixture(p, 100_000, 0.0, 99)
    assert np.allclose(np.bincount(w0.astype(np.int64), minlength=4) / w0.size, 0.25, atol=0.01)
