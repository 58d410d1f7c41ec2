"""The fidelity workload (main text Eq. (2), Fig. 4): bitstrings sampled from
a mixture of the exact output distribution (weight F) and the uniform one,
their amplitudes computed on the GPU, F estimated from them.

For a 20-qubit circuit the oracle gives the exact distribution p.  Under the
mixture the linear estimate 2^n <p(b)> - 1 has expectation
F (2^n sum_b p(b)^2 - 1), and for Porter-Thomas statistics its standard
deviation is sqrt((1 + 2F - F^2) / k); both fits (linear XEB on the GPU,
maximum likelihood on the host) must land within 5 of those deviations of
their targets, the GPU amplitudes must match the oracle's to the precision's
bar, and the histogram of x = 2^n |a|^2 must be normalised.
"""

import numpy as np
import pytest

from gpu_util import assert_close, require_gpu, say
from oracle import statevector, xeb as oxeb
from workload import GridSpec, random_circuit, sample_mixture

pytestmark = pytest.mark.gpu

N_QUBITS = 20
K = 4096


@pytest.mark.parametrize("fidelity,precision,tol", [(1.0, "c64", 1e-5), (0.5, "c64", 1e-5), (0.0, "c64", 1e-5),
                                                    (1.0, "chalf", 3e-3), (0.2, "chalf", 3e-3)])
def test_fidelity_recovered_from_gpu_amplitudes(fidelity, precision, tol):
    require_gpu()
    from paper_2212_04749_amd import analysis, api
    circ = random_circuit(GridSpec(4, 5), 12, 4501)
    psi = statevector.final_state(circ)
    p = statevector.probabilities(circ)
    ideal = float(np.ldexp(np.sum(p * p), N_QUBITS) - 1.0)  # expected linear estimate at F = 1
    words = sample_mixture(p, K, fidelity, 4502 + int(100 * fidelity))
    ref = statevector.amplitudes_from_state(psi, words)
    run = api.Contraction.from_circuit(circ, words, cap=18, precision=precision, slice_batch=2, trials=4)
    amps = run.execute()
    f_gpu = run.xeb(amps)
    a = amps.cpu().numpy()
    got = a[:, 0, 0] + 1j * a[:, 0, 1]
    run.close()
    err = assert_close(got, ref, tol)
    assert abs(f_gpu - oxeb.linear_xeb(ref, N_QUBITS)) <= 1e-4
    x = analysis.x_values(got, N_QUBITS)
    f_mle = analysis.fit_fidelity(x)
    sigma = np.sqrt((1 + 2 * fidelity - fidelity ** 2) / K)
    say(f"F={fidelity} {precision}: rel err {err:.2e}, linear XEB {f_gpu:.4f} (expected {fidelity * ideal:.4f}), "
        f"MLE {f_mle:.4f}, sigma {sigma:.4f}")
    assert abs(f_gpu - fidelity * ideal) <= 5 * sigma
    assert abs(f_mle - fidelity) <= 5 * sigma
    assert abs(f_mle - oxeb.mle_fidelity(x)) <= 1e-9
    h = analysis.porter_thomas_histogram(x, f_mle)
    width = h["edges"][1] - h["edges"][0]
    inside = K - h["beyond_range"]
    assert abs(sum(h["density"]) * width - inside / K) <= 1e-12
