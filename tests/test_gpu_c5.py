"""The uneven batch through one queue: the circuits of the seeded uneven
batch with at most 25 qubits (10 of the 32: 20-25 qubits, depth 10-16,
256-4096 bitstrings), with their stored plans, contracted in complex-half as
one captured queue, against the oracle's state vector; every replay of the
queue must be bit-identical to the first."""

import numpy as np
import pytest

from gpu_util import rel_err, require_gpu, say
from oracle import sv_native, xeb as oxeb

pytestmark = pytest.mark.gpu


def test_uneven_queue_against_statevector():
    torch = require_gpu()
    from paper_2212_04749_amd import api
    from paper_2212_04749_amd.circuit_tn import build_network
    from paper_2212_04749_amd.plans import make_c5
    from workload.configs import uneven_batch_c5
    plans = make_c5.load()
    stream = torch.cuda.Stream()
    runs, refs = [], []
    for w in uneven_batch_c5():
        if w.n_qubits > 25:
            continue
        e = plans[w.name]
        net = build_network(w.circuit())
        spec = api.PlanSpec([tuple(x) for x in e["pairs"]], e["sliced"], (), e["cap"])
        runs.append(api.Contraction(net, spec, w.bitstrings(), precision="chalf", stream=stream))
        refs.append((w.name, w.n_qubits, sv_native.amplitudes(w.circuit(), w.bitstrings())))
    assert len(runs) == 10
    say(f"uneven queue of {len(runs)} circuits")
    q = api.Queue(runs)
    amps, xeb = q.execute()
    stream.synchronize()
    first = [a.cpu().numpy() for a in amps]
    xs = xeb.cpu().numpy()
    for (name, n, ref), a, x in zip(refs, first, xs):
        got = a[:, 0, 0] + 1j * a[:, 0, 1]
        e = rel_err(got, ref)
        say(f"{name}: {n} qubits, rel err {e:.2e}, xeb {x:.4f}")
        assert e <= 3e-3, name
        assert abs(x - oxeb.linear_xeb(ref, n)) <= 1e-4, name
    for rep in range(2):
        q.execute(amps, xeb)
        stream.synchronize()
        assert all(np.array_equal(f, a.cpu().numpy()) for f, a in zip(first, amps)), f"replay {rep}"
    q.close()
    for r in runs:
        r.close()
