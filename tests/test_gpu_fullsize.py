"""Exact checks at full workload size, where no state vector fits.

On a permutation circuit (X/I single-qubit layers, fSim(pi/2, phi), any
last layer) every wire between two-qubit gates carries one basis value, so
of all slices of a sliced network exactly one -- the assignment of the
trajectory -- contributes, and its partial amplitudes are the full
amplitudes a(b) = c prod_q U_q[b_q, y_q] (oracle.closed_forms).  Running
that one slice on the GPU checks the plan, gathers, open legs, groups and
scaling of the 6x6 depth-14 workload (36 qubits, 8 open legs, 64 groups,
2^8 slices) against exact values; a neighbouring slice must give zero.
"""

import functools

import numpy as np
import pytest

from gpu_util import assert_close, rel_err, require_gpu, say
from oracle import closed_forms
from workload import CONFIGS, permutation_circuit

pytestmark = pytest.mark.gpu


def trajectory_slice(net, sliced, traj):
    """Slice id whose bits are the trajectory's values on the sliced wires.
    Tensor t of the fused network is the t-th two-qubit gate; its first two
    indices are that gate's output wires (qubit a, qubit b)."""
    sigma = 0
    for j, bond in enumerate(sliced):
        for t, ix in enumerate(net.indices[:len(traj)]):
            if bond in ix[:2]:
                (qa, va), (qb, vb) = traj[t]
                sigma |= (va if bond == ix[0] else vb) << j
                break
        else:
            raise AssertionError("sliced index is not a two-qubit gate output wire")
    return sigma


def expected_block(circ, groups, opens):
    words = []
    for g in groups:
        for j in range(1 << len(opens)):
            word = int(g)
            for t, q in enumerate(opens):
                word |= ((j >> t) & 1) << q
            words.append(word)
    a = closed_forms.permutation_amplitudes(circ, np.array(words, dtype=np.uint64))
    return a.reshape(len(groups), 1 << len(opens))


@functools.lru_cache(maxsize=1)
def c3_permutation_plan():
    from paper_2212_04749_amd import planner
    from paper_2212_04749_amd.circuit_tn import build_network
    w = CONFIGS["C3"]
    circ = permutation_circuit(w.grid, w.depth, 303)
    net = build_network(circ)
    say("C3-size permutation: planning")
    pl = planner.find_plan(net, w.bitstrings(), w.open_qubits, w.cap, trials=4, exact_slices=8, refine_top=1)
    return w, circ, net, pl


@pytest.mark.parametrize("precision,tol", [("c64", 1e-5), ("chalf", 3e-3)])
def test_c3_stored_plan_permutation_circuit(precision, tol):
    # the stored 6x6 plan that the bench times (plans/c3_cap30.json), bound
    # as the bench binds it (slice batch 8, key chunks under the default
    # memory budget) to the random circuit; then the permutation circuit's
    # leaves are swapped in (matnc_plan_set_tensor) and the slice batch
    # holding the trajectory's slice is run through the captured graph: it
    # must give the exact amplitudes, a batch without it zero, and swapping
    # the random leaves back must reproduce the first result bit for bit
    require_gpu()
    from paper_2212_04749_amd import api
    from paper_2212_04749_amd.circuit_tn import build_network
    from paper_2212_04749_amd.plans import make_c3
    w = CONFIGS["C3"]
    e = make_c3.load()
    net = build_network(w.circuit())
    circ = permutation_circuit(w.grid, w.depth, 303)
    pnet = build_network(circ)
    assert pnet.indices == net.indices
    groups, opens = w.bitstrings(), w.open_qubits
    spec = api.PlanSpec([tuple(p) for p in e["pairs"]], e["sliced"], tuple(opens), e["cap"])
    batch = 8
    run = api.Contraction(net, spec, groups, precision=precision, slice_batch=batch)
    sigma = trajectory_slice(pnet, e["sliced"], closed_forms.permutation_trajectory(circ))
    b0 = sigma - sigma % batch
    say(f"stored 6x6 plan {precision}: {run.n_slices} slices, {run.info.n_chunks} key chunks, "
        f"workspace {run.info.workspace_bytes / 2**30:.1f} GiB, trajectory slice {sigma}, batch [{b0}, {b0 + batch})")
    assert run.n_slices == 256
    first = run.execute(None, b0, b0 + batch)
    run.synchronize()
    first = first.cpu().numpy()
    for t, x in enumerate(pnet.tensors):
        run.set_tensor(t, x)
    amps = run.execute(None, b0, b0 + batch)
    run.synchronize()
    a = amps.cpu().numpy()
    got = a[..., 0] + 1j * a[..., 1]
    ref = expected_block(circ, groups, opens)
    assert np.allclose(np.abs(ref), 2.0 ** -18, rtol=1e-12)
    err = assert_close(got, ref, tol)
    say(f"stored 6x6 plan {precision}: permutation leaves, rel err {err:.2e}")
    b1 = (b0 + batch) % run.n_slices
    amps2 = run.execute(None, b1, b1 + batch)
    run.synchronize()
    assert np.max(np.abs(amps2.cpu().numpy())) <= 1e-6 * 2.0 ** -18
    for t, x in enumerate(net.tensors):
        run.set_tensor(t, x)
    again = run.execute(None, b0, b0 + batch)
    run.synchronize()
    assert np.array_equal(again.cpu().numpy(), first)
    run.close()


def test_c3_size_permutation_every_fp16_configuration(tmp_path):
    # the complex-half plan of the 6x6 workload has plain FP16 MFMA steps
    # (no fan-out): every FP16 tile configuration forced on them, against the
    # exact amplitudes of the one contributing slice
    require_gpu()
    from paper_2212_04749_amd import api
    from test_gpu_chalf import force_fp16_configs
    w, circ, net, pl = c3_permutation_plan()
    groups = w.bitstrings()
    opens = w.open_qubits
    spec = api.PlanSpec(pl.pairs, pl.sliced, tuple(opens), w.cap)
    run = api.Contraction(net, spec, groups, precision="chalf", slice_batch=1)
    sigma = trajectory_slice(net, pl.sliced, closed_forms.permutation_trajectory(circ))
    ref = expected_block(circ, groups, opens)

    def check(c, kids):
        amps = run.execute(None, sigma, sigma + 1)
        run.synchronize()
        a = amps.cpu().numpy()
        err = assert_close(a[..., 0] + 1j * a[..., 1], ref, 3e-3, f"configuration {c}")
        say(f"FP16 tile configuration {c}: kernels {kids}, rel err {err:.2e}")

    ran = force_fp16_configs(run, str(tmp_path / "tune.json"), check)
    assert any(300 <= kid < 400 for kid in ran)
    run.close()


@pytest.mark.parametrize("precision,tol", [("c64", 1e-5), ("chalf", 3e-3)])
def test_c4_size_permutation_circuit(precision, tol):
    # the 53-qubit workload's network structure and stored plan (4096
    # slices), on a permutation circuit: the one contributing slice gives
    # the exact amplitudes (modulus 2^-26.5, which also exercises the
    # complex-half exponents) and a neighbouring slice gives zero
    require_gpu()
    from paper_2212_04749_amd import api
    from paper_2212_04749_amd.circuit_tn import build_network
    from paper_2212_04749_amd.plans import make_c4
    w = CONFIGS["C4"]
    circ = permutation_circuit(w.grid, w.depth, 404)
    net = build_network(circ)
    e = make_c4.load()
    spec = api.PlanSpec([tuple(p) for p in e["pairs"]], e["sliced"], (), e["cap"])
    words = w.bitstrings()
    run = api.Contraction(net, spec, words, precision=precision, slice_batch=1)
    sigma = trajectory_slice(net, e["sliced"], closed_forms.permutation_trajectory(circ))
    say(f"53-qubit permutation {precision}: {run.n_slices} slices, slice {sigma}")
    amps = run.execute(None, sigma, sigma + 1)
    run.synchronize()
    a = amps.cpu().numpy()
    got = a[..., 0, 0] + 1j * a[..., 0, 1]
    ref = closed_forms.permutation_amplitudes(circ, words)
    assert np.allclose(np.abs(ref), 2.0 ** -26.5, rtol=1e-12)
    assert_close(got, ref, tol)
    other = sigma ^ 1
    amps2 = run.execute(None, other, other + 1)
    run.synchronize()
    assert np.max(np.abs(amps2.cpu().numpy())) <= 1e-6 * 2.0 ** -26.5
    run.close()
