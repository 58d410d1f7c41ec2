"""Complex-half path (FP16 storage + per-instance exponents, FP16 MFMA, FP32
accumulation, FP64 slice-sum) against the FP64 oracle.

Bar: ||a - a_ref|| / ||a_ref|| <= 3e-3 over the batch and |XEB - XEB_ref|
<= 1e-4.  The intermediates whose steps carry the most estimated time are
stored in FP16, as many as the batch size allows (the plan's precision
budget, min(16, K / 282) tensors for K amplitudes); leaves and the rest stay
FP32.
"""

import json
import os

import numpy as np
import pytest

from gpu_util import assert_close, require_gpu, say
from oracle import closed_forms, statevector, xeb as oxeb
from workload import CONFIGS, GridSpec, permutation_circuit, random_circuit, sub_instance_c4, uniform_bitstrings

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def contraction(circ, words, open_qubits=(), cap=None, batch=1, trials=8, half_nodes=-1):
    # half_nodes > 0 forces FP16 tensors into small batches whose default
    # budget is none (checks of the amplitude bar only)
    from paper_2212_04749_amd import api
    return api.Contraction.from_circuit(circ, words, open_qubits=open_qubits, cap=cap, precision="chalf",
                                        slice_batch=batch, trials=trials, half_nodes=half_nodes)


def xeb_of(a, n):
    return float(np.ldexp(np.mean(np.abs(a) ** 2), n) - 1)


def test_chalf_c1_and_sliced():
    require_gpu()
    w = CONFIGS["C1"]
    circ, words = w.circuit(), w.bitstrings()
    ref = statevector.amplitudes(circ, words)
    say("chalf C1")
    run = contraction(circ, words)
    got = run.amplitudes()
    e1 = assert_close(got, ref, 3e-3)
    f = run.xeb()
    run.close()
    say(f"chalf C1 rel err {e1:.2e} xeb err {abs(f - oxeb.linear_xeb(ref, 16)):.2e}")
    assert abs(f - oxeb.linear_xeb(ref, 16)) <= 1e-4
    say("chalf C1 sliced cap 12, 12 FP16 tensors")
    run = contraction(circ, words, cap=12, batch=4, half_nodes=12)
    assert run.info.n_half_nodes == 12
    assert run.n_slices >= 4
    got = run.amplitudes()
    run.close()
    assert_close(got, ref, 3e-3)


def test_chalf_open_legs():
    require_gpu()
    circ = random_circuit(GridSpec(3, 4), 7, 8)
    opens = (1, 6, 10)
    words = uniform_bitstrings(12, 20, 9)
    psi = statevector.final_state(circ)
    say("chalf open legs")
    run = contraction(circ, words, open_qubits=opens, cap=9, half_nodes=12)
    got = run.amplitudes()
    run.close()
    ref = np.zeros_like(got)
    for i, w0 in enumerate(words):
        for j in range(8):
            word = int(w0)
            for t, q in enumerate(opens):
                word = (word & ~(1 << q)) | (((j >> t) & 1) << q)
            ref[i, j] = statevector.amplitudes_from_state(psi, [word])[0]
    assert_close(got, ref, 3e-3)


@pytest.mark.parametrize("precision,tol", [("c64", 1e-5), ("chalf", 3e-3)])
def test_c4_sub_instance(precision, tol):
    """The 20-qubit, depth-14 instance on which the precision error is stated,
    sliced to 64 slices (cap = greedy max rank - 6), 1024 bitstrings, in
    both precisions side by side."""
    require_gpu()
    from paper_2212_04749_amd import api, planner
    from paper_2212_04749_amd.circuit_tn import build_network
    w = sub_instance_c4()
    g = json.load(open(os.path.join(GOLDEN, "c4_sub.json")))
    circ, words = w.circuit(), w.bitstrings()
    assert [str(int(x)) for x in words] == g["words"]
    ref = np.array([complex(a, b) for a, b in g["amps"]])
    net = build_network(circ)
    full = planner.find_plan(net, words, (), None, trials=8)
    cap = full.costs.max_rank - 6
    say(f"{precision} C4 sub-instance cap {cap}")
    run = api.Contraction.from_circuit(circ, words, cap=cap, precision=precision, slice_batch=8, trials=8,
                                       exact_slices=6)
    got = run.amplitudes()
    run.close()
    err = assert_close(got, ref, tol)
    xe = abs(xeb_of(got, 20) - xeb_of(ref, 20))
    say(f"{precision} C4 sub rel err {err:.2e} slices {run.n_slices} xeb err {xe:.2e}")
    assert run.n_slices == 64
    assert xe <= 1e-4


def test_chalf_c2_against_stored_oracle():
    require_gpu()
    w = CONFIGS["C2"]
    g = json.load(open(os.path.join(GOLDEN, "c2_subset.json")))
    circ, words = w.circuit(), w.bitstrings()
    idx = np.array(g["indices"])
    ref = np.array([complex(a, b) for a, b in g["amps"]])
    say("chalf C2 full config")
    run = contraction(circ, words, cap=28, batch=4, trials=4)
    got = run.amplitudes()[idx]
    run.close()
    err = assert_close(got, ref, 3e-3)
    say(f"chalf C2 rel err {err:.2e} xeb err {abs(xeb_of(got, 30) - xeb_of(ref, 30)):.2e}")
    assert abs(xeb_of(got, 30) - xeb_of(ref, 30)) <= 1e-4


def test_chalf_permutation_scaling_c2_size():
    """|a| = 2^-15 for every bitstring: exercises the exponent bookkeeping."""
    require_gpu()
    w = CONFIGS["C2"]
    circ = permutation_circuit(w.grid, w.depth, 77)
    words = uniform_bitstrings(30, 512, 78)
    say("chalf permutation 5x6 d12")
    run = contraction(circ, words, cap=28, batch=2, trials=4, half_nodes=20)
    got = run.amplitudes()
    run.close()
    ref = closed_forms.permutation_amplitudes(circ, words)
    assert_close(got, ref, 3e-3)



FP16_TILE_CONFIGS = 9
FP16_FAN_CONFIGS = {c for c in range(FP16_TILE_CONFIGS) if c != 7}  # 7: 128 columns, no fan table


def force_fp16_configs(run, cache, check):
    """Force each FP16 MFMA tile configuration c, through the tuning cache, on
    every FP16-stored MFMA step class of run's plan, and call check(c) after
    each; returns the kernel ids the profile showed (300 + c plain tiles,
    400 + c fan-out tiles)."""
    run.autotune(reps=1, cache_path=cache)
    tuned = json.load(open(cache))
    hkeys = [k for k in tuned if k.startswith("chalf/h/")]
    say(f"FP16 MFMA step classes: {hkeys}")
    assert hkeys
    ran = set()
    for c in range(FP16_TILE_CONFIGS):
        forced = dict(tuned)
        forced.update({k: c for k in hkeys})
        with open(cache, "w") as f:
            json.dump(forced, f)
        run.autotune(reps=1, cache_path=cache)
        kids = {kid for _, kid, _, _ in run.profile() if kid >= 300}
        ran |= kids
        check(c, sorted(kids))
    say(f"FP16 kernels exercised: {sorted(ran)}")
    return ran


def test_every_fp16_fan_out_configuration(tmp_path):
    # a plan whose widest step (w ~ 4000, m/n/k = 9/0/10 bits) is stored in
    # FP16 and runs as fan-out tiles: every FP16 tile configuration (32- and
    # 64-column fan tables) against the state vector
    require_gpu()
    circ = random_circuit(GridSpec(5, 5), 12, 8)
    words = uniform_bitstrings(25, 4096, 9)
    ref = statevector.amplitudes(circ, words)
    run = contraction(circ, words, trials=4)

    def check(c, kids):
        err = assert_close(run.amplitudes(), ref, 3e-3, f"configuration {c}")
        say(f"FP16 tile configuration {c}: kernels {kids}, rel err {err:.2e}")

    ran = force_fp16_configs(run, str(tmp_path / "tune.json"), check)
    assert {kid - 400 for kid in ran if kid >= 400} == FP16_FAN_CONFIGS
    run.close()
