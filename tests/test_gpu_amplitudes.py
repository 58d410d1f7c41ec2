"""End-to-end amplitudes and XEB through the C ABI vs the FP64 oracle.

Tolerances (complex64 path): ||a - a_ref||_2 / ||a_ref||_2 <= 1e-5 over the
batch, |XEB - XEB_ref| <= 1e-4 (the stated bars for complex64).
"""

import numpy as np
import pytest

from gpu_util import assert_close, rel_err, require_gpu, say
from oracle import closed_forms, statevector, tn as otn, xeb as oxeb
from workload import CONFIGS, GridSpec, permutation_circuit, product_circuit, random_circuit, uniform_bitstrings

pytestmark = pytest.mark.gpu


def contraction(circ, words, open_qubits=(), cap=None, batch=1, precision="c64", trials=8, exact=None):
    from paper_2212_04749_amd import api
    return api.Contraction.from_circuit(circ, words, open_qubits=open_qubits, cap=cap, precision=precision,
                                        slice_batch=batch, trials=trials, exact_slices=exact)


def test_c1_against_statevector():
    require_gpu()
    w = CONFIGS["C1"]
    circ, words = w.circuit(), w.bitstrings()
    say("C1 c64 k=64")
    run = contraction(circ, words)
    got = run.amplitudes()
    ref = statevector.amplitudes(circ, words)
    assert_close(got, ref, 1e-5)
    f = run.xeb()
    assert abs(f - oxeb.linear_xeb(ref, 16)) <= 1e-4
    run.close()


@pytest.mark.parametrize("batch", [1, 3, 8])
def test_sliced_matches_unsliced_and_oracle(batch):
    require_gpu()
    circ = random_circuit(GridSpec(3, 4), 8, 5)
    words = uniform_bitstrings(12, 50, 6)
    ref = statevector.amplitudes(circ, words)
    say(f"sliced 3x4 d8 cap=7 batch={batch}")
    run = contraction(circ, words, cap=7, batch=batch)
    assert run.n_slices >= 8
    got = run.amplitudes()
    assert_close(got, ref, 1e-5)
    # the sum over slices is not any single slice: splitting the range and
    # adding into one buffer is bit-identical to a single call
    amps = run.new_amplitudes()
    cut = run.n_slices // 3
    run.execute(amps, 0, cut)
    run.execute(amps, cut, run.n_slices)
    run.synchronize()
    whole = run.execute()
    run.synchronize()
    assert run.torch.equal(amps, whole)
    run.close()


def test_open_legs_against_statevector():
    require_gpu()
    circ = random_circuit(GridSpec(3, 4), 7, 8)
    opens = (1, 6, 10)
    words = uniform_bitstrings(12, 20, 9)
    psi = statevector.final_state(circ)
    say("open legs 3x4 d7, 3 open")
    run = contraction(circ, words, open_qubits=opens, cap=9)
    got = run.amplitudes()
    ref = np.zeros_like(got)
    for i, w0 in enumerate(words):
        for j in range(8):
            word = int(w0)
            for t, q in enumerate(opens):
                word = (word & ~(1 << q)) | (((j >> t) & 1) << q)
            ref[i, j] = statevector.amplitudes_from_state(psi, [word])[0]
    assert_close(got, ref, 1e-5)
    run.close()


def test_duplicates_and_determinism():
    require_gpu()
    circ = random_circuit(GridSpec(3, 3), 6, 10)
    base = uniform_bitstrings(9, 12, 11)
    words = np.concatenate([base, base[:5], base[3:4]])
    say("duplicates 3x3")
    run = contraction(circ, words, cap=6, batch=2)
    a1 = run.amplitudes()
    a2 = run.amplitudes()
    assert np.array_equal(a1, a2)
    ref = statevector.amplitudes(circ, words)
    assert_close(a1, ref, 1e-5)
    assert np.array_equal(a1[12:17], a1[:5])
    run.close()


def test_product_state():
    require_gpu()
    circ = product_circuit(GridSpec(2, 3), 12)
    words = np.arange(64, dtype=np.uint64)
    say("product 2x3")
    run = contraction(circ, words)
    got = run.amplitudes()
    assert_close(got, closed_forms.product_amplitudes(circ, words), 1e-6)
    run.close()


def test_all_amplitudes_normalised_and_xeb_zero():
    require_gpu()
    circ = random_circuit(GridSpec(3, 4), 8, 13)
    words = np.arange(1 << 12, dtype=np.uint64)
    say("all 2^12 amplitudes")
    run = contraction(circ, words, cap=9, batch=4)
    amps = run.execute()
    f = run.xeb(amps)
    a = amps.cpu().numpy()
    p = (a[..., 0] ** 2 + a[..., 1] ** 2).sum()
    assert abs(p - 1.0) < 1e-5
    assert abs(f) < 1e-4
    run.close()


def test_permutation_circuit_c2_size():
    require_gpu()
    w = CONFIGS["C2"]
    circ = permutation_circuit(w.grid, w.depth, 77)
    words = uniform_bitstrings(30, 512, 78)
    say("permutation 5x6 d12 cap 28 k=512")
    run = contraction(circ, words, cap=28, batch=2, trials=4)
    got = run.amplitudes()
    ref = closed_forms.permutation_amplitudes(circ, words)
    assert_close(got, ref, 1e-5)
    run.close()


def test_c2_full_config_against_stored_oracle():
    """5x6 depth-12, 4096 bitstrings, cap 28 (all slices): the seeded
    256-bitstring subset against the stored FP64 state-vector amplitudes."""
    import json
    import os
    require_gpu()
    w = CONFIGS["C2"]
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_subset.json")))
    circ, words = w.circuit(), w.bitstrings()
    idx = np.array(g["indices"])
    assert [str(int(x)) for x in words[idx]] == g["words"]
    ref = np.array([complex(a, b) for a, b in g["amps"]])
    say("C2 full config, cap 28, k=4096, batch 4")
    run = contraction(circ, words, cap=28, batch=4, trials=4)
    got = run.amplitudes()[idx]
    assert_close(got, ref, 1e-5)
    n = 30
    assert abs((np.ldexp(np.mean(np.abs(got) ** 2), n) - 1) - (np.ldexp(np.mean(np.abs(ref) ** 2), n) - 1)) <= 1e-4
    run.close()


@pytest.mark.parametrize("precision", ["c64", "chalf"])
def test_key_chunks_match_single_pass(precision):
    # a memory budget below the breadth-first workspace splits the batch into
    # trie-ordered key chunks; every instance is computed by the same kernel
    # on the same operands, so the amplitudes are bit-identical
    torch = require_gpu()
    from paper_2212_04749_amd import api, planner
    from paper_2212_04749_amd.circuit_tn import build_network
    circ = random_circuit(GridSpec(4, 4), 12, 21)
    words = uniform_bitstrings(16, 1024, 22)
    words[5] = words[900]  # a repeated bitstring lands in one chunk's row list twice
    opens = (3, 9)
    net = build_network(circ)
    pl = planner.find_plan(net, words, opens, 14, trials=4)
    spec = api.PlanSpec(pl.pairs, pl.sliced, opens, 14)
    say(f"key chunks {precision}")
    one = api.Contraction(net, spec, words, precision=precision, slice_batch=2)
    assert one.info.n_chunks == 1
    budget = int(0.7 * one.info.workspace_bytes)
    many = api.Contraction(net, spec, words, precision=precision, slice_batch=2, memory_budget=budget)
    assert many.info.n_chunks >= 2 and many.info.workspace_bytes <= budget
    a = one.execute()
    one.synchronize()
    b = many.execute()
    many.synchronize()
    assert torch.equal(a, b)
    psi = statevector.final_state(circ)
    full = []
    for w0 in words:
        for j in range(4):
            word = int(w0)
            for t, q in enumerate(opens):
                word = (word & ~(1 << q)) | (((j >> t) & 1) << q)
            full.append(word)
    ref = statevector.amplitudes_from_state(psi, full)
    got = b.cpu().numpy()
    assert_close(got[..., 0] + 1j * got[..., 1], ref, (3e-3 if precision == "chalf" else 1e-5))
    one.close()
    many.close()


@pytest.mark.parametrize("grid,depth,cap,k,seed,precision", [
    ((4, 4), 10, 12, 512, 21, "c64"),
    ((4, 5), 14, None, 1024, 8, "c64"),
    ((4, 5), 14, None, 1024, 8, "chalf"),
])
def test_fan_out_tiles_against_statevector(grid, depth, cap, k, seed, precision):
    # plans whose gathered steps run as fan-out MFMA tiles (the output
    # instances sharing an A instance as one GEMM), before and after the
    # tile autotuner has timed every fitting configuration
    require_gpu()
    n = grid[0] * grid[1]
    circ = random_circuit(GridSpec(*grid), depth, seed)
    words = uniform_bitstrings(n, k, seed + 1)
    ref = statevector.amplitudes(circ, words)
    say(f"fan-out {grid} d{depth} k={k} {precision}")
    run = contraction(circ, words, cap=cap, batch=2, precision=precision, trials=4)
    assert run.info.n_fan_nodes >= 1
    bar = 3e-3 if precision == "chalf" else 1e-5
    assert_close(run.amplitudes(), ref, bar)
    run.autotune(reps=1, cache_path="")
    assert_close(run.amplitudes(), ref, bar)
    assert abs(run.xeb() - oxeb.linear_xeb(ref, n)) <= 1e-4
    run.close()
