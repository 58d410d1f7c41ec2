"""matnc_plan_set_tensor: new leaf data on a bound plan (same structure).

Two random circuits on the same grid and depth (different seeds) have fused
networks with identical index lists, so a plan made for circuit A computes
circuit B once B's leaves are swapped in.  Checked against the oracle's
state vector of each circuit, in both precisions, through direct execution
(graph replays of a full slice batch and eager partial batches) and through
a queue, across swaps in both directions.
"""

import numpy as np
import pytest

from gpu_util import assert_close, require_gpu, say
from oracle import statevector, xeb as oxeb
from workload import GridSpec, random_circuit, uniform_bitstrings

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("c64", 1e-5), ("chalf", 3e-3)])
def test_set_tensor_swaps_circuits(precision, tol):
    torch = require_gpu()
    from paper_2212_04749_amd import api
    from paper_2212_04749_amd.circuit_tn import build_network
    grid, depth = GridSpec(3, 5), 10
    ca, cb = random_circuit(grid, depth, 61), random_circuit(grid, depth, 62)
    na, nb = build_network(ca), build_network(cb)
    assert na.indices == nb.indices
    words = uniform_bitstrings(15, 300, 63)
    ref_a, ref_b = statevector.amplitudes(ca, words), statevector.amplitudes(cb, words)
    stream = torch.cuda.Stream()
    run = api.Contraction.from_circuit(ca, words, cap=9, precision=precision, slice_batch=4, trials=4,
                                       stream=stream)
    say(f"set_tensor {precision}: {run.n_slices} slices, batch 4")
    assert run.n_slices >= 8
    amps = run.new_amplitudes()
    run.execute(amps)   # captures the batch graphs for this buffer
    run.synchronize()
    a = amps.cpu().numpy()
    assert_close(a[:, 0, 0] + 1j * a[:, 0, 1], ref_a, tol, "circuit A")
    for t, x in enumerate(nb.tensors):
        run.set_tensor(t, x)
    # same buffer: the captured graphs are replayed with the new leaves (and
    # the stem cache is recomputed); a split range mixes graphs and eager
    # partial batches
    with torch.cuda.stream(stream):
        amps.zero_()
    cut = 5
    run.execute(amps, 0, cut)
    run.execute(amps, cut, run.n_slices)
    run.synchronize()
    a = amps.cpu().numpy()
    got_b = a[:, 0, 0] + 1j * a[:, 0, 1]
    e = assert_close(got_b, ref_b, tol, "circuit B")
    say(f"set_tensor {precision}: circuit B rel err {e:.2e}")
    assert abs(run.xeb(amps) - oxeb.linear_xeb(ref_b, 15)) <= 1e-4
    # through a queue (one captured graph with prologue, slices, sums, XEB)
    q = api.Queue([run])
    qa, qx = q.execute()
    stream.synchronize()
    first = qa[0].cpu().numpy()
    assert_close(first[:, 0, 0] + 1j * first[:, 0, 1], ref_b, tol, "queue, circuit B")
    assert abs(float(qx.cpu()[0]) - oxeb.linear_xeb(ref_b, 15)) <= 1e-4
    for t, x in enumerate(na.tensors):
        run.set_tensor(t, x)
    q.execute(qa, qx)
    stream.synchronize()
    back = qa[0].cpu().numpy()
    assert_close(back[:, 0, 0] + 1j * back[:, 0, 1], ref_a, tol, "queue, circuit A again")
    assert abs(float(qx.cpu()[0]) - oxeb.linear_xeb(ref_a, 15)) <= 1e-4
    q.close()
    run.close()

