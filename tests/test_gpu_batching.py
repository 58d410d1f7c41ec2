"""Batching features: slice batches replayed from a captured HIP graph, the
MFMA tile autotuner, and the graph-captured queue of uneven plans.

Graph replays are compared bit for bit with eager launches of the same
kernels (a plan bound to the null stream is never captured), with eager work
and synchronisation between the replays; every replay is checked.
"""

import json
import os

import numpy as np
import pytest

from gpu_util import assert_close, rel_err, require_gpu, say
from oracle import statevector, xeb as oxeb
from workload import GridSpec, random_circuit, uniform_bitstrings

pytestmark = pytest.mark.gpu


def build(circ, words, cap, batch, precision="c64", stream=None, spec=None):
    from paper_2212_04749_amd import api, planner
    from paper_2212_04749_amd.circuit_tn import build_network
    net = build_network(circ)
    if spec is None:
        pl = planner.find_plan(net, words, (), cap, trials=4)
        spec = api.PlanSpec(pl.pairs, pl.sliced, (), cap if cap is not None else 32)
    return api.Contraction(net, spec, words, precision=precision, slice_batch=batch, stream=stream), spec


@pytest.mark.parametrize("precision", ["c64", "chalf"])
def test_graph_replays_match_eager(precision):
    torch = require_gpu()
    circ = random_circuit(GridSpec(3, 4), 8, 5)
    words = uniform_bitstrings(12, 64, 6)
    say(f"graph vs eager {precision}")
    g_run, spec = build(circ, words, 7, 4, precision)
    e_run, _ = build(circ, words, 7, 4, precision, stream=torch.cuda.default_stream(), spec=spec)
    assert g_run.n_slices >= 8
    eager = e_run.execute()
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    for rep in range(4):
        got = g_run.execute()
        g_run.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref), f"replay {rep}"
        del junk
    g_run.close()
    e_run.close()


@pytest.mark.parametrize("precision", ["c64", "chalf"])
def test_timed_execute_matches_graph_pass(precision):
    # the event-timed pass launches the same kernels one by one: bit-identical
    # amplitudes to the graph replay; a slice-dependent step is timed once per
    # slice batch, an invariant one once on a cold stem cache and never after
    torch = require_gpu()
    circ = random_circuit(GridSpec(3, 4), 8, 5)
    words = uniform_bitstrings(12, 64, 6)
    say(f"timed execute {precision}")
    run, _ = build(circ, words, 7, 4, precision)
    ref = run.execute()
    run.synchronize()
    ref = ref.cpu().numpy()
    dep = run.step_dep()
    prof = run.profile()
    n_batches = -(-run.n_slices // run.slice_batch)
    j_dep = max((j for j in range(len(dep)) if dep[j]), key=lambda j: prof[j][0])
    j_inv = next((j for j in range(len(dep)) if not dep[j] and prof[j][0] >= 0), None)
    for j in [j_dep] + ([j_inv] if j_inv is not None else []):
        run.reset_cache()
        amps = run.new_amplitudes()
        ms, n = run.execute_timed(amps, j)
        assert np.array_equal(amps.cpu().numpy(), ref), f"step {j}"
        if dep[j]:
            assert n == n_batches * run.info.n_chunks, (j, n)
        else:
            assert n in (1, run.info.n_chunks), (j, n)
        assert ms > 0.0
        # warm stem cache: a cached invariant step is not launched again (one
        # wider than a key chunk is, once per chunk)
        amps.zero_()
        ms2, n2 = run.execute_timed(amps, j)
        assert np.array_equal(amps.cpu().numpy(), ref)
        assert n2 == n if dep[j] else n2 in (0, run.info.n_chunks)
    say(f"timed steps {j_dep} (slice-dependent), {j_inv} (invariant)")
    run.close()


def test_autotune_keeps_parity_and_writes_cache(tmp_path):
    require_gpu()
    from paper_2212_04749_amd import binding as B
    circ = random_circuit(GridSpec(4, 4), 10, 21)
    words = uniform_bitstrings(16, 128, 22)
    ref = statevector.amplitudes(circ, words)
    say("autotune 4x4 d10")
    run, _ = build(circ, words, 12, 4)
    path = str(tmp_path / "tune.json")
    run.autotune(reps=2, cache_path=path)
    got = run.amplitudes()
    assert_close(got, ref, 1e-5)
    if run.info.n_mfma_nodes:
        table = json.load(open(path))
        assert table and all(isinstance(v, int) for v in table.values())
        # a second plan reads its choices from the cache
        run2, _ = build(circ, words, 12, 4)
        run2.autotune(reps=2, cache_path=path)
        assert_close(run2.amplitudes(), ref, 1e-5)
        run2.close()
    run.close()


def test_queue_of_uneven_plans():
    torch = require_gpu()
    from paper_2212_04749_amd import api
    stream = torch.cuda.Stream()
    cases = [(GridSpec(3, 3), 6, 31, 40, None), (GridSpec(3, 4), 8, 32, 96, 8), (GridSpec(2, 5), 10, 33, 17, 6),
             (GridSpec(4, 4), 8, 34, 256, 12)]
    runs, refs = [], []
    for spec, depth, seed, k, cap in cases:
        circ = random_circuit(spec, depth, seed)
        n = spec.rows * spec.cols
        words = uniform_bitstrings(n, k, seed + 100)
        r, _ = build(circ, words, cap, 2, stream=stream)
        runs.append(r)
        refs.append((statevector.amplitudes(circ, words), n))
    say("queue of 4 plans")
    q = api.Queue(runs)
    first = None
    for rep in range(3):
        amps, xeb = q.execute()
        stream.synchronize()
        xs = xeb.cpu().numpy()
        for i, (a, (ref, n)) in enumerate(zip(amps, refs)):
            c = a.cpu().numpy()
            c = c[..., 0, 0] + 1j * c[..., 0, 1]
            assert_close(c, ref, 1e-5)
            assert abs(xs[i] - oxeb.linear_xeb(ref, n)) <= 1e-4
        snap = [a.cpu().numpy() for a in amps]
        if first is None:
            first = snap
        else:
            assert all(np.array_equal(x, y) for x, y in zip(first, snap))
    q.close()
    for r in runs:
        r.close()
