"""Pins of the multi-amplitude cost figures and of the native oracle.

* Table I of the paper prints, per depth, the flop counts of single- and
  multi-amplitude contraction and the ideal speedup; the ideal speedup is
  k * FPOs(single) / FPOs(multi) (k = one million), the quantity the plan
  reports as k S / S_k (tests/golden/table_speedup.json).
* S_k brute force: every bitstring's own single-amplitude tree visits each
  node v with its projection b|O(v); the distinct (v, projection) pairs,
  each costing CMAC(v), add up to the library's S_k (Eq. (1) with optimal
  reuse), and S (one bitstring) to its single-amplitude cost.
* The plain-C state vector equals the numpy one.
"""

import json
import os

import numpy as np

from oracle import statevector, sv_native
from workload import GridSpec, random_circuit, uniform_bitstrings

HERE = os.path.dirname(os.path.abspath(__file__))


def test_ideal_speedup_column_of_table_one():
    g = json.load(open(os.path.join(HERE, "golden", "table_speedup.json")))
    for row in g["rows"]:
        ideal = g["k"] * row["fpos_single"] / row["fpos_multi"]
        # the table rounds its flop counts to two digits
        assert abs(ideal - row["ideal_speedup"]) / row["ideal_speedup"] < 0.005


def test_multi_amplitude_cost_by_brute_force():
    from paper_2212_04749_amd import api, binding as B, planner as P
    from paper_2212_04749_amd.circuit_tn import build_network
    circ = random_circuit(GridSpec(3, 4), 8, 17)
    words = uniform_bitstrings(12, 40, 18)
    net = build_network(circ)
    pl = P.find_plan(net, words, (), None, trials=2)
    # brute force over bitstrings: which nodes see which projections
    n = len(net.indices)
    out_of = {net.output_index[q]: q for q in range(net.n_qubits)}
    leaf_idx = [set(ix) for ix in net.indices]
    below = [{out_of[i] for i in ix if i in out_of} for ix in net.indices]
    free = [set(i for i in ix if i not in out_of) for ix in net.indices]
    pairs_seen = set()
    cmac = {}
    for j, (a, b) in enumerate(pl.pairs):
        v = n + j
        below.append(below[a] | below[b])
        cmac[v] = 2 ** len(free[a] | free[b])
        free.append(free[a] ^ free[b])
    for w in words:
        for v in range(n, n + len(pl.pairs)):
            proj = tuple(sorted((q, (int(w) >> q) & 1) for q in below[v]))
            pairs_seen.add((v, proj))
    s_k = sum(cmac[v] for v, _ in pairs_seen)
    s_1 = sum(cmac.values())
    ranks, ids, data = api.network_arrays(net)
    h = B.matnc_network_create(ranks, ids, data, net.n_qubits, net.output_index)
    p = B.matnc_plan_create(h, pl.pairs, [], [], words, 0, 32, 1)
    info = B.matnc_plan_info(p)
    assert info.cmac_multi == s_k
    assert info.cmac_single == s_1
    assert s_k < len(set(int(x) for x in words)) * s_1  # reuse saves work
    B.matnc_plan_destroy(p)
    B.matnc_network_destroy(h)


def test_native_statevector_matches_numpy():
    circ = random_circuit(GridSpec(3, 4), 9, 23)
    words = uniform_bitstrings(12, 200, 24)
    a = statevector.amplitudes(circ, words)
    b = sv_native.amplitudes(circ, words)
    assert np.max(np.abs(a - b)) < 1e-14


def test_slice_refiner_reaches_a_local_optimum_of_the_multi_amplitude_loss():
    # from the worst valid sliced set of the slicer's size, the refiner must
    # end at a valid set whose loss is no higher, no lower than the
    # brute-force best set, and that no single exchange improves
    import itertools
    from paper_2212_04749_amd import planner as P
    from paper_2212_04749_amd.circuit_tn import build_network
    from workload import GridSpec, random_circuit, uniform_bitstrings
    net = build_network(random_circuit(GridSpec(3, 3), 8, 31))
    words = uniform_bitstrings(9, 24, 32)
    st = P.Structure.from_network(net)
    pairs = P.greedy_pairs(st)
    w = P.widths(P.build_tree(st, pairs), words)
    cap = max(m.bit_count() for m in P.build_tree(st, pairs).masks) - 2
    bonds = sorted(set(i for m in st.leaf_masks for i in P._bits(m)))
    n_sl = len(P.slice_to_cap(st, pairs, w, cap, objective="flops")[0])

    def loss(sl):
        mask = sum(1 << i for i in sl)
        t = P.build_tree(st, pairs, mask)
        if max(m.bit_count() for m in t.masks) > cap:
            return None
        return P.costs(st, t, w, mask).total

    valid = [(loss(c), c) for c in itertools.combinations(bonds, n_sl)]
    valid = [(v, c) for v, c in valid if v is not None]
    best = min(v for v, _ in valid)
    start_loss, start = max(valid)
    s2, c2 = P.refine_slices(st, pairs, w, list(start), cap, objective="flops", exact=True)
    assert len(s2) == n_sl and loss(s2) == c2.total
    assert best <= c2.total < start_loss
    for pos in range(n_sl):
        for j in bonds:
            if j in s2:
                continue
            trial = list(s2)
            trial[pos] = j
            v = loss(trial)
            assert v is None or v >= c2.total * (1 - 1e-9)


def test_complex_half_budget_time_estimate():
    # the complex-half time estimate under a precision budget N prices the N
    # steps with the most estimated complex64 time at complex-half rates and
    # the rest at complex64 rates: N = 0 is the complex64 estimate, N at or
    # above the step count the all-FP16 one, and each step moved between
    # the two changes the total by its own difference
    from paper_2212_04749_amd import planner as P
    from paper_2212_04749_amd.circuit_tn import build_network
    net = build_network(random_circuit(GridSpec(4, 4), 10, 3))
    words = uniform_bitstrings(16, 300, 9)
    pl = P.find_plan(net, words, (), 10, seed=0, trials=2)
    st = P.Structure.from_network(net, ())
    mask = sum(1 << i for i in pl.sliced)
    tree = P.build_tree(st, pl.pairs, mask)
    w = P.widths(P.build_tree(st, pl.pairs), words)

    def est(*model):
        with P.time_model(*model):
            return P.costs(st, tree, w, mask).time

    def per_step(model):
        n, nsl, dep, out = st.n_tensors, bin(mask).count("1"), [bool(m & mask) for m in st.leaf_masks], []
        for j, (a, b) in enumerate(tree.pairs):
            dep.append(dep[a] or dep[b])
            ra, rb, wa, wb = tree.masks[a].bit_count(), tree.masks[b].bit_count(), w[a], w[b]
            if rb > ra:
                ra, rb, wa, wb = rb, ra, wb, wa
            with P.time_model(model):
                t = P.step_time(w[n + j], wa, wb, ra, rb, tree.masks[n + j].bit_count(),
                                (tree.masks[a] & tree.masks[b]).bit_count())
            out.append(t * (2.0 ** nsl if dep[-1] else 1.0))
        return out

    t32, t16 = per_step("c64"), per_step("chalf")
    assert np.isclose(est("c64"), sum(t32)) and np.isclose(est("chalf"), sum(t16))
    assert np.isclose(est("chalf", 0), sum(t32)) and np.isclose(est("chalf", len(t32)), sum(t16))
    order = sorted(range(len(t32)), key=lambda i: -t32[i])
    for N in (1, 3, 5):
        want = sum(t32) + sum(t16[i] - t32[i] for i in order[:N])
        assert np.isclose(est("chalf", N), want)
    # the budget never prices a step above its complex64 time here
    assert est("chalf", 5) <= est("chalf", 0) + 1e-12
    # the default model is restored after the block
    assert np.isclose(est("c64"), P.costs(st, tree, w, mask).time)
