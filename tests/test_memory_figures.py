"""M^BFT and M^DFT of the reuse tree (Supplementary Sec. III.C) against an
explicit traversal of the reuse tree, built here from the bitstrings and a
path-shaped contraction order without the planner's helpers: the stem, the
ranks, the prefixes at every step and the live tensors of both traversals."""

import numpy as np
import pytest

from paper_2212_04749_amd import planner
from paper_2212_04749_amd.circuit_tn import build_network
from workload import GridSpec, random_circuit, uniform_bitstrings


def _network(seed):
    net = build_network(random_circuit(GridSpec(3, 3), 8, seed))
    return net, planner.Structure.from_network(net, ())


def _path_pairs(n):
    # leaf 0, then absorb leaves 1, 2, ... one by one
    return [(0, 1)] + [(n + i, i + 2) for i in range(n - 2)]


def _explicit(st, words):
    n = st.n_tensors
    idx, outs = st.leaf_masks[0], st.leaf_outputs[0]
    steps = [(idx, outs)]
    for t in range(1, n):
        idx ^= st.leaf_masks[t]
        outs |= st.leaf_outputs[t]
        steps.append((idx, outs))
    words = [int(x) for x in words]
    prefixes = [sorted({x & o for x in words}) for _, o in steps]
    layers = [j for j in range(1, n) if len(prefixes[j]) > len(prefixes[j - 1])]
    size = {j: 1 << bin(steps[j - 1][0]).count("1") for j in layers}
    # breadth first: every prefix before the branching step holds its tensor
    bft = max((len(prefixes[j - 1]) * size[j] for j in layers), default=0)
    # depth first: a trie node holds its tensor while its subtree is walked
    live, peak = 0, 0

    def visit(li, prefix):
        nonlocal live, peak
        j = layers[li]
        live += size[j]
        peak = max(peak, live)
        if li + 1 < len(layers):
            before = steps[j - 1][1]
            nxt = steps[layers[li + 1] - 1][1]
            for c in sorted({x & nxt for x in words if x & before == prefix}):
                visit(li + 1, c)
        live -= size[j]

    if layers:
        for p in prefixes[layers[0] - 1]:
            visit(0, p)
    return [(len(prefixes[j - 1]), bin(steps[j - 1][0]).count("1")) for j in layers], bft, peak


@pytest.mark.parametrize("seed,k", [(1, 40), (2, 200), (3, 512)])
def test_memory_figures_match_explicit_traversal(seed, k):
    net, st = _network(seed)
    words = uniform_bitstrings(9, k, 50 + seed) if k < 512 else np.arange(512, dtype=np.uint64)
    tree = planner.build_tree(st, _path_pairs(st.n_tensors))
    assert planner.stem_path(tree) == [0] + list(range(st.n_tensors, st.n_tensors + len(tree.pairs)))
    m = planner.memory_figures(tree, words)
    layers, bft, dft = _explicit(st, words)
    assert m["layers"] == layers
    assert m["M_BFT"] == bft and m["M_DFT"] == dft
    assert len(layers) >= 2 and m["M_DFT"] <= len(layers) * max(1 << d for _, d in layers)


def test_full_batch_layer_widths_are_powers_of_two():
    # with all 2^9 bitstrings every prefix occurs, so the number of reuse-tree
    # nodes before a branching is 2 to the number of closed outputs absorbed
    # so far (the paper's all-amplitude example has w_l = 2^(l-1))
    net, st = _network(4)
    words = np.arange(512, dtype=np.uint64)
    tree = planner.build_tree(st, _path_pairs(st.n_tensors))
    s = planner.stem_path(tree)
    m = planner.memory_figures(tree, words)
    branch_points = [s[j - 1] for j in range(1, len(s)) if tree.outputs[s[j]] != tree.outputs[s[j - 1]]]
    assert [w for w, _ in m["layers"]] == [1 << bin(tree.outputs[v]).count("1") for v in branch_points]
    assert m["layers"][0][0] == 1 or tree.outputs[s[0]] != 0


def test_single_bitstring_has_no_branching_and_searched_trees_have_a_stem():
    # one amplitude: the reuse tree is a path, nothing is stored for reuse;
    # on a searched (not path-shaped) tree the stem is a root-to-leaf path
    net, st = _network(5)
    words = uniform_bitstrings(9, 64, 7)
    one = planner.memory_figures(planner.build_tree(st, _path_pairs(st.n_tensors)), words[:1])
    assert one == {"layers": [], "M_BFT": 0, "M_DFT": 0}
    pl = planner.find_plan(net, words, (), None, seed=0, trials=4)
    tree = planner.build_tree(st, pl.pairs)
    s = planner.stem_path(tree)
    assert s[-1] == tree.root and s[0] < st.n_tensors
    n = st.n_tensors
    for child, parent in zip(s, s[1:]):
        assert child in tree.pairs[parent - n]
    m = planner.memory_figures(tree, words)
    assert m["M_DFT"] <= m["M_BFT"] * len(m["layers"])
