"""CPU checks of the C ABI: exports, plan figures and error paths.

No kernel runs here: plan creation and its validation are host code.
"""

import math
import os
import re

import numpy as np
import pytest

from paper_2212_04749_amd import api, binding as B, planner as P
from paper_2212_04749_amd.circuit_tn import build_network
from workload import CONFIGS, GridSpec, random_circuit, uniform_bitstrings

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "matnc.h")).read()
    return sorted(set(re.findall(r"\b(matnc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = header_functions()
    assert "matnc_execute" in names and len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert B.matnc_version().startswith("matnc ")


def _plan(circ, words, opens=(), cap=None, trials=4, batch=1, precision=0):
    net = build_network(circ)
    pl = P.find_plan(net, words, opens, cap, trials=trials)
    ranks, ids, data = api.network_arrays(net)
    h = B.matnc_network_create(ranks, ids, data, net.n_qubits, net.output_index)
    p = B.matnc_plan_create(h, pl.pairs, pl.sliced, list(opens), words, precision, cap or 32, batch)
    return net, pl, h, p


def test_plan_costs_match_planner():
    w = CONFIGS["C1"]
    net, pl, h, p = _plan(w.circuit(), w.bitstrings())
    info = B.matnc_plan_info(p)
    assert info.cmac_single == pl.costs.S
    assert info.cmac_multi == pl.costs.S_k
    assert info.max_rank == pl.costs.max_rank
    assert info.n_amplitudes == 64
    B.matnc_plan_destroy(p)
    B.matnc_network_destroy(h)


def test_sliced_costs_and_workspace_growth():
    circ = random_circuit(GridSpec(3, 4), 8, 5)
    words = uniform_bitstrings(12, 50, 6)
    net, pl, h, p1 = _plan(circ, words, cap=7)
    i1 = B.matnc_plan_info(p1)
    assert i1.n_slices == 2 ** len(pl.sliced) and i1.max_rank <= 7
    assert math.isclose(i1.cmac_total, pl.costs.total)
    p4 = B.matnc_plan_create(h, pl.pairs, pl.sliced, [], words, 0, 7, 4)
    i4 = B.matnc_plan_info(p4)
    assert i4.workspace_bytes >= i1.workspace_bytes
    for p in (p1, p4):
        B.matnc_plan_destroy(p)
    B.matnc_network_destroy(h)


def test_error_paths():
    circ = random_circuit(GridSpec(3, 3), 6, 1)
    words = uniform_bitstrings(9, 10, 2)
    net = build_network(circ)
    pl = P.find_plan(net, words, (), None, trials=2)
    ranks, ids, data = api.network_arrays(net)
    h = B.matnc_network_create(ranks, ids, data, net.n_qubits, net.output_index)
    # rank cap too small
    with pytest.raises(B.MatncError) as e:
        B.matnc_plan_create(h, pl.pairs, [], [], words, 0, 2, 1)
    assert e.value.code == B.MATNC_E_RANK
    # broken tree: a tensor used twice
    bad = [list(x) for x in pl.pairs]
    bad[1][0] = bad[0][0]
    with pytest.raises(B.MatncError) as e:
        B.matnc_plan_create(h, bad, [], [], words, 0, 32, 1)
    assert e.value.code == B.MATNC_E_INVALID
    # bit beyond n_qubits
    with pytest.raises(B.MatncError) as e:
        B.matnc_plan_create(h, pl.pairs, [], [], np.array([1 << 9], dtype=np.uint64), 0, 32, 1)
    assert e.value.code == B.MATNC_E_INVALID
    # slicing an output index is not allowed
    with pytest.raises(B.MatncError) as e:
        B.matnc_plan_create(h, pl.pairs, [net.output_index[0]], [], words, 0, 32, 1)
    assert e.value.code == B.MATNC_E_INVALID
    # repeated open qubit
    with pytest.raises(B.MatncError) as e:
        B.matnc_plan_create(h, pl.pairs, [], [2, 2], words, 0, 32, 1)
    assert e.value.code == B.MATNC_E_INVALID
    # execute before bind
    p = B.matnc_plan_create(h, pl.pairs, [], [], words, 0, 32, 1)
    with pytest.raises(B.MatncError) as e:
        B.matnc_execute(p, 0, 1, 0x1000)
    assert e.value.code == B.MATNC_E_STATE
    assert "bind" in B.matnc_last_error()
    with pytest.raises(B.MatncError) as e:
        B.matnc_execute_timed(p, 0, 1, 0x1000, 0)
    assert e.value.code == B.MATNC_E_STATE
    # set_tensor: tensor id out of range; a valid id on an unbound plan only
    # replaces the host copy (uploaded at bind)
    with pytest.raises(B.MatncError) as e:
        B.matnc_plan_set_tensor(p, len(net.tensors), np.zeros(32))
    assert e.value.code == B.MATNC_E_INVALID
    B.matnc_plan_set_tensor(p, 0, api.tensor_array(net.tensors[0]))
    with pytest.raises(ValueError):
        B.matnc_plan_set_tensor(p, 0, np.zeros(3))
    B.matnc_plan_destroy(p)
    # network: bond index on three tensors
    with pytest.raises(B.MatncError) as e:
        B.matnc_network_create([1, 1, 1], [5, 5, 5], np.zeros(12), 1, [7])
    assert e.value.code == B.MATNC_E_INVALID
    B.matnc_network_destroy(h)


def test_width_law_for_uniform_batches():
    # Table S3's widths follow the occupancy law E[w] = 2^m (1 - (1 - 2^-m)^k)
    # of uniform bitstrings (checked to <1% for k = 3e6); the reuse widths of
    # a uniform batch follow it too
    k = 3_000_000
    rows = [(3, 8), (4, 16), (5, 32), (10, 1024), (14, 16384), (16, 65536), (20, 981285),
            (22, 2123441), (24, 2737958), (26, 2931054), (27, 2965352), (29, 2991260),
            (30, 2995698), (31, 2997840), (33, 2999468), (34, 2999722)]
    for m, w in rows:
        law = 2.0 ** m * (1 - (1 - 2.0 ** -m) ** k)
        assert abs(law - w) / w < 0.01
    # same law on our widths: a node with m outputs over a uniform batch
    words = uniform_bitstrings(30, 4096, 3)
    for m in (4, 8, 12, 16):
        mask = np.uint64((1 << m) - 1)
        wv = np.unique(words & mask).size
        law = 2.0 ** m * (1 - (1 - 2.0 ** -m) ** 4096)
        assert abs(wv - law) / law < 0.05


def test_contract_pair_batch_counts_complex_elements():
    # regression: a float32 view holds two floats per complex element, so the
    # batch must come from the byte size, and mismatched operands are refused
    # before any launch
    torch = pytest.importorskip("torch")
    nm, nn, nk = 4, 2, 2
    pos = {"posA_m": [0, 1, 2, 3], "posA_k": [4, 5], "posB_k": [0, 1], "posB_n": [2, 3],
           "posC_m": [0, 1, 2, 3], "posC_n": [4, 5]}
    A = torch.zeros(3, 2 << (nm + nk), dtype=torch.float32)
    Bt = torch.zeros(3, 2 << (nn + nk), dtype=torch.float32)
    C = torch.zeros(3, 2 << (nm + nn), dtype=torch.float32)
    with pytest.raises(ValueError, match="device"):
        api.contract_pair(A, Bt, C, pos)          # sizes agree: only the device check fails
    with pytest.raises(ValueError, match="sizes"):
        api.contract_pair(A, Bt[:2], C, pos)      # B holds 2 instances, A 3
    with pytest.raises(ValueError, match="sizes"):
        api.contract_pair(A[:, :-2], Bt, C, pos)  # A not a whole number of instances


def test_memory_budget_splits_keys_into_chunks():
    # a budget below the breadth-first workspace splits the bitstrings into
    # trie-ordered chunks; a budget no single key fits in is refused
    circ = random_circuit(GridSpec(4, 4), 12, 21)
    words = uniform_bitstrings(16, 1024, 22)
    net, pl, h, p1 = _plan(circ, words, cap=14, batch=2)
    full = B.matnc_plan_info(p1)
    assert full.n_chunks == 1
    budget = int(0.7 * full.workspace_bytes)
    p2 = B.matnc_plan_create(h, pl.pairs, pl.sliced, [], words, 0, 14, 2, budget)
    part = B.matnc_plan_info(p2)
    assert part.n_chunks >= 2 and part.workspace_bytes <= budget
    assert part.cmac_multi == full.cmac_multi and part.n_unique == full.n_unique
    with pytest.raises(B.MatncError) as e:
        B.matnc_plan_create(h, pl.pairs, pl.sliced, [], words, 0, 14, 2, 4096)
    assert e.value.code == B.MATNC_E_NOMEM
    for p in (p1, p2):
        B.matnc_plan_destroy(p)
    B.matnc_network_destroy(h)


def test_memory_cap_bounds_multi_amplitude_tensors():
    # the rank cap bounds one instance of a tensor; the memory cap bounds the
    # w(v) instances the device holds for node v
    circ = random_circuit(GridSpec(3, 4), 8, 5)
    words = uniform_bitstrings(12, 200, 6)
    net = build_network(circ)
    st = P.Structure.from_network(net, ())

    def biggest(pl):
        tree = P.build_tree(st, pl.pairs, sum(1 << i for i in pl.sliced))
        w = P.widths(tree, words)
        return max(math.log2(w[v]) + tree.masks[v].bit_count() for v in range(len(tree.masks)))

    free = P.find_plan(net, words, (), None, trials=4)
    assert biggest(free) > 10
    capped = P.find_plan(net, words, (), None, trials=4, mem_cap=10)
    assert biggest(capped) <= 10 + 1e-9
    assert len(capped.sliced) >= 1


def _check_stored_plan(w, e):
    net = build_network(w.circuit())
    words = w.bitstrings()
    opens = list(e.get("open_qubits", ()))
    st = P.Structure.from_network(net, opens)
    pairs = [tuple(x) for x in e["pairs"]]
    smask = sum(1 << i for i in e["sliced"])
    tree = P.build_tree(st, pairs, smask)
    wd = P.widths(P.build_tree(st, pairs), words)
    assert max(m.bit_count() for m in tree.masks) <= e["cap"]
    if "mem_cap" in e:
        assert max(math.log2(wd[v]) + tree.masks[v].bit_count() for v in range(len(tree.masks))) <= e["mem_cap"] + 1e-9
    ranks, ids, data = api.network_arrays(net)
    h = B.matnc_network_create(ranks, ids, data, net.n_qubits, net.output_index)
    p = B.matnc_plan_create(h, pairs, e["sliced"], opens, words, 0, e["cap"], 1)
    info = B.matnc_plan_info(p)
    assert info.n_slices == 2 ** len(e["sliced"]) and info.max_rank <= e["cap"]
    assert math.isclose(info.cmac_total, e["cmac_total"], rel_tol=1e-9)
    B.matnc_plan_destroy(p)
    B.matnc_network_destroy(h)


def test_stored_plans_are_valid_library_inputs():
    # the stored trees of the 6x6 and 53-qubit workloads and of the uneven
    # batch meet their rank and memory caps, and the library's cost figures
    # agree with the planner's
    from paper_2212_04749_amd.plans import make_c3, make_c4, make_c5
    from workload.configs import uneven_batch_c5
    _check_stored_plan(CONFIGS["C3"], make_c3.load())
    _check_stored_plan(CONFIGS["C4"], make_c4.load())
    plans = make_c5.load()
    for w in uneven_batch_c5():
        _check_stored_plan(w, plans[w.name])


def test_c_program_uses_the_abi(tmp_path):
    # the boundary from plain C: include/matnc.h + libmatnc.so, host calls
    # only (network, plan, figures, an invalid tree, execute before bind)
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    B.lib()  # built
    libdir = os.path.join(ROOT, "paper_2212_04749_amd")
    exe = str(tmp_path / "plan_info")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi", "plan_info.c"), "-L", libdir, "-lmatnc",
                    f"-Wl,-rpath,{libdir}", "-o", exe], check=True, capture_output=True, text=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120).stdout
    assert "n_amplitudes 4 n_unique 4 n_slices 1 n_nodes 1 max_rank 1" in out
    # S = 2^|{bond}| = 2 complex MACs per amplitude; S_k = 4 keys x 2
    assert "cmac_single 2.0 cmac_multi 8.0" in out
    assert f"bad tree rc {B.MATNC_E_INVALID} (invalid) message present" in out
    assert f"execute before bind rc {B.MATNC_E_STATE}" in out


def test_queue_workspace_is_one_arena_plus_static_regions():
    # plans of a queue share one arena: the queue needs more than its largest
    # plan (every static region) but less than all plans side by side
    ps, hs = [], []
    for seed in (21, 22, 23):
        circ = random_circuit(GridSpec(3, 4), 8, seed)
        net, pl, h, p = _plan(circ, uniform_bitstrings(12, 40, seed + 100), cap=8)
        ps.append(p)
        hs.append(h)
    q = B.matnc_queue_create(ps)
    need = B.matnc_queue_workspace_bytes(q)
    sizes = [int(B.matnc_plan_info(p).workspace_bytes) for p in ps]
    assert max(sizes) < need < sum(sizes)
    with pytest.raises(B.MatncError) as e:
        B.matnc_queue_bind(q, 0x1000, need - 256, 0)
    assert e.value.code == B.MATNC_E_NOMEM
    B.matnc_queue_destroy(q)
    for p in ps:
        B.matnc_plan_destroy(p)
    for h in hs:
        B.matnc_network_destroy(h)
