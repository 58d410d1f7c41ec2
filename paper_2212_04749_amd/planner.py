"""Host planner: contraction order (TNCO), first-level slicing and cost model.

Inputs are the fused network from ``circuit_tn``, the set of open qubits and
the bitstring batch.  Outputs are an SSA pair list (ids >= n_tensors are
intermediates), a list of sliced index ids, and the cost figures of the
multi-amplitude method:

* CMAC(v) = 2^|idx(A) u idx(B)|, the complex multiply-adds of one instance of
  the pairwise step at tree node v (every index has dimension 2);
* w(v) = number of distinct projections of the bitstring batch onto the closed
  output qubits below v (the width of the reuse tree at that step,
  Eq. (1) and Supplementary Sec. III.B); on a path-shaped order this is the
  layer width w_l of Eq. (1);
* S = sum_v CMAC(v) (single-amplitude cost) and S_k = sum_v w(v) CMAC(v)
  (multi-amplitude cost with optimal reuse, Eq. (1));
* with a sliced set, nodes that see no sliced index run once, the others once
  per slice;
* M^BFT and M^DFT (Supplementary Sec. III.C), the memory of the breadth- and
  depth-first traversals of the reuse tree along the tree's stem
  (``memory_figures``).

Order search.  The paper searches orders with the multi-amplitude cost S_k
as the loss (Supplementary Sec. IV.A).  Here a seeded randomised search
builds candidate trees in two phases -- first the tensors without a closed
output index (the dark part, which becomes the stem/trunk), then the bright
tensors absorbed one by one with the step cost w(out) * CMAC -- slices each
candidate to the rank cap and keeps the one with the lowest total cost.  The
deterministic greedy order (contract the connected pair minimising
size(out) - size(A) - size(B), ties to the smaller CMAC and then the lowest
id pair) is also available and is one of the candidates.

Slicer: while some tensor is over the cap, slice the index that most
reduces the total rank overflow above the cap (sum over tensors of
rank - cap), then the one with the lowest total cost (slice-invariant nodes
once, the rest times 2^|S|), ties to the lowest index id.  The rank cap
bounds one instance; a multi-amplitude tensor holds w(v) of them, so an
optional second cap bounds log2(w(v) 2^|v|), the elements the device holds
for node v, and counts in the overflow the same way.

Objective.  ``objective="flops"`` scores plans by the paper's loss: the
complex MACs over all slices.  ``objective="time"`` (the default) scores
them by a roofline estimate of the step times on one MI355X: a step moves
eb * (w(v) 2^|v| + w(a) 2^|a| + w(b) 2^|b|) bytes and does 8 w(v) CMAC(v)
flops, and takes the longer of bytes / HBM rate and flops / arithmetic rate
(MFMA for GEMM-shaped steps, vector ALU otherwise), times 2^|S| when it is
slice-dependent.  The rates and the element size eb are those of the
precision the plan is for (``time_model``: complex64 by default, or
complex-half, whose costly steps run on FP16 MFMA with 4-byte elements).  Both count the same arithmetic; the time objective also
sees that wide steps over large tensors are bound by memory traffic, which
the flop count does not.
"""

from __future__ import annotations

import contextlib
import heapq
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .circuit_tn import TensorNetwork


def _bits(mask: int):
    while mask:
        b = mask & -mask
        yield b.bit_length() - 1
        mask ^= b


@dataclass
class Structure:
    """Index structure of a network for a given open-qubit set."""
    n_tensors: int
    leaf_masks: List[int]        # free indices per leaf (closed outputs removed)
    leaf_outputs: List[int]      # closed-output qubit mask per leaf
    open_indices: int            # mask of open output index ids
    n_qubits: int

    @classmethod
    def from_network(cls, net: TensorNetwork, open_qubits: Sequence[int] = ()) -> "Structure":
        open_set = set(open_qubits)
        closed_idx = {net.output_index[q]: q for q in range(net.n_qubits) if q not in open_set}
        masks, outs = [], []
        for ix in net.indices:
            m, o = 0, 0
            for i in ix:
                if i in closed_idx:
                    o |= 1 << closed_idx[i]
                else:
                    m |= 1 << i
            masks.append(m)
            outs.append(o)
        om = 0
        for q in open_set:
            om |= 1 << net.output_index[q]
        return cls(len(net.indices), masks, outs, om, net.n_qubits)


@dataclass
class Tree:
    pairs: List[Tuple[int, int]]
    n_tensors: int
    masks: List[int] = field(default_factory=list)     # idx(v) for all nodes (leaves first)
    outputs: List[int] = field(default_factory=list)   # O(v) qubit masks
    leafsets: List[int] = field(default_factory=list)  # bitmask of leaves below v (Python int)

    @property
    def root(self) -> int:
        return self.n_tensors + len(self.pairs) - 1 if self.pairs else 0


def build_tree(st: Structure, pairs: Sequence[Tuple[int, int]], sliced_mask: int = 0) -> Tree:
    n = st.n_tensors
    masks = [m & ~sliced_mask for m in st.leaf_masks]
    outs = list(st.leaf_outputs)
    leafsets = [1 << t for t in range(n)]
    used = [False] * (n + len(pairs))
    for a, b in pairs:
        if a == b or used[a] or used[b] or a >= len(masks) or b >= len(masks):
            raise ValueError("pairs do not form a contraction tree")
        used[a] = used[b] = True
        masks.append(masks[a] ^ masks[b])
        outs.append(outs[a] | outs[b])
        leafsets.append(leafsets[a] | leafsets[b])
    if len(pairs) != n - 1:
        raise ValueError("pairs must have n_tensors - 1 entries")
    return Tree(list(pairs), n, masks, outs, leafsets)


def widths(tree: Tree, words: np.ndarray) -> List[int]:
    """w(v): number of distinct projections of the batch onto O(v)."""
    words = np.asarray(words, dtype=np.uint64)
    cache: Dict[int, int] = {}
    out = []
    for o in tree.outputs:
        if o not in cache:
            cache[o] = 1 if o == 0 else int(np.unique(words & np.uint64(o)).size)
        out.append(cache[o])
    return out


@dataclass(frozen=True)
class TimeModel:
    """Sustained rates of the contraction kernels on one MI355X."""
    mfma: float           # flop/s of GEMM-shaped steps
    valu: float           # flop/s of streaming steps
    hbm: float            # byte/s
    elem_bytes: float     # bytes per stored complex element
    launch_s: float = 3e-6


# complex64: FP32 MFMA on the GEMM steps; complex-half: FP16 MFMA (measured
# 750 TFLOP/s on the 6x6 stem steps) and half the bytes (the costliest
# steps are the ones a complex-half plan stores in FP16)
TIME_MODELS = {
    "c64": TimeModel(mfma=100e12, valu=40e12, hbm=3.0e12, elem_bytes=8.0),
    "chalf": TimeModel(mfma=750e12, valu=40e12, hbm=3.3e12, elem_bytes=4.0),
}
_model = TIME_MODELS["c64"]
# complex-half precision budget of the plan being scored: None prices every
# step at complex-half rates; N prices only the N steps with the most
# estimated complex64 time so (the library's choice of FP16 tensors), the
# others at complex64 rates
_half_budget: Optional[int] = None


@contextlib.contextmanager
def time_model(precision: str, half_budget: Optional[int] = None):
    """Score plans with the rates of `precision` ("c64" or "chalf") inside
    the block (the default is complex64).  For "chalf", `half_budget` is the
    number of intermediates the plan will store in FP16 (the library's
    default is min(16, k / 282) for k amplitudes); None assumes every step
    runs at complex-half rates."""
    global _model, _half_budget
    prev = (_model, _half_budget)
    _model = TIME_MODELS[precision]
    _half_budget = half_budget if precision == "chalf" else None
    try:
        yield _model
    finally:
        _model, _half_budget = prev


def step_time(w: float, wa: float, wb: float, ra: int, rb: int, rc: int, k: int) -> float:
    """Estimated seconds of one slice of a pairwise step (see the module
    docstring) under the current time model; ra >= rb are the operand ranks,
    k the contracted bits."""
    md = _model
    m, n = ra - k, rb - k
    flops = 8.0 * w * 2.0 ** (m + n + k)
    by = md.elem_bytes * (w * 2.0 ** rc + wa * 2.0 ** ra + wb * 2.0 ** rb)
    rate = md.valu
    if n + k >= 8 and m >= 6 and n >= 5 and k >= 3:
        rate = md.mfma
    elif m >= 6 and k >= 3 and n < 5:
        # fan-out tiles: output instances sharing an A instance fill the
        # 32 columns of one MFMA tile; the rate scales with the fill
        slots = 32 >> n
        group = w / max(wa, 1.0)
        if group >= 2.0 or (n == 4 and k >= 6):
            rows = math.ceil(group / slots)
            rate = max(md.valu, md.mfma * group / (rows * slots))
    return max(flops / rate, by / md.hbm) + md.launch_s


@dataclass
class Costs:
    S: float            # single-amplitude CMAC per slice
    S_k: float          # multi-amplitude CMAC per slice (all nodes)
    total: float        # CMAC over all slices (slice-invariant nodes once)
    max_rank: int
    n_sliced: int
    time: float = 0.0   # estimated seconds over all slices

    def score(self, objective: str) -> float:
        return self.time if objective == "time" else self.total


def costs(st: Structure, tree: Tree, w: Sequence[int], sliced_mask: int = 0) -> Costs:
    global _model
    n = st.n_tensors
    dep = [bool(st.leaf_masks[t] & sliced_mask) for t in range(n)]
    S = Sk = total = tm = 0.0
    nsl = bin(sliced_mask).count("1")
    budget = _half_budget
    t32: List[float] = []
    t16: List[float] = []
    for j, (a, b) in enumerate(tree.pairs):
        v = n + j
        dep.append(dep[a] or dep[b])
        c = float(2 ** (tree.masks[a] | tree.masks[b]).bit_count())
        mult = 2.0 ** nsl if dep[v] else 1.0
        S += c
        Sk += w[v] * c
        total += w[v] * c * mult
        ra, rb = tree.masks[a].bit_count(), tree.masks[b].bit_count()
        wa, wb = w[a], w[b]
        if rb > ra:
            ra, rb, wa, wb = rb, ra, wb, wa
        args = (w[v], wa, wb, ra, rb, tree.masks[v].bit_count(), (tree.masks[a] & tree.masks[b]).bit_count())
        if budget is None:
            tm += mult * step_time(*args)
        else:
            t16.append(mult * step_time(*args))
            model, _model = _model, TIME_MODELS["c64"]
            t32.append(mult * step_time(*args))
            _model = model
    if budget is not None:
        top = sorted(range(len(t32)), key=lambda i: -t32[i])[:budget]
        tm = sum(t32) + sum(t16[i] - t32[i] for i in top)
    mr = max(m.bit_count() for m in tree.masks)
    return Costs(S, Sk, total, mr, nsl, tm)


# --------------------------------------------------------------------------
# order search


def greedy_pairs(st: Structure) -> List[Tuple[int, int]]:
    """Deterministic greedy: contract the connected pair minimising
    size(out) - size(A) - size(B); ties to smaller CMAC then lowest ids."""
    return _greedy(st, list(range(st.n_tensors)), st.leaf_masks, None, 1.0, 0.0, None)[0]


def _greedy(st: Structure, active: List[int], masks_in: List[int], rng, alpha: float,
            temp: float, score=None, start_id: Optional[int] = None,
            pairs_in: Optional[List[Tuple[int, int]]] = None, join: bool = True):
    """Greedy over the tensors in ``active`` (ids into masks_in).  Returns the
    SSA pairs appended to pairs_in and the final list of live ids."""
    masks = list(masks_in)
    pairs = list(pairs_in or [])
    live = set(active)
    owners: Dict[int, set] = {}
    for t in live:
        for i in _bits(masks[t]):
            owners.setdefault(i, set()).add(t)
    nxt = len(masks) if start_id is None else start_id
    heap: List[tuple] = []

    def cost(a: int, b: int):
        if score is not None:
            c = score(a, b, masks)
        else:
            out = masks[a] ^ masks[b]
            c = (2.0 ** out.bit_count()) - alpha * (2.0 ** masks[a].bit_count() + 2.0 ** masks[b].bit_count())
        if temp > 0.0:
            c = c - temp * math.log(-math.log(rng.random())) * (abs(c) + 1.0)
        cm = 2.0 ** (masks[a] | masks[b]).bit_count()
        return (c, cm)

    def push(t: int):
        seen = set()
        for i in _bits(masks[t]):
            for u in owners.get(i, ()):
                if u != t and u not in seen:
                    seen.add(u)
                    a, b = (t, u) if t < u else (u, t)
                    c, cm = cost(a, b)
                    heapq.heappush(heap, (c, cm, a, b))

    for t in sorted(live):
        push(t)
    while heap:
        _, _, a, b = heapq.heappop(heap)
        if a not in live or b not in live:
            continue
        out = masks[a] ^ masks[b]
        for i in _bits(masks[a] | masks[b]):
            s = owners.get(i)
            if s is not None:
                s.discard(a)
                s.discard(b)
        live.discard(a)
        live.discard(b)
        while len(masks) < nxt:
            masks.append(0)
        masks.append(out)
        live.add(nxt)
        for i in _bits(out):
            owners.setdefault(i, set()).add(nxt)
        pairs.append((a, b))
        push(nxt)
        nxt += 1
    # join disconnected components: smallest first
    while join and len(live) > 1:
        a, b = sorted(live, key=lambda t: (masks[t].bit_count(), t))[:2]
        a, b = min(a, b), max(a, b)
        live.discard(a)
        live.discard(b)
        masks.append(masks[a] | masks[b])
        live.add(len(masks) - 1)
        pairs.append((a, b))
    return pairs, sorted(live), masks


def _expected_width(m: int, k: int) -> float:
    if m == 0:
        return 1.0
    if m > 60:
        return float(k)
    N = 2.0 ** m
    return N * (1.0 - (1.0 - 1.0 / N) ** k)


def stem_branch_pairs(st: Structure, k_eff: int, rng, alpha: float, temp: float,
                      temp2: float = 0.0) -> List[Tuple[int, int]]:
    """Two-phase candidate: dark tensors first (randomised greedy), then every
    remaining tensor with the multi-amplitude step cost w(out)*CMAC."""
    n = st.n_tensors
    dark = [t for t in range(n) if st.leaf_outputs[t] == 0]
    pairs, live, masks = _greedy(st, dark, st.leaf_masks, rng, alpha, temp, join=False)
    # phase two: the dark components plus the bright leaves, scored by the
    # multi-amplitude cost of the step
    live = sorted(set(live) | {t for t in range(n) if st.leaf_outputs[t] != 0})
    outs_all = list(st.leaf_outputs)
    for a, b in pairs:
        outs_all.append(outs_all[a] | outs_all[b])

    def score(a, b, mk):
        o = outs_all[a] | outs_all[b]
        w = _expected_width(o.bit_count(), k_eff)
        return w * 2.0 ** (mk[a] | mk[b]).bit_count()

    pairs2 = list(pairs)
    masks2 = list(masks)
    live2 = set(live)
    owners: Dict[int, set] = {}
    for t in live2:
        for i in _bits(masks2[t]):
            owners.setdefault(i, set()).add(t)
    heap: List[tuple] = []

    def push(t):
        seen = set()
        for i in _bits(masks2[t]):
            for u in owners.get(i, ()):
                if u != t and u not in seen:
                    seen.add(u)
                    a, b = (t, u) if t < u else (u, t)
                    c = score(a, b, masks2)
                    if temp2 > 0:
                        c = c * math.exp(temp2 * rng.standard_normal())
                    heapq.heappush(heap, (c, a, b))

    for t in sorted(live2):
        push(t)
    while heap:
        _, a, b = heapq.heappop(heap)
        if a not in live2 or b not in live2:
            continue
        out = masks2[a] ^ masks2[b]
        for i in _bits(masks2[a] | masks2[b]):
            s = owners.get(i)
            if s is not None:
                s.discard(a)
                s.discard(b)
        live2.discard(a)
        live2.discard(b)
        v = len(masks2)
        masks2.append(out)
        while len(outs_all) <= v:
            outs_all.append(0)
        outs_all[v] = outs_all[a] | outs_all[b]
        live2.add(v)
        for i in _bits(out):
            owners.setdefault(i, set()).add(v)
        pairs2.append((a, b))
        push(v)
    while len(live2) > 1:
        a, b = sorted(live2, key=lambda t: (masks2[t].bit_count(), t))[:2]
        a, b = min(a, b), max(a, b)
        live2.discard(a)
        live2.discard(b)
        masks2.append(masks2[a] | masks2[b])
        outs_all.append(outs_all[a] | outs_all[b])
        live2.add(len(masks2) - 1)
        pairs2.append((a, b))
    return pairs2


def timeline_pairs(st: Structure, k_eff: int, rng=None) -> List[Tuple[int, int]]:
    """Time-ordered trunk: the tensors without closed outputs are absorbed one
    by one in circuit order (tensor ids follow gate order), as a state is
    evolved gate by gate; the bright tensors then join by the multi-amplitude
    step cost, as in the second phase of stem_branch_pairs."""
    n = st.n_tensors
    dark = [t for t in range(n) if st.leaf_outputs[t] == 0]
    pairs: List[Tuple[int, int]] = []
    masks = list(st.leaf_masks)
    outs = list(st.leaf_outputs)
    cur = dark[0] if dark else None
    for t in dark[1:]:
        pairs.append((cur, t))
        masks.append(masks[cur] ^ masks[t])
        outs.append(0)
        cur = n + len(pairs) - 1
    live = ([cur] if cur is not None else []) + [t for t in range(n) if st.leaf_outputs[t] != 0]
    # absorb bright tensors: at each step the connected pair with the lowest
    # multi-amplitude cost (exhaustive over live pairs; few bright tensors)
    live = list(live)
    while len(live) > 1:
        best = None
        for i in range(len(live)):
            for j in range(i + 1, len(live)):
                a, b = live[i], live[j]
                conn = bool(masks[a] & masks[b])
                o = outs[a] | outs[b]
                cost = _expected_width(o.bit_count(), k_eff) * 2.0 ** (masks[a] | masks[b]).bit_count()
                key = (not conn, cost, min(a, b), max(a, b))
                if best is None or key < best[0]:
                    best = (key, a, b)
        _, a, b = best
        pairs.append((a, b))
        masks.append(masks[a] ^ masks[b])
        outs.append(outs[a] | outs[b])
        live.remove(a)
        live.remove(b)
        live.append(n + len(pairs) - 1)
    return pairs


def _overflow(masks: Sequence[int], lw: Sequence[float], cap: Optional[int], mem_cap: Optional[float]) -> float:
    """Sum over tensors of the rank above ``cap`` plus log2(w(v) 2^|v|)
    above ``mem_cap`` (lw: log2 w per node)."""
    over = 0.0
    for m, l in zip(masks, lw):
        r = m.bit_count()
        if cap is not None and r > cap:
            over += r - cap
        if mem_cap is not None and r + l > mem_cap + 1e-9:
            over += r + l - mem_cap
    return over


def slice_to_cap(st: Structure, pairs: Sequence[Tuple[int, int]], w: Sequence[int],
                 cap: Optional[int], min_slices: int = 0,
                 max_sliced: int = 40, objective: str = "time",
                 mem_cap: Optional[float] = None) -> Tuple[List[int], Costs]:
    """Slicer: while some tensor is over the rank cap or its multi-amplitude
    form (w(v) instances of 2^|v| elements) is over 2^mem_cap elements (or
    fewer than min_slices indices are sliced), add the index that most
    reduces the overflow above the caps, then minimises the total cost, ties
    to the lowest id.  Open output indices are never sliced."""
    sliced_mask = 0
    chosen: List[int] = []
    lw = [math.log2(max(x, 1)) for x in w]
    tree = build_tree(st, pairs, 0)
    while True:
        tree = build_tree(st, pairs, sliced_mask)
        over_now = _overflow(tree.masks, lw, cap, mem_cap)
        if over_now == 0.0 and len(chosen) >= min_slices:
            return chosen, costs(st, tree, w, sliced_mask)
        if len(chosen) >= max_sliced:
            raise ValueError("slicer: too many sliced indices for the cap")
        cand = 0
        if over_now > 0.0:
            for m, l in zip(tree.masks, lw):
                r = m.bit_count()
                if (cap is not None and r > cap) or (mem_cap is not None and r + l > mem_cap + 1e-9):
                    cand |= m
        else:
            for m in tree.masks:
                cand |= m
        cand &= ~st.open_indices
        best = None
        for i in _bits(cand):
            trial_mask = sliced_mask | (1 << i)
            t2 = build_tree(st, pairs, trial_mask)
            c = costs(st, t2, w, trial_mask)
            # first shrink the total overflow above the caps, then cost
            over = _overflow(t2.masks, lw, cap, mem_cap)
            key = (over, c.score(objective), i)
            if best is None or key < best[0]:
                best = (key, i)
        if best is None:
            raise ValueError("slicer: no index left to slice")
        chosen.append(best[1])
        sliced_mask |= 1 << best[1]


def refine_slices(st: Structure, pairs: Sequence[Tuple[int, int]], w: Sequence[int], sliced: Sequence[int],
                  cap: Optional[int], objective: str = "time", mem_cap: Optional[float] = None,
                  min_slices: int = 0, exact: bool = False, max_rounds: int = 8) -> Tuple[List[int], Costs]:
    """Slice refiner, with the multi-amplitude loss (Supplementary Sec.
    IV.B).  An index's lifetime runs from the first contraction of a tensor
    holding it to its own contraction; slicing it multiplies by 2^|S| every
    step its lifetime does not cover, so the best sliced sets cover the
    costly steps.  With the multi-amplitude loss the costly steps are the
    wide ones of the branch and twig, after the memory peak of the stem.
    Local search: drop a sliced index (unless ``min_slices`` or ``exact``
    forbids it), or exchange one for an unsliced bond, whenever both caps
    still hold and the loss -- sum_v w(v) CMAC(v) over all slices, or the
    time estimate -- falls; until a round brings no gain."""
    lw = [math.log2(max(x, 1)) for x in w]
    cur = list(sliced)
    mask = sum(1 << i for i in cur)
    best = costs(st, build_tree(st, pairs, mask), w, mask)
    bonds = 0
    for m in st.leaf_masks:
        bonds |= m
    bonds &= ~st.open_indices

    def trial(m2: int):
        t2 = build_tree(st, pairs, m2)
        if _overflow(t2.masks, lw, cap, mem_cap) > 0.0:
            return None
        return costs(st, t2, w, m2)

    for _ in range(max_rounds):
        improved = False
        if not exact:
            for i in list(cur):
                if len(cur) <= min_slices:
                    break
                c2 = trial(mask & ~(1 << i))
                if c2 is not None and c2.score(objective) < best.score(objective) * (1 - 1e-9):
                    cur.remove(i)
                    mask &= ~(1 << i)
                    best = c2
                    improved = True
        for pos in range(len(cur)):
            i = cur[pos]
            base = mask & ~(1 << i)
            pick = None
            for j in _bits(bonds & ~mask):
                c2 = trial(base | (1 << j))
                if c2 is not None and c2.score(objective) < (pick[0].score(objective) if pick else
                                                             best.score(objective) * (1 - 1e-9)):
                    pick = (c2, j)
            if pick is not None:
                best, j = pick
                cur[pos] = j
                mask = base | (1 << j)
                improved = True
        if not improved:
            break
    return cur, best


@dataclass
class Plan:
    pairs: List[Tuple[int, int]]
    sliced: List[int]
    costs: Costs
    widths: List[int]
    method: str


def refine(st: Structure, plan: Plan, words: np.ndarray, cap: Optional[int],
           exact_slices: Optional[int] = None, rounds: int = 4, objective: str = "time",
           min_slices: int = 0, mem_cap: Optional[float] = None) -> Plan:
    """Alternate subtree reconfiguration (sizes 6, 8, 10) with re-slicing
    until the objective stops falling."""
    best = plan
    pairs = list(plan.pairs)
    sliced = list(plan.sliced)
    for _ in range(rounds):
        sl = sum(1 << i for i in sliced)
        for size in (6, 8, 10):
            pairs = reconfigure(st, pairs, words, cap, sl, size=size, passes=4, objective=objective,
                                mem_cap=mem_cap)
        tree = build_tree(st, pairs)
        w = widths(tree, words)
        c = costs(st, build_tree(st, pairs, sl), w, sl)
        cand = Plan(pairs, sliced, c, w, best.method + "+reconf")
        try:
            s2, c2 = slice_to_cap(st, pairs, w, cap, min_slices=exact_slices or min_slices, objective=objective,
                                  mem_cap=mem_cap)
            if (exact_slices is None or len(s2) == exact_slices) and c2.score(objective) < c.score(objective):
                cand = Plan(pairs, s2, c2, w, best.method + "+reconf")
        except ValueError:
            pass
        if cand.costs.score(objective) < best.costs.score(objective) * (1 - 1e-6):
            best = cand
            pairs, sliced = list(cand.pairs), list(cand.sliced)
        else:
            break
    return best


def find_plan(net: TensorNetwork, words: np.ndarray, open_qubits: Sequence[int] = (),
              cap: Optional[int] = None, seed: int = 0, trials: int = 64,
              min_slices: int = 0, exact_slices: Optional[int] = None,
              include_greedy: bool = True, refine_top: int = 3, partition_trials: int = 0,
              rgreedy_trials: int = 0, timeline: bool = False, max_sliced: int = 40,
              objective: str = "time", progress=None, mem_cap: Optional[float] = None) -> Plan:
    """Search candidate orders; slice each to the cap; refine the cheapest
    few by subtree reconfiguration; keep the cheapest under ``objective``
    ("time" or "flops", see the module docstring).  ``mem_cap`` bounds
    log2 of the elements of every multi-amplitude tensor, w(v) 2^|v|."""
    if objective not in ("time", "flops"):
        raise ValueError("objective must be 'time' or 'flops'")
    st = Structure.from_network(net, open_qubits)
    words = np.asarray(words, dtype=np.uint64)
    k_eff = int(np.unique(words).size)
    rng = np.random.default_rng(seed)
    candidates = []
    if include_greedy:
        candidates.append(("greedy", greedy_pairs(st)))
    for t in range(trials):
        alpha = float(rng.uniform(0.0, 1.5))
        temp = float(rng.uniform(0.0, 1.0))
        temp2 = float(rng.uniform(0.0, 0.5)) if t % 2 else 0.0
        candidates.append((f"stem-branch[{t}]", stem_branch_pairs(st, k_eff, rng, alpha, temp, temp2)))
    if timeline:
        candidates.append(("timeline", timeline_pairs(st, k_eff)))
    for t in range(rgreedy_trials):
        alpha = float(rng.uniform(0.0, 1.5))
        temp = float(rng.uniform(0.0, 1.0))
        candidates.append((f"rgreedy[{t}]",
                           _greedy(st, list(range(st.n_tensors)), st.leaf_masks, rng, alpha, temp)[0]))
    for t in range(partition_trials):
        imb = float(rng.uniform(0.05, 0.35))
        candidates.append((f"bisection[{t}]", partition_pairs(st, rng, imb)))
    scored = []
    for ci, (name, pairs) in enumerate(candidates):
        if progress is not None:
            progress(f"candidate {ci + 1}/{len(candidates)}")
        tree = build_tree(st, pairs)
        w = widths(tree, words)
        try:
            sliced, c = slice_to_cap(st, pairs, w, cap, min_slices=(exact_slices or min_slices),
                                     max_sliced=max_sliced, objective=objective, mem_cap=mem_cap)
        except ValueError:
            continue
        # an exact slice count (C3's 2^8) is preferred; a plan that needs more
        # indices to reach the cap keeps its real count
        miss = 0 if exact_slices is None else abs(len(sliced) - exact_slices)
        key = (miss, c.score(objective), c.max_rank)
        scored.append((key, Plan(list(pairs), sliced, c, w, name)))
    if not scored:
        raise ValueError("no plan meets the cap")
    scored.sort(key=lambda x: x[0])
    out = []
    for key, pl in scored[:max(1, refine_top)]:
        if progress is not None:
            progress(f"refining {pl.method}")
        r = pl
        if refine_top > 0:
            # the flop objective's local search first (it escapes the poor
            # initial shapes best), then the time objective from there
            r = refine(st, pl, words, cap, exact_slices, objective="flops", min_slices=min_slices,
                       mem_cap=mem_cap)
            if objective == "time":
                r = refine(st, r, words, cap, exact_slices, objective="time", min_slices=min_slices,
                           mem_cap=mem_cap)
        # the slice refiner on the refined tree (exchanges of sliced indices)
        s2, c2 = refine_slices(st, r.pairs, r.widths, r.sliced, cap, objective=objective, mem_cap=mem_cap,
                               min_slices=exact_slices or min_slices, exact=exact_slices is not None)
        if c2.score(objective) < r.costs.score(objective):
            r = Plan(r.pairs, s2, c2, r.widths, r.method + "+slice-refiner")
        miss = 0 if exact_slices is None else abs(len(r.sliced) - exact_slices)
        out.append(((miss, r.costs.score(objective), r.costs.max_rank), r))
    out.sort(key=lambda x: x[0])
    return out[0][1]


def greedy_plan(net: TensorNetwork, words: np.ndarray, open_qubits: Sequence[int] = (),
                cap: Optional[int] = None, min_slices: int = 0, objective: str = "time",
                mem_cap: Optional[float] = None) -> Plan:
    """The deterministic greedy order alone (no search, no refinement), sliced
    to the cap: the plan the workloads name as "greedy order", kept as the
    reference point of a searched plan."""
    st = Structure.from_network(net, open_qubits)
    words = np.asarray(words, dtype=np.uint64)
    pairs = greedy_pairs(st)
    w = widths(build_tree(st, pairs), words)
    sliced, c = slice_to_cap(st, pairs, w, cap, min_slices=min_slices, objective=objective, mem_cap=mem_cap)
    return Plan(list(pairs), sliced, c, w, "greedy")


def plan_from(net: TensorNetwork, words: np.ndarray, open_qubits: Sequence[int], pairs, sliced,
              method: str = "given") -> Plan:
    """A Plan (costs, widths) for a given tree and sliced set."""
    st = Structure.from_network(net, open_qubits)
    words = np.asarray(words, dtype=np.uint64)
    pairs = [tuple(p) for p in pairs]
    mask = sum(1 << i for i in sliced)
    w = widths(build_tree(st, pairs), words)
    return Plan(pairs, list(sliced), costs(st, build_tree(st, pairs, mask), w, mask), w, method)


def report(plan: Plan, words: np.ndarray) -> dict:
    """Cost figures of a plan (Eq. (1) per slice and over all slices): S, S_k,
    the ideal multi-amplitude speedup k S / S_k (k distinct bitstrings), total
    CMAC, slices, largest rank and the planner's time estimate."""
    k = int(np.unique(np.asarray(words, dtype=np.uint64)).size)
    c = plan.costs
    return {"S": c.S, "S_k": c.S_k, "kS_over_Sk": k * c.S / c.S_k, "cmac_total": c.total,
            "n_slices": 2 ** c.n_sliced, "max_rank": c.max_rank, "est_seconds": c.time, "method": plan.method}


def stem_path(tree: Tree) -> List[int]:
    """The stem of a contraction tree, bottom-up: from the root down to a leaf
    through the child with more leaves below it (ties: the first of the pair).  On a
    path-shaped order (each step absorbs one leaf) this is the order itself."""
    n = tree.n_tensors
    path = []
    v = tree.root
    while v >= n:
        path.append(v)
        a, b = tree.pairs[v - n]
        ca, cb = bin(tree.leafsets[a]).count("1"), bin(tree.leafsets[b]).count("1")
        v = a if ca >= cb else b
    path.append(v)
    return path[::-1]


def memory_figures(tree: Tree, words: np.ndarray) -> dict:
    """Memory of the two traversals of the reuse tree (Supplementary
    Sec. III.C), in tensor elements, along the stem s_0 (a leaf), s_1, ...
    of the tree.  The reuse tree branches at each stem step j whose width
    grows, w(s_j) > w(s_{j-1}): what s_j absorbs carries closed outputs not
    seen before.  Its layer l holds the nodes at that point, one per
    distinct prefix, w_l = w(s_{j-1}) of them (w_1 = 1 at the end of the
    trunk), and each stores the tensor immediately before it, s_{j-1}, of
    rank d_l = |idx(s_{j-1})|, for its children to reuse.  Breadth first,
    all of one layer's tensors are held at once: M^BFT = max_l w_l 2^{d_l}.
    Depth first, one per layer on the current root-to-leaf path:
    M^DFT = sum_l 2^{d_l}; the twig after the last branching stores nothing.
    A sliced index is fixed in every slice, so a tree built with a sliced
    set gives the figures of one slice."""
    w = widths(tree, words)
    s = stem_path(tree)
    layers = [(w[s[j - 1]], bin(tree.masks[s[j - 1]]).count("1")) for j in range(1, len(s)) if w[s[j]] > w[s[j - 1]]]
    return {"layers": layers, "M_BFT": max((wl << d for wl, d in layers), default=0),
            "M_DFT": sum(1 << d for _, d in layers)}


# --------------------------------------------------------------------------
# local refinement: subtree reconfiguration
#
# Take a subtree whose frontier is m <= 8 sub-trees, and replace its internal
# shape by the cheapest binary tree over that frontier, found by dynamic
# programming over subsets (3^m work).  The cost of a node is the
# multi-amplitude step cost w(v) * CMAC(v) (Eq. (1)) or its estimated time,
# multiplied by the number of slices when a sliced index lies below it; a
# node over the rank cap costs infinity.  Repeating this over all nodes is a
# local search that never increases the total cost.


class _Tree:
    def __init__(self, st: Structure, pairs, sliced_mask: int, words: np.ndarray):
        n = st.n_tensors
        self.n = n
        self.st = st
        self.children = {}
        self.masks = [m & ~sliced_mask for m in st.leaf_masks]
        self.outs = list(st.leaf_outputs)
        self.dep = [bool(m & sliced_mask) for m in st.leaf_masks]
        self.nsl = bin(sliced_mask).count("1")
        self.words = words
        self._w = {}
        for j, (a, b) in enumerate(pairs):
            v = n + j
            self.children[v] = (a, b)
            self.masks.append(self.masks[a] ^ self.masks[b])
            self.outs.append(self.outs[a] | self.outs[b])
            self.dep.append(self.dep[a] or self.dep[b])
        self.root = n + len(pairs) - 1 if pairs else 0

    def width(self, o: int) -> int:
        if o == 0:
            return 1
        w = self._w.get(o)
        if w is None:
            w = int(np.unique(self.words & np.uint64(o)).size)
            self._w[o] = w
        return w

    def new_node(self, a, b):
        v = len(self.masks)
        self.children[v] = (a, b)
        self.masks.append(self.masks[a] ^ self.masks[b])
        self.outs.append(self.outs[a] | self.outs[b])
        self.dep.append(self.dep[a] or self.dep[b])
        return v

    def to_pairs(self):
        pairs = []
        ids = {t: t for t in range(self.n)}

        def visit(v):
            if v < self.n:
                return ids[v]
            a, b = self.children[v]
            x, y = visit(a), visit(b)
            pairs.append((x, y))
            return self.n + len(pairs) - 1

        import sys
        sys.setrecursionlimit(max(10000, 4 * self.n))
        visit(self.root)
        return pairs


def _node_cost(T: _Tree, objective: str, my: int, mz: int, oy: int, oz: int, w: float) -> float:
    """Cost of one slice of the step joining operands with index masks my,
    mz and closed-output masks oy, oz (w: width of the result)."""
    if objective != "time":
        return w * 2.0 ** (my | mz).bit_count()
    ra, rb = my.bit_count(), mz.bit_count()
    wa, wb = T.width(oy), T.width(oz)
    if rb > ra:
        ra, rb, wa, wb = rb, ra, wb, wa
    return step_time(w, wa, wb, ra, rb, (my ^ mz).bit_count(), (my & mz).bit_count())


def _optimal_subtree(T: _Tree, frontier, cap, objective: str = "flops", mem_cap: Optional[float] = None):
    m = len(frontier)
    full = (1 << m) - 1
    fm = [T.masks[f] for f in frontier]
    fo = [T.outs[f] for f in frontier]
    fd = [T.dep[f] for f in frontier]
    mask = [0] * (1 << m)
    outs = [0] * (1 << m)
    dep = [False] * (1 << m)
    for s in range(1, 1 << m):
        low = s & -s
        i = low.bit_length() - 1
        rest = s ^ low
        mask[s] = mask[rest] ^ fm[i]
        outs[s] = outs[rest] | fo[i]
        dep[s] = dep[rest] or fd[i]
    mult = 2.0 ** T.nsl
    INF = float("inf")
    best = [INF] * (1 << m)
    split = [0] * (1 << m)
    for i in range(m):
        best[1 << i] = 0.0
    for s in range(1, 1 << m):
        if s & (s - 1) == 0:
            continue
        if cap is not None and bin(mask[s]).count("1") > cap:
            continue
        w = T.width(outs[s])
        if mem_cap is not None and s != full and bin(mask[s]).count("1") + math.log2(w) > mem_cap + 1e-9:
            continue
        f = mult if dep[s] else 1.0
        # enumerate splits with the lowest set bit in y to halve the work
        low = s & -s
        sub = (s - 1) & s
        b = INF
        bs = 0
        while sub:
            if sub & low:
                y, z = sub, s ^ sub
                if best[y] < INF and best[z] < INF:
                    c = best[y] + best[z] + f * _node_cost(T, objective, mask[y], mask[z], outs[y], outs[z], w)
                    if c < b:
                        b, bs = c, y
            sub = (sub - 1) & s
        best[s] = b
        split[s] = bs
    return best[full], split


def _subtree_cost(T: _Tree, v, frontier_set, objective: str = "flops"):
    if v in frontier_set:
        return 0.0
    a, b = T.children[v]
    mult = 2.0 ** T.nsl if T.dep[v] else 1.0
    c = mult * _node_cost(T, objective, T.masks[a], T.masks[b], T.outs[a], T.outs[b], T.width(T.outs[v]))
    return c + _subtree_cost(T, a, frontier_set, objective) + _subtree_cost(T, b, frontier_set, objective)


def reconfigure(st: Structure, pairs, words, cap: Optional[int], sliced_mask: int = 0,
                size: int = 8, passes: int = 2, objective: str = "flops",
                mem_cap: Optional[float] = None) -> List[Tuple[int, int]]:
    """Local search over subtrees of ``size`` frontier nodes (see above)."""
    words = np.asarray(words, dtype=np.uint64)
    T = _Tree(st, pairs, sliced_mask, words)
    for _ in range(passes):
        changed = False
        # visit internal nodes from the root down
        order = []
        stack = [T.root]
        while stack:
            v = stack.pop()
            if v >= T.n:
                order.append(v)
                stack.extend(T.children[v])
        for v in order:
            if v not in T.children:
                continue
            # grow the frontier by expanding the most expensive internal node
            frontier = list(T.children[v])
            while len(frontier) < size:
                cand = [f for f in frontier if f >= T.n]
                if not cand:
                    break
                f = max(cand, key=lambda x: (bin(T.masks[x]).count("1"), x))
                frontier.remove(f)
                frontier.extend(T.children[f])
            if len(frontier) < 3:
                continue
            old = _subtree_cost(T, v, set(frontier), objective)
            new, split = _optimal_subtree(T, frontier, cap, objective, mem_cap)
            if new < old * (1 - 1e-9):
                def build(s):
                    if s & (s - 1) == 0:
                        return frontier[s.bit_length() - 1]
                    y = split[s]
                    return T.new_node(build(y), build(s ^ y))
                a_s = split[(1 << len(frontier)) - 1]
                full = (1 << len(frontier)) - 1
                na, nb = build(a_s), build(full ^ a_s)
                # rewire v in place so that its parent keeps pointing at it
                T.children[v] = (na, nb)
                T.masks[v] = T.masks[na] ^ T.masks[nb]
                changed = True
        if not changed:
            break
    return T.to_pairs()


# --------------------------------------------------------------------------
# recursive bisection
#
# Partition-based order search: split the tensors into two balanced halves
# that share as few indices as possible, contract each half recursively and
# join them; small groups are ordered exactly by the subset DP above.  A
# split starts from a region grown breadth-first from a random tensor and is
# improved by Fiduccia-Mattheyses passes (move the unlocked tensor whose move
# cuts the most shared indices, keep the best prefix of the pass).  The
# paper searches orders with hypergraph partitioning (KaHyPar) under the
# multi-amplitude loss; this is a small self-contained stand-in, with the
# loss applied afterwards by subtree reconfiguration.


def _fm_bisect(nodes: List[int], nbrs: Dict[int, Dict[int, int]], rng, imbalance: float) -> Tuple[set, set]:
    n = len(nodes)
    node_set = set(nodes)
    target = n // 2
    lo = max(1, int(n * (0.5 - imbalance)))
    hi = min(n - 1, int(math.ceil(n * (0.5 + imbalance))))
    # BFS-grown initial region
    start = nodes[int(rng.integers(0, n))]
    left = {start}
    frontier = [start]
    while len(left) < target:
        nxt = []
        for u in frontier:
            for v in nbrs[u]:
                if v in node_set and v not in left:
                    left.add(v)
                    nxt.append(v)
                    if len(left) >= target:
                        break
            if len(left) >= target:
                break
        if not nxt:
            rest = [v for v in nodes if v not in left]
            if not rest:
                break
            nxt = [rest[int(rng.integers(0, len(rest)))]]
            left.add(nxt[0])
        frontier = nxt
    side = {v: (0 if v in left else 1) for v in nodes}

    def cut_of():
        c = 0
        for u in nodes:
            for v, wgt in nbrs[u].items():
                if v in node_set and u < v and side[u] != side[v]:
                    c += wgt
        return c

    best_cut = cut_of()
    for _ in range(8):
        gain = {}
        for u in nodes:
            g = 0
            for v, wgt in nbrs[u].items():
                if v in node_set:
                    g += wgt if side[v] != side[u] else -wgt
            gain[u] = g
        locked = set()
        size0 = sum(1 for v in nodes if side[v] == 0)
        cur = best_cut
        moves = []
        best_prefix, best_val = 0, best_cut
        for _step in range(n):
            cand = None
            for u in nodes:
                if u in locked:
                    continue
                s0 = size0 - 1 if side[u] == 0 else size0 + 1
                if s0 < lo or s0 > hi:
                    continue
                key = (gain[u], rng.random())
                if cand is None or key > cand[0]:
                    cand = (key, u)
            if cand is None:
                break
            u = cand[1]
            locked.add(u)
            cur -= gain[u]
            old = side[u]
            side[u] = 1 - old
            size0 += -1 if old == 0 else 1
            moves.append(u)
            for v, wgt in nbrs[u].items():
                if v in node_set:
                    gain[v] += (2 * wgt) if side[v] == old else (-2 * wgt)
            gain[u] = -gain[u]
            if cur < best_val:
                best_val, best_prefix = cur, len(moves)
        for u in moves[best_prefix:]:
            side[u] = 1 - side[u]
        if best_val >= best_cut:
            best_cut = best_val
            break
        best_cut = best_val
    L = {v for v in nodes if side[v] == 0}
    R = node_set - L
    return L, R


def partition_pairs(st: Structure, rng, imbalance: float = 0.2, leaf_size: int = 8) -> List[Tuple[int, int]]:
    """Contraction tree by recursive balanced bisection (see above)."""
    n = st.n_tensors
    owners: Dict[int, List[int]] = {}
    for t in range(n):
        for i in _bits(st.leaf_masks[t]):
            owners.setdefault(i, []).append(t)
    nbrs: Dict[int, Dict[int, int]] = {t: {} for t in range(n)}
    for i, ts in owners.items():
        for a in ts:
            for b in ts:
                if a != b:
                    nbrs[a][b] = nbrs[a].get(b, 0) + 1
    masks = list(st.leaf_masks)
    pairs: List[Tuple[int, int]] = []

    def join(a: int, b: int) -> int:
        pairs.append((a, b))
        masks.append(masks[a] ^ masks[b])
        return n + len(pairs) - 1

    def small(group: List[int]) -> int:
        # exact order of a small group by subset DP on size(out) cost
        m = len(group)
        if m == 1:
            return group[0]
        fm = [masks[g] for g in group]
        sm = [0] * (1 << m)
        for s in range(1, 1 << m):
            low = s & -s
            sm[s] = sm[s ^ low] ^ fm[low.bit_length() - 1]
        best = [0.0] * (1 << m)
        split = [0] * (1 << m)
        for s in range(1, 1 << m):
            if s & (s - 1) == 0:
                continue
            low = s & -s
            sub = (s - 1) & s
            b, bs = float("inf"), 0
            while sub:
                if sub & low:
                    y, z = sub, s ^ sub
                    c = best[y] + best[z] + 2.0 ** bin(sm[y] | sm[z]).count("1")
                    if c < b:
                        b, bs = c, y
                sub = (sub - 1) & s
            best[s], split[s] = b, bs

        def build(s):
            if s & (s - 1) == 0:
                return group[s.bit_length() - 1]
            y = split[s]
            return join(build(y), build(s ^ y))
        return build((1 << m) - 1)

    def rec(group: List[int]) -> int:
        if len(group) <= leaf_size:
            return small(group)
        L, R = _fm_bisect(group, nbrs, rng, imbalance)
        if not L or not R:
            half = len(group) // 2
            L, R = set(group[:half]), set(group[half:])
        a = rec(sorted(L))
        b = rec(sorted(R))
        return join(a, b)

    import sys
    sys.setrecursionlimit(max(10000, 8 * n))
    rec(list(range(n)))
    return pairs
