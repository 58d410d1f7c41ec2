"""Plain tensor-network contraction of circuit amplitudes in complex128.

The circuit becomes a network of one tensor per object (Supplementary
Information, Sec. II): |0> is a rank-1 tensor, a single-qubit gate a rank-2
tensor U[out, in], fSim a rank-4 tensor G[out_a, out_b, in_a, in_b].  There
is no gate fusion here: this network is deliberately not the one the library
contracts.  The last wire of each qubit is its output index.  Fixing the
output index of qubit q to b_q (a slice of that index) for every qubit leaves
a network with no open index whose value is <b|psi>; leaving some outputs
open gives the block of correlated amplitudes over those qubits.

Order: a greedy pass over pairs of tensors that share an index, taking the
pair whose result grows the stored size least (size(out) - size(a) - size(b)),
ties to the lower tensor ids; disconnected parts are joined last by outer
products.  Each pairwise step is numpy.tensordot over the shared indices.

Slicing (Sec. IV.B): fixing a set of indices to every assignment of values
and summing the contractions gives the unsliced value.  With a rank cap, the
oracle slices the index that occurs in the most over-cap intermediates of its
own order, until none is over the cap.
"""

from __future__ import annotations

import heapq
import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .circuit import gate_list, words_to_bits


class Network:
    """Unfused circuit network.  ``indices[t]`` names the axes of ``tensors[t]``."""

    def __init__(self, circ: dict):
        n, glist = gate_list(circ)
        self.n = n
        self.tensors: List[np.ndarray] = []
        self.indices: List[Tuple[int, ...]] = []
        fresh = itertools.count()
        wire = []
        for q in range(n):
            w = next(fresh)
            wire.append(w)
            self.tensors.append(np.array([1.0, 0.0], dtype=np.complex128))
            self.indices.append((w,))
        for qubits, mat in glist:
            if len(qubits) == 1:
                (q,) = qubits
                new = next(fresh)
                self.tensors.append(mat.copy())
                self.indices.append((new, wire[q]))
                wire[q] = new
            else:
                qa, qb = qubits
                na, nb = next(fresh), next(fresh)
                self.tensors.append(mat.reshape(2, 2, 2, 2).copy())
                self.indices.append((na, nb, wire[qa], wire[qb]))
                wire[qa], wire[qb] = na, nb
        self.output_index = list(wire)
        self.n_index = next(fresh)


def _fix(tensor: np.ndarray, idx: Tuple[int, ...], fixed: Dict[int, int]):
    """Take the slice of every fixed index present in this tensor."""
    keep = []
    for pos, i in enumerate(idx):
        if i in fixed:
            continue
        keep.append(i)
    sel = tuple(fixed[i] if i in fixed else slice(None) for i in idx)
    return tensor[sel], tuple(keep)


def greedy_order(index_sets: Sequence[Tuple[int, ...]]) -> List[Tuple[int, int]]:
    """Pairwise order as SSA pairs (ids >= len(index_sets) are results)."""
    live: Dict[int, frozenset] = {t: frozenset(ix) for t, ix in enumerate(index_sets)}
    count: Dict[int, int] = {}
    for ix in live.values():
        for i in ix:
            count[i] = count.get(i, 0) + 1
    owners: Dict[int, set] = {}
    for t, ix in live.items():
        for i in ix:
            owners.setdefault(i, set()).add(t)

    def result(a: int, b: int) -> frozenset:
        shared = live[a] & live[b]
        # an index shared by both operands and by no other tensor is summed
        summed = {i for i in shared if count[i] == 2}
        return (live[a] | live[b]) - summed

    def cost(a: int, b: int) -> int:
        return (1 << len(result(a, b))) - (1 << len(live[a])) - (1 << len(live[b]))

    heap: List[Tuple[int, int, int]] = []

    def push_neighbours(t: int):
        seen = set()
        for i in live[t]:
            for u in owners[i]:
                if u != t and u not in seen:
                    seen.add(u)
                    a, b = min(t, u), max(t, u)
                    heapq.heappush(heap, (cost(a, b), a, b))

    for t in list(live):
        push_neighbours(t)
    order: List[Tuple[int, int]] = []
    nxt = len(index_sets)
    while heap:
        c, a, b = heapq.heappop(heap)
        if a not in live or b not in live or not (live[a] & live[b]):
            continue
        if c != cost(a, b):
            continue
        out = result(a, b)
        for i in live[a] | live[b]:
            owners[i].discard(a)
            owners[i].discard(b)
        for i in live[a] & live[b]:
            count[i] -= 1 if i in out else 2
        del live[a]
        del live[b]
        live[nxt] = out
        for i in out:
            owners[i].add(nxt)
        order.append((a, b))
        push_neighbours(nxt)
        nxt += 1
    # join disconnected parts, smallest first
    while len(live) > 1:
        a, b = sorted(live, key=lambda t: (len(live[t]), t))[:2]
        a, b = min(a, b), max(a, b)
        live[nxt] = live.pop(a) | live.pop(b)
        order.append((a, b))
        nxt += 1
    return order


def _intermediates(index_sets, order):
    sets = [frozenset(x) for x in index_sets]
    count: Dict[int, int] = {}
    for s in sets:
        for i in s:
            count[i] = count.get(i, 0) + 1
    out = []
    for a, b in order:
        shared = sets[a] & sets[b]
        summed = {i for i in shared if count[i] == 2}
        for i in shared:
            count[i] -= 1 if i not in summed else 2
        r = (sets[a] | sets[b]) - summed
        sets.append(r)
        out.append(r)
    return out


def choose_slices(index_sets, order, cap: int, protected=()) -> List[int]:
    """Indices to slice so that every intermediate of ``order`` has rank <= cap."""
    inter = [set(s) for s in _intermediates(index_sets, order)]
    leaves = [set(s) for s in index_sets]
    chosen: List[int] = []
    protected = set(protected)
    while True:
        over = [s for s in inter + leaves if len(s) > cap]
        if not over:
            return chosen
        tally: Dict[int, int] = {}
        for s in over:
            for i in s:
                if i not in protected:
                    tally[i] = tally.get(i, 0) + 1
        if not tally:
            raise ValueError("oracle: cannot meet the rank cap")
        best = min(tally, key=lambda i: (-tally[i], i))
        chosen.append(best)
        for s in inter + leaves:
            s.discard(best)


def contract(tensors: Sequence[np.ndarray], indices: Sequence[Tuple[int, ...]],
             order: Sequence[Tuple[int, int]], final_order: Sequence[int]) -> np.ndarray:
    """Run a pairwise order with numpy.tensordot; return the result with its
    axes in ``final_order``."""
    ts = list(tensors)
    ix = [tuple(x) for x in indices]
    count: Dict[int, int] = {}
    for s in ix:
        for i in s:
            count[i] = count.get(i, 0) + 1
    for a, b in order:
        A, B = ts[a], ts[b]
        ia, ib = ix[a], ix[b]
        shared = [i for i in ia if i in ib and count[i] == 2]
        for i in ia:
            if i in ib:
                count[i] -= 2 if i in shared else 1
        pa = [ia.index(i) for i in shared]
        pb = [ib.index(i) for i in shared]
        if any(i in ib and i not in shared for i in ia):
            raise ValueError("oracle: hyper-index not supported")
        C = np.tensordot(A, B, axes=(pa, pb))
        ic = tuple(i for i in ia if i not in shared) + tuple(i for i in ib if i not in shared)
        ts.append(C)
        ix.append(ic)
        ts[a] = ts[b] = None  # release memory
    res, ires = ts[-1], ix[-1]
    if len(order) == 0:
        res, ires = ts[0], ix[0]
    perm = [ires.index(i) for i in final_order]
    return np.transpose(res, perm) if perm else res


class Plan:
    """The oracle's own order and sliced set for one circuit and one open set."""

    def __init__(self, circ: dict, open_qubits: Sequence[int] = (), cap: Optional[int] = None,
                 sliced: Optional[Sequence[int]] = None):
        self.net = Network(circ)
        self.open_qubits = tuple(sorted(open_qubits))
        closed_out = {self.net.output_index[q] for q in range(self.net.n) if q not in self.open_qubits}
        self.struct = [tuple(i for i in ix if i not in closed_out) for ix in self.net.indices]
        self.order = greedy_order(self.struct)
        opens = [self.net.output_index[q] for q in self.open_qubits]
        if sliced is not None:
            self.sliced = list(sliced)
        elif cap is not None:
            self.sliced = choose_slices(self.struct, self.order, cap, protected=opens)
        else:
            self.sliced = []
        sl = set(self.sliced)
        inter = _intermediates([tuple(i for i in s if i not in sl) for s in self.struct], self.order)
        self.max_rank = max([len(s) for s in inter] + [len(s) for s in self.struct] + [0])

    def _tensors_for(self, bits: np.ndarray, slice_values: Dict[int, int]):
        fixed = dict(slice_values)
        for q in range(self.net.n):
            if q not in self.open_qubits:
                fixed[self.net.output_index[q]] = int(bits[q])
        ts, ix = [], []
        for t, idx in zip(self.net.tensors, self.net.indices):
            a, i = _fix(t, idx, fixed)
            ts.append(a)
            ix.append(i)
        return ts, ix

    def slice_partial(self, bits: np.ndarray, assignment: Sequence[int]) -> np.ndarray:
        """Contraction of one slice: sliced index j takes assignment[j]."""
        values = {i: int(v) for i, v in zip(self.sliced, assignment)}
        ts, ix = self._tensors_for(bits, values)
        # the open qubits in descending order, so that a C-order flatten puts
        # the lowest open qubit in bit 0 of the within-group index
        final = [self.net.output_index[q] for q in reversed(self.open_qubits)]
        out = contract(ts, ix, self.order, final)
        return np.asarray(out).reshape(-1)

    def amplitude_block(self, bits: np.ndarray) -> np.ndarray:
        total = None
        for assignment in itertools.product((0, 1), repeat=len(self.sliced)):
            part = self.slice_partial(bits, assignment)
            total = part if total is None else total + part
        return total


def amplitudes(circ: dict, words, open_qubits: Sequence[int] = (), cap: Optional[int] = None,
               plan: Optional[Plan] = None) -> np.ndarray:
    """Amplitudes of the batch.  Without open qubits: shape (k,).  With m open
    qubits: shape (k, 2^m), entry [i, j] for the bitstring whose closed bits
    come from words[i] and whose t-th open qubit (ascending) is bit t of j."""
    if plan is None:
        plan = Plan(circ, open_qubits, cap)
    bits = words_to_bits(words, plan.net.n)
    rows = [plan.amplitude_block(bits[i]) for i in range(len(bits))]
    arr = np.array(rows, dtype=np.complex128)
    return arr[:, 0] if not plan.open_qubits else arr
