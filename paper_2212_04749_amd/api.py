"""Convenience layer over the C ABI: torch supplies device memory and streams.

    from paper_2212_04749_amd import api
    run = api.Contraction.from_circuit(circ, words, cap=28, precision="c64")
    amps = run.amplitudes()          # complex128 numpy array (k,) or (k, 2^n_open)
    f = run.xeb()

All contraction work happens in libmatnc's HIP kernels; this module only
builds host arrays, owns the torch workspace and calls the binding.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import binding as B
from .circuit_tn import TensorNetwork, build_network
from . import planner

PRECISIONS = {"c64": B.MATNC_C64, "chalf": B.MATNC_CHALF}


def network_arrays(net: TensorNetwork):
    ranks = [len(ix) for ix in net.indices]
    ids = [i for ix in net.indices for i in ix]
    parts = []
    for t in net.tensors:
        c = np.ascontiguousarray(t, dtype=np.complex128).reshape(-1)
        parts.append(np.stack([c.real, c.imag], axis=1).reshape(-1))
    data = np.concatenate(parts) if parts else np.zeros(0)
    return ranks, ids, data


def tensor_array(t: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(t, dtype=np.complex128).reshape(-1)
    return np.stack([c.real, c.imag], axis=1).reshape(-1)


@dataclass
class PlanSpec:
    pairs: list
    sliced: list
    open_qubits: tuple
    cap: int
    method: str = "given"


class Contraction:
    """One network + plan bound to a torch workspace and stream."""

    def __init__(self, net: TensorNetwork, spec: PlanSpec, words, precision: str = "c64",
                 slice_batch: int = 1, stream=None, device: str = "cuda", memory_budget: Optional[int] = None,
                 half_nodes: int = -1, bind: bool = True):
        """memory_budget: largest workspace in bytes (None: 90% of the device
        memory free now); above it the bitstrings are processed in chunks.
        half_nodes: complex-half plans, how many intermediates are stored in
        FP16 (-1: the library's default; see matnc_plan_create_ex).
        bind=False: create the plan only; a Queue(shared=True) binds it."""
        import torch

        self.torch = torch
        self.net = net
        self.spec = spec
        self.words = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
        self.precision = precision
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        if memory_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            memory_budget = int(0.9 * free)
        ranks, ids, data = network_arrays(net)
        self._net = B.matnc_network_create(ranks, ids, data, net.n_qubits, net.output_index)
        self._plan = None
        try:
            self._plan = B.matnc_plan_create_ex(self._net, spec.pairs, spec.sliced, list(spec.open_qubits),
                                                self.words, PRECISIONS[precision], spec.cap, slice_batch,
                                                memory_budget, half_nodes)
            self.info = B.matnc_plan_info(self._plan)
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
            self.workspace = None
            if bind:
                # allocate on the plan's stream so that the caching allocator
                # orders reuse of this memory after the plan's kernels
                with torch.cuda.stream(self.stream):
                    self.workspace = torch.empty(max(256, int(self.info.workspace_bytes)), dtype=torch.uint8,
                                                 device=self.device)
                B.matnc_plan_bind(self._plan, self.workspace.data_ptr(), self.workspace.numel(),
                                  self.stream.cuda_stream)
        except Exception:
            self.close()
            raise
        self.n_open = len(spec.open_qubits)
        self.slice_batch = slice_batch
        self.k = len(self.words)
        self.n_slices = int(self.info.n_slices)

    @classmethod
    def from_circuit(cls, circ: dict, words, open_qubits: Sequence[int] = (), cap: Optional[int] = None,
                     precision: str = "c64", slice_batch: int = 1, seed: int = 0, trials: int = 32,
                     exact_slices: Optional[int] = None, stream=None, device: str = "cuda",
                     memory_budget: Optional[int] = None, half_nodes: int = -1):
        net = build_network(circ)
        plan = planner.find_plan(net, words, open_qubits, cap, seed=seed, trials=trials,
                                 exact_slices=exact_slices)
        spec = PlanSpec(plan.pairs, plan.sliced, tuple(sorted(open_qubits)),
                        cap if cap is not None else 32, plan.method)
        return cls(net, spec, words, precision, slice_batch, stream, device, memory_budget, half_nodes)

    # ------------------------------------------------------------------
    def new_amplitudes(self):
        """Zeroed float64 [k, 2^open, 2] buffer, allocated and cleared on the plan's stream."""
        with self.torch.cuda.stream(self.stream):
            return self.torch.zeros((self.k, 1 << self.n_open, 2), dtype=self.torch.float64, device=self.device)

    def _check_amps(self, amps):
        if (amps.dtype != self.torch.float64 or not amps.is_contiguous() or amps.device != self.device
                or amps.numel() != self.k * (2 << self.n_open)):
            raise ValueError("amps must be a contiguous float64 device tensor of k * 2^n_open * 2 values")

    def execute(self, amps=None, begin: int = 0, end: Optional[int] = None):
        """Add slices [begin, end) into amps (a torch float64 [k, 2^open, 2]
        device tensor, created zeroed if None) and return it.  Work is queued
        on the plan's stream after everything already queued on the current
        stream."""
        if amps is None:
            amps = self.new_amplitudes()
        else:
            self._check_amps(amps)
            self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
            amps.record_stream(self.stream)
        if end is None:
            end = self.n_slices
        B.matnc_execute(self._plan, begin, end, amps.data_ptr())
        return amps

    def execute_timed(self, amps, step: int, begin: int = 0, end: Optional[int] = None):
        """execute() launched one by one with HIP events around every launch
        of contraction step `step`; waits for the pass and returns (summed
        milliseconds of those launches, their number)."""
        self._check_amps(amps)
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        amps.record_stream(self.stream)
        if end is None:
            end = self.n_slices
        return B.matnc_execute_timed(self._plan, begin, end, amps.data_ptr(), step)

    def xeb_dev(self, amps):
        self._check_amps(amps)
        with self.torch.cuda.stream(self.stream):
            out = self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        B.matnc_xeb(self._plan, amps.data_ptr(), out.data_ptr())
        return out

    def synchronize(self):
        self.stream.synchronize()

    def amplitudes(self, begin: int = 0, end: Optional[int] = None) -> np.ndarray:
        amps = self.execute(None, begin, end)
        self.synchronize()
        a = amps.cpu().numpy()
        c = a[..., 0] + 1j * a[..., 1]
        return c[:, 0] if self.n_open == 0 else c

    def xeb(self, amps=None) -> float:
        if amps is None:
            amps = self.execute()
        out = self.xeb_dev(amps)
        self.synchronize()
        return float(out.cpu().item())

    def step_dep(self):
        """Per contraction step: True if a sliced index lies below it (runs once per slice)."""
        sl = set(self.spec.sliced)
        dep = [any(i in sl for i in ix) for ix in self.net.indices]
        for a, b in self.spec.pairs:
            dep.append(dep[a] or dep[b])
        return dep[len(self.net.indices):]

    def autotune(self, reps: int = 3, cache_path: Optional[str] = None) -> None:
        """Pick MFMA tile shapes by timing them (see matnc_plan_autotune);
        cache_path defaults to $MATNC_AUTOTUNE_CACHE."""
        import os
        B.matnc_plan_autotune(self._plan, reps, cache_path or os.environ.get("MATNC_AUTOTUNE_CACHE"))

    def reset_cache(self) -> None:
        B.matnc_plan_reset_cache(self._plan)

    def profile(self, slice_begin: int = 0, nb: Optional[int] = None):
        """Per contraction step: (time_ms, kernel id, cmac, bytes) of one batch."""
        nb = nb or min(self.slice_batch, self.n_slices - slice_begin)
        return B.matnc_plan_profile(self._plan, slice_begin, nb, len(self.net.tensors) - 1)

    def set_tensor(self, t: int, data: np.ndarray) -> None:
        """Replace the numbers of tensor t (same index list, so the same
        shape); the next execute uses them."""
        if not 0 <= t < len(self.net.tensors):
            raise ValueError(f"tensor id {t} out of range")
        if np.shape(data) != np.shape(self.net.tensors[t]):
            raise ValueError(f"tensor {t} has shape {np.shape(self.net.tensors[t])}, got {np.shape(data)}")
        B.matnc_plan_set_tensor(self._plan, t, tensor_array(data))

    def close(self):
        if getattr(self, "_plan", None):
            if getattr(self, "stream", None) is not None:
                self.stream.synchronize()
            B.matnc_plan_destroy(self._plan)
            self._plan = None
        if getattr(self, "_net", None):
            B.matnc_network_destroy(self._net)
            self._net = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def contract_pair(A, Bt, C, pos, kernel: int = -1, stream=None):
    """One bit-permuted pairwise contraction on torch complex64 tensors
    (flattened, batch-major).  pos = dict with posA_m, posA_k, posB_k,
    posB_n, posC_m, posC_n; batch = A.numel() // 2^rank(A)."""
    import torch

    nm, nn, nk = len(pos["posA_m"]), len(pos["posB_n"]), len(pos["posA_k"])
    # sizes in complex64 elements (8 bytes), whatever dtype views the storage
    na = A.numel() * A.element_size() // 8
    nb = Bt.numel() * Bt.element_size() // 8
    nc = C.numel() * C.element_size() // 8
    batch = na >> (nm + nk)
    if (batch << (nm + nk)) != na or (batch << (nn + nk)) != nb or (batch << (nm + nn)) != nc:
        raise ValueError(f"operand sizes do not match one batch of ranks "
                         f"({nm + nk}, {nn + nk}, {nm + nn}): {na}, {nb}, {nc} complex elements")
    for t in (A, Bt, C):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("operands must be contiguous device tensors")
    stream = stream if stream is not None else torch.cuda.current_stream()
    scratch = torch.empty(B.matnc_contract_scratch_bytes(), dtype=torch.uint8, device=A.device)
    B.matnc_contract(A.data_ptr(), Bt.data_ptr(), C.data_ptr(), batch, pos["posA_m"], pos["posA_k"],
                     pos["posB_k"], pos["posB_n"], pos["posC_m"], pos["posC_n"], kernel,
                     scratch.data_ptr(), scratch.numel(), stream.cuda_stream)
    return scratch  # keep alive until the stream has run the kernel


class Queue:
    """Several contractions executed as one captured graph (uneven batches);
    they must share one stream.  shared=True binds them all to one workspace
    (their static regions side by side and one arena as large as the
    largest plan's, see matnc_queue_bind), so the runs may be created with
    bind=False."""

    def __init__(self, runs, shared: bool = False):
        import torch
        self.runs = list(runs)
        self._q = B.matnc_queue_create([r._plan for r in self.runs])
        self.stream = self.runs[0].stream
        self.workspace = None
        if shared:
            need = B.matnc_queue_workspace_bytes(self._q)
            dev = self.runs[0].device
            with torch.cuda.stream(self.stream):
                self.workspace = torch.empty(max(256, need), dtype=torch.uint8, device=dev)
            B.matnc_queue_bind(self._q, self.workspace.data_ptr(), self.workspace.numel(), self.stream.cuda_stream)
            for r in self.runs:
                r.stream = self.stream
                r.workspace = self.workspace  # keeps the shared memory alive with every run

    def execute(self, amps=None, xeb=None):
        """One pass of every plan; returns (list of amplitude tensors, XEB
        tensor).  Without buffers, fresh zeroed ones are allocated; given
        buffers (from an earlier call) are zeroed on the queue's stream and
        reused, so that the captured graph is replayed, not re-captured."""
        import torch
        with torch.cuda.stream(self.stream):
            if amps is None:
                amps = [r.new_amplitudes() for r in self.runs]
                xeb = torch.zeros(len(self.runs), dtype=torch.float64, device=self.runs[0].device)
            else:
                for a in amps:
                    a.zero_()
        B.matnc_queue_execute(self._q, [a.data_ptr() for a in amps], xeb.data_ptr())
        return amps, xeb

    def close(self):
        if getattr(self, "_q", None):
            B.matnc_queue_destroy(self._q)
            self._q = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
