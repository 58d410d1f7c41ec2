"""ctypes binding of libmatnc (same names as the C ABI in include/matnc.h).

Argument marshalling only: every contraction step runs in the library's HIP
kernels.  Loading fails loudly when the built library is missing; there is
no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmatnc.so")

MATNC_OK = 0
MATNC_E_INVALID = 1
MATNC_E_RANK = 2
MATNC_E_NOMEM = 3
MATNC_E_HIP = 4
MATNC_E_STATE = 5
MATNC_C64 = 0
MATNC_CHALF = 1

ERROR_NAMES = {1: "E_INVALID", 2: "E_RANK", 3: "E_NOMEM", 4: "E_HIP", 5: "E_STATE"}


class MatncError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"matnc {ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("cmac_single", c_double),
        ("cmac_multi", c_double),
        ("cmac_invariant", c_double),
        ("cmac_total", c_double),
        ("bytes_per_slice", c_double),
        ("bytes_invariant", c_double),
        ("n_slices", c_int64),
        ("n_amplitudes", c_int64),
        ("n_unique", c_int64),
        ("max_rank", c_int),
        ("n_nodes", c_int),
        ("n_mfma_nodes", c_int),
        ("n_launches_per_batch", c_int),
        ("workspace_bytes", c_size_t),
        ("cache_bytes", c_size_t),
        ("n_chunks", c_int),
        ("n_fan_nodes", c_int),
        ("n_half_nodes", c_int),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

EXPORTS = [
    "matnc_version", "matnc_last_error", "matnc_network_create", "matnc_network_destroy",
    "matnc_plan_create", "matnc_plan_info", "matnc_plan_set_tensor", "matnc_plan_bind",
    "matnc_execute", "matnc_xeb", "matnc_plan_destroy", "matnc_queue_create",
    "matnc_queue_execute", "matnc_queue_destroy", "matnc_contract_scratch_bytes",
    "matnc_mfma_config_count", "matnc_contract", "matnc_plan_reset_cache", "matnc_plan_profile",
    "matnc_plan_autotune", "matnc_contract_noalloc", "matnc_plan_create_ex", "matnc_queue_workspace_bytes",
    "matnc_queue_bind", "matnc_execute_timed",
]


def lib():
    """Load the in-tree libmatnc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmatnc.so not built ({LIB_PATH}); run python -m paper_2212_04749_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    L.matnc_version.restype = c_char_p
    L.matnc_version.argtypes = []
    L.matnc_last_error.restype = c_char_p
    L.matnc_last_error.argtypes = []
    L.matnc_network_create.argtypes = [c_int, POINTER(c_int), POINTER(c_int), POINTER(c_double), c_int,
                                       POINTER(c_int), POINTER(c_void_p)]
    L.matnc_network_destroy.argtypes = [c_void_p]
    L.matnc_plan_create.argtypes = [c_void_p, POINTER(c_int), c_int, POINTER(c_int), c_int, POINTER(c_int),
                                    c_int64, POINTER(c_uint64), c_int, c_int, c_int, c_size_t, POINTER(c_void_p)]
    L.matnc_plan_info.argtypes = [c_void_p, POINTER(PlanInfo)]
    L.matnc_plan_set_tensor.argtypes = [c_void_p, c_int, POINTER(c_double)]
    L.matnc_plan_bind.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
    L.matnc_execute.argtypes = [c_void_p, c_int64, c_int64, c_void_p]
    L.matnc_execute_timed.argtypes = [c_void_p, c_int64, c_int64, c_void_p, c_int, POINTER(c_double),
                                      POINTER(ctypes.c_int64)]
    L.matnc_xeb.argtypes = [c_void_p, c_void_p, c_void_p]
    L.matnc_plan_destroy.argtypes = [c_void_p]
    L.matnc_queue_create.argtypes = [c_int, POINTER(c_void_p), POINTER(c_void_p)]
    L.matnc_queue_execute.argtypes = [c_void_p, POINTER(c_void_p), c_void_p]
    L.matnc_queue_destroy.argtypes = [c_void_p]
    L.matnc_plan_reset_cache.argtypes = [c_void_p]
    L.matnc_plan_autotune.argtypes = [c_void_p, c_int, c_char_p]
    L.matnc_plan_profile.argtypes = [c_void_p, c_int64, c_int, POINTER(ctypes.c_float), POINTER(c_int),
                                     POINTER(c_double), POINTER(c_double)]
    L.matnc_contract_scratch_bytes.restype = c_size_t
    L.matnc_contract_scratch_bytes.argtypes = []
    L.matnc_mfma_config_count.restype = c_int
    L.matnc_mfma_config_count.argtypes = []
    L.matnc_contract.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_int, c_int, c_int,
                                 POINTER(c_int), POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                 POINTER(c_int), POINTER(c_int), c_int, c_void_p, c_size_t, c_void_p]
    L.matnc_plan_create_ex.argtypes = [c_void_p, POINTER(c_int), c_int, POINTER(c_int), c_int, POINTER(c_int),
                                       c_int64, POINTER(c_uint64), c_int, c_int, c_void_p, POINTER(c_void_p)]
    L.matnc_queue_workspace_bytes.argtypes = [c_void_p, POINTER(c_size_t)]
    L.matnc_queue_bind.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
    L.matnc_contract_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_int, c_int, c_int,
                                         POINTER(c_int), POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                         POINTER(c_int), POINTER(c_int), c_int, c_void_p]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("matnc_version", "matnc_last_error", "matnc_contract_scratch_bytes",
                        "matnc_mfma_config_count"):
            f.restype = c_int
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != MATNC_OK:
        msg = lib().matnc_last_error().decode(errors="replace")
        raise MatncError(rc, msg)


def int_array(values):
    values = [int(v) for v in values]
    arr = (c_int * max(1, len(values)))(*values)
    return arr


def u64_array(values):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(values, dtype=np.uint64))
    return a, a.ctypes.data_as(POINTER(c_uint64))


def f64_array(values):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
    return a, a.ctypes.data_as(POINTER(c_double))


def matnc_version() -> str:
    return lib().matnc_version().decode()


def matnc_last_error() -> str:
    return lib().matnc_last_error().decode()


def matnc_network_create(ranks, index_ids, data_c128, n_qubits, output_index_of_qubit) -> int:
    out = c_void_p()
    data, pdata = f64_array(data_c128)
    check(lib().matnc_network_create(len(ranks), int_array(ranks), int_array(index_ids), pdata, int(n_qubits),
                                     int_array(output_index_of_qubit), ctypes.byref(out)))
    return out.value


def matnc_network_destroy(net: int) -> None:
    check(lib().matnc_network_destroy(c_void_p(net)))


def matnc_plan_create(net: int, pairs, sliced_ids, open_qubits, bitstrings, precision: int, max_rank: int,
                      slice_batch: int, memory_budget: int = 0) -> int:
    out = c_void_p()
    flat = [x for p in pairs for x in p]
    words, pwords = u64_array(bitstrings)
    check(lib().matnc_plan_create(c_void_p(net), int_array(flat), len(sliced_ids), int_array(sliced_ids),
                                  len(open_qubits), int_array(open_qubits), len(words), pwords, int(precision),
                                  int(max_rank), int(slice_batch), c_size_t(int(memory_budget)),
                                  ctypes.byref(out)))
    return out.value


class PlanOptions(ctypes.Structure):
    _fields_ = [("slice_batch", c_int), ("memory_budget", c_size_t), ("half_nodes", c_int)]


def matnc_plan_create_ex(net: int, pairs, sliced_ids, open_qubits, bitstrings, precision: int, max_rank: int,
                         slice_batch: int = 1, memory_budget: int = 0, half_nodes: int = -1) -> int:
    out = c_void_p()
    flat = [x for p in pairs for x in p]
    words, pwords = u64_array(bitstrings)
    opts = PlanOptions(int(slice_batch), int(memory_budget), int(half_nodes))
    check(lib().matnc_plan_create_ex(c_void_p(net), int_array(flat), len(sliced_ids), int_array(sliced_ids),
                                     len(open_qubits), int_array(open_qubits), len(words), pwords, int(precision),
                                     int(max_rank), ctypes.byref(opts), ctypes.byref(out)))
    return out.value


def matnc_plan_info(plan: int) -> PlanInfo:
    info = PlanInfo()
    check(lib().matnc_plan_info(c_void_p(plan), ctypes.byref(info)))
    return info


def matnc_plan_set_tensor(plan: int, t: int, data_c128) -> None:
    """data_c128: 2 * 2^rank(t) doubles (the library reads exactly that many;
    the caller -- api.Contraction.set_tensor -- checks the tensor's shape)."""
    data, pdata = f64_array(data_c128)
    n = data.size // 2
    if data.ndim != 1 or data.size != 2 * n or n < 1 or n & (n - 1):
        raise ValueError("tensor data must be 2 * 2^rank interleaved doubles")
    check(lib().matnc_plan_set_tensor(c_void_p(plan), int(t), pdata))


def matnc_plan_bind(plan: int, dev_workspace: int, nbytes: int, hip_stream: int) -> None:
    check(lib().matnc_plan_bind(c_void_p(plan), c_void_p(dev_workspace), c_size_t(nbytes), c_void_p(hip_stream)))


def matnc_execute(plan: int, slice_begin: int, slice_end: int, amps_dev: int) -> None:
    check(lib().matnc_execute(c_void_p(plan), c_int64(slice_begin), c_int64(slice_end), c_void_p(amps_dev)))


def matnc_execute_timed(plan: int, slice_begin: int, slice_end: int, amps_dev: int, step: int):
    """(summed event ms, number of launches) of step's launches in the pass."""
    ms = c_double(0.0)
    n = ctypes.c_int64(0)
    check(lib().matnc_execute_timed(c_void_p(plan), c_int64(slice_begin), c_int64(slice_end), c_void_p(amps_dev),
                                    int(step), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def matnc_xeb(plan: int, amps_dev: int, xeb_dev: int) -> None:
    check(lib().matnc_xeb(c_void_p(plan), c_void_p(amps_dev), c_void_p(xeb_dev)))


def matnc_plan_destroy(plan: int) -> None:
    check(lib().matnc_plan_destroy(c_void_p(plan)))


def matnc_queue_create(plans) -> int:
    out = c_void_p()
    arr = (c_void_p * len(plans))(*[c_void_p(p) for p in plans])
    check(lib().matnc_queue_create(len(plans), arr, ctypes.byref(out)))
    return out.value


def matnc_queue_execute(queue: int, amps_devs, xeb_dev: int) -> None:
    arr = (c_void_p * len(amps_devs))(*[c_void_p(a) for a in amps_devs])
    check(lib().matnc_queue_execute(c_void_p(queue), arr, c_void_p(xeb_dev)))


def matnc_queue_workspace_bytes(queue: int) -> int:
    out = c_size_t()
    check(lib().matnc_queue_workspace_bytes(c_void_p(queue), ctypes.byref(out)))
    return int(out.value)


def matnc_queue_bind(queue: int, dev_workspace: int, nbytes: int, hip_stream: int) -> None:
    check(lib().matnc_queue_bind(c_void_p(queue), c_void_p(dev_workspace), c_size_t(nbytes), c_void_p(hip_stream)))


def matnc_queue_destroy(queue: int) -> None:
    check(lib().matnc_queue_destroy(c_void_p(queue)))


def matnc_contract_scratch_bytes() -> int:
    return int(lib().matnc_contract_scratch_bytes())


def matnc_mfma_config_count() -> int:
    return int(lib().matnc_mfma_config_count())


def matnc_contract(A: int, B: int, C: int, batch: int, posA_m, posA_k, posB_k, posB_n, posC_m, posC_n,
                   kernel: int, scratch: int, scratch_bytes: int, hip_stream: int) -> None:
    check(lib().matnc_contract(c_void_p(A), c_void_p(B), c_void_p(C), c_int64(batch), len(posA_m), len(posB_n),
                               len(posA_k), int_array(posA_m), int_array(posA_k), int_array(posB_k),
                               int_array(posB_n), int_array(posC_m), int_array(posC_n), int(kernel),
                               c_void_p(scratch), c_size_t(scratch_bytes), c_void_p(hip_stream)))


def matnc_contract_noalloc(A: int, B: int, C: int, batch: int, posA_m, posA_k, posB_k, posB_n, posC_m, posC_n,
                           kernel: int, hip_stream: int) -> None:
    check(lib().matnc_contract_noalloc(c_void_p(A), c_void_p(B), c_void_p(C), c_int64(batch), len(posA_m),
                                       len(posB_n), len(posA_k), int_array(posA_m), int_array(posA_k),
                                       int_array(posB_k), int_array(posB_n), int_array(posC_m),
                                       int_array(posC_n), int(kernel), c_void_p(hip_stream)))


def matnc_plan_reset_cache(plan: int) -> None:
    check(lib().matnc_plan_reset_cache(c_void_p(plan)))


def matnc_plan_profile(plan: int, slice_begin: int, nb: int, n_steps: int):
    """Per-step (time_ms, kernel id, cmac, bytes) of one profiled batch."""
    t = (ctypes.c_float * max(1, n_steps))()
    k = (c_int * max(1, n_steps))()
    c = (c_double * max(1, n_steps))()
    b = (c_double * max(1, n_steps))()
    check(lib().matnc_plan_profile(c_void_p(plan), c_int64(slice_begin), int(nb), t, k, c, b))
    return [(t[j], k[j], c[j], b[j]) for j in range(n_steps)]


def matnc_plan_autotune(plan: int, reps: int = 3, cache_path=None) -> None:
    path = cache_path.encode() if cache_path else None
    check(lib().matnc_plan_autotune(c_void_p(plan), int(reps), path))
