"""ctypes binding of libpq.so (argument marshalling only).

torch is imported first so that libpq.so binds to the HIP runtime torch has
already loaded (both carry the soname libamdhip64.so.7); device memory and
streams then come from torch.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load order: torch's HIP runtime first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpq.so")

PQ_OK, PQ_EINVAL, PQ_ERANGE, PQ_ENOMEM, PQ_EDEVICE, PQ_ECANCELLED = range(6)
PQ_OP_PERM, PQ_OP_EXTEND_ROW = 0, 1
PQ_FAULT_NONE, PQ_FAULT_ALLOC, PQ_FAULT_LAUNCH = 0, 1, 2
PQ_MAX_N = 48
PQ_GRAD_MAX_DIM = 32
PQ_ALL_MAX_OUTPUTS = 1 << 31
PQ_NOALLOC_SCRATCH_BYTES = 160 * 1024


class pq_c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class pq_job(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("nr", ctypes.c_int32),
        ("nc", ctypes.c_int32),
        ("row_idx", ctypes.POINTER(ctypes.c_int32)),
        ("row_mult", ctypes.POINTER(ctypes.c_int32)),
        ("col_idx", ctypes.POINTER(ctypes.c_int32)),
        ("col_mult", ctypes.POINTER(ctypes.c_int32)),
        ("out_offset", ctypes.c_int64),
    ]


class pq_plan_info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("n", ctypes.c_int32), ("trivial", ctypes.c_int32),
        ("transposed", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
        ("fixed_row", ctypes.c_int32), ("lane_digits", ctypes.c_int32),
        ("lane_states", ctypes.c_int32), ("time_digits", ctypes.c_int32),
        ("inner_digits", ctypes.c_int32), ("inner_states", ctypes.c_int32),
        ("binary", ctypes.c_int32), ("terms", ctypes.c_uint64),
        ("time_states", ctypes.c_uint64), ("log2_norm", ctypes.c_double),
    ]


class PqError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        super().__init__(f"pq status {status}: {detail}")


_I32P = ctypes.POINTER(ctypes.c_int32)
_VP = ctypes.c_void_p

_SIGNATURES = {
    "pq_version": ([], ctypes.c_char_p),
    "pq_device_peak": ([_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                        ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "pq_create": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int], ctypes.c_int),
    "pq_destroy": ([_VP], None),
    "pq_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "pq_last_error": ([_VP], ctypes.c_char_p),
    "pq_perm": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, _I32P, _I32P, _VP, _VP, _VP], ctypes.c_int),
    "pq_perm_noalloc": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, _I32P, _I32P, _VP, _VP, _VP], ctypes.c_int),
    "pq_perm_batched": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(pq_job), ctypes.c_int32,
                         _VP, _VP, _VP], ctypes.c_int),
    "pq_perm_many": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(pq_job), ctypes.c_int32,
                      _VP, _VP, _VP], ctypes.c_int),
    "pq_perm_grad": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _I32P, _I32P, _VP, _VP,
                      _VP, ctypes.c_int64, _VP], ctypes.c_int),
    "pq_plan_describe": ([ctypes.c_int32, _I32P, _I32P, ctypes.POINTER(pq_plan_info)], ctypes.c_int),
    "pq_gray_unrank": ([ctypes.c_int32, _I32P, ctypes.c_uint64, _I32P], ctypes.c_int),
    "pq_profile_enable": ([_VP, ctypes.c_int], ctypes.c_int),
    "pq_mesh_unitary": ([_VP, ctypes.c_int32, ctypes.c_int32, _I32P, _VP, _VP, ctypes.c_int64, _VP], ctypes.c_int),
    "pq_mesh_unitary_vjp": ([_VP, ctypes.c_int32, ctypes.c_int32, _I32P, _VP, _VP, ctypes.c_int64, _VP, _VP],
                            ctypes.c_int),
    "pq_neg_log_prob": ([_VP, ctypes.c_int32, _VP, _VP, _VP, _VP], ctypes.c_int),
    "pq_neg_log_prob_vjp": ([_VP, ctypes.c_int32, _VP, _VP, _VP, _VP], ctypes.c_int),
    "pq_profile_read": ([_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "pq_perm_all_outputs": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, _I32P, _VP, _VP, _VP], ctypes.c_int),
    "pq_fock_count": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int64),
    "pq_loss_dilation": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _VP,
                          ctypes.c_int64, _VP], ctypes.c_int),
    "pq_loss_dilation_vw": ([_VP, _VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), _VP, ctypes.c_int64,
                             ctypes.c_int32, _VP, ctypes.c_int64, _VP], ctypes.c_int),
    "pq_sample_chain": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP,
                         _VP], ctypes.c_int),
    "pq_fock_unrank": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _I32P], ctypes.c_int),
    "pq_lhaf": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _I32P, _VP, _VP], ctypes.c_int),
    "pq_lhaf_many": ([_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _I32P, ctypes.c_int32, _VP, _VP],
                     ctypes.c_int),
    "pq_autotune_enable": ([_VP, ctypes.c_int], ctypes.c_int),
    "pq_cancel": ([_VP, ctypes.c_int], ctypes.c_int),
    "pq_fault_inject": ([_VP, ctypes.c_int], ctypes.c_int),
    "pq_graph_enable": ([_VP, ctypes.c_int], ctypes.c_int),
    "pq_walk_variant": ([_VP, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "pq_queue_mode": ([_VP, ctypes.c_int], ctypes.c_int),
    "pq_lhaf_pack": ([_VP, ctypes.c_int], ctypes.c_int),
    "pq_all_outputs_gemm": ([_VP, ctypes.c_int], ctypes.c_int),
    "pq_autotune_last": ([_VP, _I32P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _I32P],
                         ctypes.c_int),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libpq.so (built by paper_2403_04006_amd._build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def i32_array(values) -> ctypes.Array:
    vals = [int(v) for v in values]
    return (ctypes.c_int32 * max(1, len(vals)))(*vals)
