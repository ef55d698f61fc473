"""ctypes declarations of the C ABI in ``include/tlfea.h`` (argument marshalling only).

The library is the in-tree ``lib/libtlfea.so`` built by ``build.py``.  There is
no fallback: if it is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libtlfea.so")

TLFEA_OK = 0
TLFEA_T10 = 1
TLFEA_ANCF3443 = 2
TLFEA_ANCF3243 = 3
TLFEA_SVK = 1
TLFEA_MOONEY_RIVLIN = 2
TLFEA_FP64 = 0
TLFEA_MIXED = 1
TLFEA_FLAG_INVERTED = 1
TLFEA_FLAG_NONFINITE = 2

EXPORTED = [
    "tlfea_status_string", "tlfea_version", "tlfea_mesh_create", "tlfea_mesh_destroy", "tlfea_mesh_info",
    "tlfea_mesh_set_material", "tlfea_mesh_set_precision", "tlfea_build_csr_pattern", "tlfea_get_csr_pattern",
    "tlfea_get_slot_map", "tlfea_internal_force", "tlfea_internal_force_noalloc", "tlfea_tangent", "tlfea_tangent_ex", "tlfea_assemble",
    "tlfea_assemble_ex", "tlfea_assemble_accumulate", "tlfea_assemble_points", "tlfea_assemble_nodes", "tlfea_internal_force_vjp", "tlfea_internal_force_p", "tlfea_internal_force_vjp_p", "tlfea_get_runtime_flags", "tlfea_batch_create",
    "tlfea_batch_destroy", "tlfea_batch_offsets", "tlfea_batch_assemble", "tlfea_batch_assemble_loop",
    "tlfea_mesh_set_gather_shape", "tlfea_mesh_get_gather_shape", "tlfea_mesh_autotune",
    "tlfea_batch_set_gather_shape", "tlfea_batch_get_gather_shape", "tlfea_batch_autotune",
    "tlfea_batch_set_schedule", "tlfea_batch_get_schedule",
    "tlfea_build_mass", "tlfea_get_mass", "tlfea_assemble_newton", "tlfea_assemble_newton_upper",
    "tlfea_newton_gradient",
    "tlfea_build_upper_pattern", "tlfea_get_csr_pattern_upper", "tlfea_assemble_upper", "tlfea_adamw_solve",
]


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("elem_type", ctypes.c_int32),
        ("n_coef", ctypes.c_int64),
        ("n_elem", ctypes.c_int64),
        ("h_conn", ctypes.POINTER(ctypes.c_int32)),
        ("h_X", ctypes.POINTER(ctypes.c_double)),
        ("gl", ctypes.c_int32 * 3),
        ("thickness", ctypes.c_double),
        ("material", ctypes.c_int32),
        ("params", ctypes.c_double * 3),
        ("kv_eta", ctypes.c_double),
        ("kv_lambda", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("width", ctypes.c_double),
    ]


class GatherShape(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("range_tasks", ctypes.c_int32), ("range_values", ctypes.c_int32)]

    def as_dict(self):
        return {"waves": self.waves, "range_tasks": self.range_tasks, "range_values": self.range_values}


class AdamwParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("weight_decay", ctypes.c_double)]


class TlfeaError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "tlfea_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "tlfea_version": ([], ctypes.c_int),
        "tlfea_mesh_create": ([P(MeshDesc), P(vp)], ctypes.c_int),
        "tlfea_mesh_destroy": ([vp], ctypes.c_int),
        "tlfea_mesh_info": ([vp, P(i64), P(i64), P(i64), P(i32), P(i32)], ctypes.c_int),
        "tlfea_mesh_set_material": ([vp, i32, P(dbl), dbl, dbl], ctypes.c_int),
        "tlfea_mesh_set_precision": ([vp, i32], ctypes.c_int),
        "tlfea_build_csr_pattern": ([vp, P(i64)], ctypes.c_int),
        "tlfea_get_csr_pattern": ([vp, vp, vp, i32, vp], ctypes.c_int),
        "tlfea_get_slot_map": ([vp, i64, i64, vp, i32, vp], ctypes.c_int),
        "tlfea_internal_force": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "tlfea_internal_force_noalloc": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "tlfea_tangent": ([vp, vp, vp, dbl, vp, vp], ctypes.c_int),
        "tlfea_tangent_ex": ([vp, vp, vp, dbl, dbl, vp, vp], ctypes.c_int),
        "tlfea_assemble": ([vp, vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "tlfea_assemble_ex": ([vp, vp, vp, dbl, dbl, vp, vp, vp], ctypes.c_int),
        "tlfea_assemble_accumulate": ([vp, vp, vp, dbl, dbl, vp, vp, vp], ctypes.c_int),
        "tlfea_assemble_points": ([vp, vp, vp, dbl, dbl, i32, vp], ctypes.c_int),
        "tlfea_assemble_nodes": ([vp, vp, vp, i32, vp], ctypes.c_int),
        "tlfea_internal_force_vjp": ([vp, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "tlfea_internal_force_p": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "tlfea_internal_force_vjp_p": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "tlfea_get_runtime_flags": ([vp, P(ctypes.c_uint32)], ctypes.c_int),
        "tlfea_batch_create": ([P(vp), i32, P(vp)], ctypes.c_int),
        "tlfea_batch_destroy": ([vp], ctypes.c_int),
        "tlfea_batch_offsets": ([vp, P(i64), P(i64)], ctypes.c_int),
        "tlfea_batch_assemble": ([vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "tlfea_batch_assemble_loop": ([vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "tlfea_mesh_set_gather_shape": ([vp, P(GatherShape)], ctypes.c_int),
        "tlfea_mesh_get_gather_shape": ([vp, P(GatherShape), P(i64)], ctypes.c_int),
        "tlfea_mesh_autotune": ([vp, vp, vp, dbl, vp, vp, i32, vp, P(GatherShape), P(ctypes.c_float)], ctypes.c_int),
        "tlfea_batch_set_gather_shape": ([vp, P(GatherShape)], ctypes.c_int),
        "tlfea_batch_get_gather_shape": ([vp, P(GatherShape), P(i64)], ctypes.c_int),
        "tlfea_batch_set_schedule": ([vp, i32, i32], ctypes.c_int),
        "tlfea_batch_get_schedule": ([vp, P(i32), P(i32), P(i32), P(i32)], ctypes.c_int),
        "tlfea_batch_autotune": ([vp, vp, vp, vp, vp, vp, i32, vp, P(GatherShape), P(ctypes.c_float)], ctypes.c_int),
        "tlfea_build_mass": ([vp, dbl], ctypes.c_int),
        "tlfea_get_mass": ([vp, vp, vp], ctypes.c_int),
        "tlfea_assemble_newton": ([vp, vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "tlfea_assemble_newton_upper": ([vp, vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "tlfea_newton_gradient": ([vp, vp, vp, vp, vp, dbl, vp, vp], ctypes.c_int),
        "tlfea_build_upper_pattern": ([vp, P(i64)], ctypes.c_int),
        "tlfea_get_csr_pattern_upper": ([vp, vp, vp, i32, vp], ctypes.c_int),
        "tlfea_assemble_upper": ([vp, vp, vp, dbl, dbl, vp, vp, vp], ctypes.c_int),
        "tlfea_adamw_solve": ([vp, P(AdamwParams), dbl, vp, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, P(i32), P(dbl),
                               vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def status_string(status: int) -> str:
    try:
        return lib().tlfea_status_string(int(status)).decode()
    except RuntimeError:
        return "library not loaded"


def check(status: int, what: str) -> None:
    if status != TLFEA_OK:
        raise TlfeaError(status, what)
