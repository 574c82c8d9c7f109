"""ctypes declarations of the C ABI in ``include/rdm.h``.

Loading fails loudly (ImportError) when ``librdm.so`` has not been built:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librdm.so")

RDM_OK, RDM_E_INVALID, RDM_E_NOMEM, RDM_E_DEVICE, RDM_E_NONFINITE, RDM_E_BUSY = 0, -1, -2, -3, -4, -5
RDM_E_CANCELLED = -6
RDM_FP64, RDM_MIXED = 0, 1
RDM_AUTO, RDM_STORED_Q, RDM_TWO_PASS = 0, 1, 2
RDM_PER_COLUMN, RDM_BLOCK, RDM_METHOD_AUTO = 0, 1, 2
RDM_APPLY_AUTO, RDM_APPLY_HOPS, RDM_APPLY_TRANSFORM, RDM_APPLY_HOPS_ROWS = 0, 1, 2, 3
DIAG_FIXED = 16
NOALLOC_MAX_BYTES = 64 << 20  # RDM_NOALLOC_MAX_BYTES

STATUS_NAMES = {0: "RDM_OK", -1: "RDM_E_INVALID", -2: "RDM_E_NOMEM", -3: "RDM_E_DEVICE",
                -4: "RDM_E_NONFINITE", -5: "RDM_E_BUSY", -6: "RDM_E_CANCELLED"}


class Coupling(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("jx", C.c_double), ("jy", C.c_double),
                ("jz", C.c_double)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("mode", C.c_int32), ("hbm_budget", C.c_uint64),
                ("slab", C.c_int32), ("rows_per_lane", C.c_int32), ("tau", C.c_double),
                ("profile", C.c_int32), ("eager", C.c_int32), ("method", C.c_int32), ("reserved", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("rho", C.POINTER(C.c_double)), ("h_star", C.POINTER(C.c_double)),
                ("log_z", C.POINTER(C.c_double)), ("entropy", C.POINTER(C.c_double)),
                ("diag", C.POINTER(C.c_double))]


class GroundResult(C.Structure):
    _fields_ = [("rho", C.POINTER(C.c_double)), ("e_total", C.POINTER(C.c_double)),
                ("e_bath", C.POINTER(C.c_double)), ("entropy", C.POINTER(C.c_double)),
                ("degeneracy", C.POINTER(C.c_int32)), ("residual", C.POINTER(C.c_double))]


class ProductResult(C.Structure):
    _fields_ = [("log_z", C.POINTER(C.c_double)), ("log_z_t", C.POINTER(C.c_double)),
                ("log_z_b", C.POINTER(C.c_double)), ("samples", C.POINTER(C.c_double))]


class BatchItem(C.Structure):
    _fields_ = [("h", C.c_void_p), ("beta", C.POINTER(C.c_double)), ("n_beta", C.c_int32),
                ("n_v", C.c_int32), ("k", C.c_int32), ("seed", C.c_uint64), ("out", Result),
                ("status", C.c_int32)]


# (name, restype, argtypes) of every exported function
SIGNATURES = [
    ("rdm_hamiltonian_create", C.c_int32,
     [C.c_int32, C.c_int32, C.POINTER(Coupling), C.c_int64, C.POINTER(C.c_double),
      C.POINTER(C.c_double), C.POINTER(C.c_void_p)]),
    ("rdm_hamiltonian_create_ex", C.c_int32,
     [C.c_int32, C.c_int32, C.POINTER(Coupling), C.c_int64, C.POINTER(C.c_double),
      C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_void_p)]),
    ("rdm_hamiltonian_destroy", None, [C.c_void_p]),
    ("rdm_hamiltonian_info", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("rdm_system_hamiltonian", C.c_int32, [C.c_void_p, C.POINTER(C.c_double)]),
    ("rdm_energy_deviation", C.c_int32,
     [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
      C.POINTER(C.c_double)]),
    ("rdm_solve", C.c_int32,
     [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
      C.POINTER(Options), C.c_void_p, C.POINTER(Result)]),
    ("rdm_workspace_size", C.c_int32,
     [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Options), C.POINTER(C.c_uint64)]),
    ("rdm_solve_ws", C.c_int32,
     [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
      C.POINTER(Options), C.c_void_p, C.POINTER(Result), C.c_void_p, C.c_uint64]),
    ("rdm_solve_noalloc", C.c_int32,
     [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
      C.POINTER(Options), C.c_void_p, C.POINTER(Result)]),
    ("rdm_solve_batch", C.c_int32, [C.c_int32, C.POINTER(BatchItem), C.POINTER(Options), C.c_void_p]),
    ("rdm_solve_batch_ws", C.c_int32,
     [C.c_int32, C.POINTER(BatchItem), C.POINTER(Options), C.c_void_p, C.c_void_p, C.c_uint64]),
    ("rdm_batch_workspace_size", C.c_int32,
     [C.c_int32, C.POINTER(BatchItem), C.POINTER(Options), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    ("rdm_apply", C.c_int32,
     [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(Options),
      C.c_void_p]),
    ("rdm_start_block", C.c_int32,
     [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p]),
    ("rdm_lanczos", C.c_int32,
     [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(Options), C.c_void_p,
      C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("rdm_tridiag_fa", C.c_int32,
     [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
      C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("rdm_block_quadrature", C.c_int32,
     [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double), C.c_double,
      C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("rdm_ground_state", C.c_int32,
     [C.c_void_p, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(Options), C.c_void_p, C.POINTER(GroundResult)]),
    ("rdm_product_trace", C.c_int32,
     [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(Options),
      C.c_void_p, C.POINTER(ProductResult)]),
    ("rdm_stream_probe", C.c_int32, [C.c_int32, C.c_uint64, C.c_int32, C.c_void_p, C.POINTER(C.c_double)]),
    ("rdm_high_temperature_term", C.c_int32,
     [C.c_void_p, C.c_int32, C.c_uint64, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("rdm_server_create", C.c_int32, [C.c_uint64, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]),
    ("rdm_server_submit", C.c_int32,
     [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
      Result, C.POINTER(C.c_uint64)]),
    ("rdm_server_poll", C.c_int32,
     [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("rdm_server_wait", C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]),
    ("rdm_server_cancel", C.c_int32, [C.c_void_p, C.c_uint64]),
    ("rdm_server_stats", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("rdm_server_destroy", None, [C.c_void_p]),
    ("rdm_last_error", C.c_char_p, []),
]


def load(path: str = LIB_PATH):
    # torch bundles its own HIP runtime (same SONAME as /opt/rocm's).  Loading
    # torch first makes librdm.so bind to that one copy, so device memory and
    # streams handed over from torch belong to the runtime that launches the
    # kernels; loading librdm.so first would put two HIP runtimes in the process.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2204_08147_amd/build.py` "
                          "(there is no fallback implementation)")
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
