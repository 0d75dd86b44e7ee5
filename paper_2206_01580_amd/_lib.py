"""ctypes binding of ``libsorf.so`` (the C ABI in ``include/sorf.h``).

Argument marshalling only: every computation runs in the HIP library. Loading
fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsorf.so")

SORF_OK = 0
SORF_ERR_INVALID_ARG = 1
SORF_ERR_UNSUPPORTED = 2
SORF_ERR_DEVICE = 3
SORF_ERR_WORKSPACE = 4
SORF_ERR_BUSY = 5

# bytes of the fixed device scratch array behind sorf_predict_noalloc
PREDICT_NOALLOC_SCRATCH_BYTES = 64 << 20

GRAM_MODES = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16_hilo": 3, "fp16_hilo": 4,
              "fp32_kahan": 5}

# every function the header declares; the load test checks each is exported
EXPORTS = (
    "sorf_abi_version", "sorf_status_string", "sorf_forward", "sorf_backward",
    "sorf_energy_grad_workspace_bytes", "sorf_energy_grad", "sorf_derivative_features", "sorf_project_workspace_bytes", "sorf_project",
    "sorf_projection_fit_workspace_bytes", "sorf_projection_fit",
    "sorf_fchl19_length", "sorf_fchl19_forward", "sorf_fchl19_backward",
    "sorf_gram_workspace_bytes", "sorf_gram_accumulate", "sorf_gram_accumulate_f64",
    "sorf_gram_split_workspace_bytes", "sorf_gram_accumulate_split",
    "sorf_solve_workspace_bytes",
    "sorf_solve", "sorf_solve_f64", "sorf_solve_streams_create", "sorf_solve_streams_destroy",
    "sorf_solve_streamed", "sorf_solve_f64_streamed",
    "sorf_predict_workspace_bytes", "sorf_predict", "sorf_predict_noalloc",
    "sorf_forces_workspace_bytes", "sorf_forces",
    "sorf_validate_batch", "sorf_server_workspace_bytes", "sorf_server_start", "sorf_server_submit",
    "sorf_server_query", "sorf_server_energies", "sorf_server_forces", "sorf_server_stop",
)


class SorfModel(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("n_stacks", ctypes.c_int32),
        ("n_transforms", ctypes.c_int32),
        ("n_elements", ctypes.c_int32),
        ("sigma", ctypes.c_float),
        ("signs", ctypes.c_void_p),
        ("bias", ctypes.c_void_p),
    ]


class SorfBatch(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p),
        ("element", ctypes.c_void_p),
        ("mol_ptr", ctypes.c_void_p),
        ("n_atoms", ctypes.c_int64),
        ("n_mols", ctypes.c_int64),
    ]


class SorfFchl19Params(ctypes.Structure):
    _fields_ = [
        ("n2", ctypes.c_int32),
        ("n3", ctypes.c_int32),
        ("eta2", ctypes.c_float),
        ("eta3", ctypes.c_float),
        ("N2", ctypes.c_float),
        ("N3", ctypes.c_float),
        ("c3", ctypes.c_float),
        ("zeta", ctypes.c_float),
        ("rcut", ctypes.c_float),
    ]


class SorfSolveStreams(ctypes.Structure):
    _fields_ = [
        ("side", ctypes.c_void_p),
        ("event_fork", ctypes.c_void_p),
        ("event_join", ctypes.c_void_p),
    ]


class SorfServerConfig(ctypes.Structure):
    _fields_ = [
        ("max_batch_atoms", ctypes.c_int64),
        ("ring_slots", ctypes.c_int32),
        ("idle_timeout_s", ctypes.c_double),
    ]


class SorfError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {status_string(code)} ({code})")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the built library (once). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2206_01580_amd.build); there is no CPU fallback")
    # PyTorch ships its own HIP runtime (torch/lib/libamdhip64.so, soname
    # libamdhip64.so.7). Loaded first, it is the runtime this library binds to.
    # Loaded after this library, torch would bring in a second runtime beside
    # /opt/rocm's, and streams handed from one to the other make every launch
    # fail. So torch, when installed, is imported before the library is opened.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    MP, BP = ctypes.POINTER(SorfModel), ctypes.POINTER(SorfBatch)
    SP = ctypes.POINTER(SorfSolveStreams)
    sig = {
        "sorf_abi_version": (i32, []),
        "sorf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "sorf_forward": (ctypes.c_int, [MP, BP, P, P]),
        "sorf_backward": (ctypes.c_int, [MP, BP, P, P, P, P]),
        "sorf_energy_grad_workspace_bytes": (sz, [i64]),
        "sorf_energy_grad": (ctypes.c_int, [MP, BP, P, P, P, P, sz, P]),
        "sorf_derivative_features": (ctypes.c_int, [MP, BP, P, P, P, P]),
        "sorf_project_workspace_bytes": (sz, [i64, i32]),
        "sorf_project": (ctypes.c_int, [i64, i32, P, P, i32, P, i32, P, P, sz, P]),
        "sorf_projection_fit_workspace_bytes": (sz, [i32]),
        "sorf_projection_fit": (ctypes.c_int, [i64, i32, P, i32, P, P, P, sz, P]),
        "sorf_fchl19_length": (i64, [i32, ctypes.POINTER(SorfFchl19Params)]),
        "sorf_fchl19_forward": (ctypes.c_int, [P, P, P, i64, i64, i32,
                                               ctypes.POINTER(SorfFchl19Params), P, P]),
        "sorf_fchl19_backward": (ctypes.c_int, [P, P, P, i64, i64, i32,
                                                ctypes.POINTER(SorfFchl19Params), P, P, P]),
        "sorf_gram_workspace_bytes": (sz, [i64, i32, ctypes.c_int]),
        "sorf_gram_accumulate": (ctypes.c_int, [i64, i32, P, P, ctypes.c_int, i32, P, P, P, sz,
                                                P]),
        "sorf_gram_accumulate_f64": (ctypes.c_int, [i64, i32, P, P, P, P, P]),
        "sorf_gram_split_workspace_bytes": (sz, [i64, i32]),
        "sorf_gram_accumulate_split": (ctypes.c_int, [i64, i32, P, P, P, P, P, sz, P]),
        "sorf_solve_workspace_bytes": (sz, [i32]),
        "sorf_solve_f64": (ctypes.c_int, [i32, P, P, f64, i32, P, P, P, sz, P]),
        "sorf_solve": (ctypes.c_int, [i32, P, P, f64, i32, P, P, P, sz, P]),
        "sorf_solve_streams_create": (ctypes.c_int, [SP]),
        "sorf_solve_streams_destroy": (ctypes.c_int, [SP]),
        "sorf_solve_streamed": (ctypes.c_int, [i32, P, P, f64, i32, P, P, P, sz, SP, P]),
        "sorf_solve_f64_streamed": (ctypes.c_int, [i32, P, P, f64, i32, P, P, P, sz, SP, P]),
        "sorf_predict_workspace_bytes": (sz, [MP, i64, i64]),
        "sorf_predict": (ctypes.c_int, [MP, BP, P, P, P, P, P, P, sz, P]),
        "sorf_predict_noalloc": (ctypes.c_int, [MP, BP, P, P, P, P, P, P]),
        "sorf_forces_workspace_bytes": (sz, [i64, i64]),
        "sorf_forces": (ctypes.c_int, [i32, i64, i64, P, P, P, P, P, P, sz, P]),
        "sorf_validate_batch": (ctypes.c_int, [BP, i32, P, P]),
        "sorf_server_workspace_bytes": (sz, [MP, ctypes.POINTER(SorfServerConfig)]),
        "sorf_server_start": (ctypes.c_int, [MP, P, P, P, P, ctypes.POINTER(SorfServerConfig), P, sz,
                                             P, ctypes.POINTER(P)]),
        "sorf_server_submit": (ctypes.c_int, [P, i32, P, P, ctypes.POINTER(i64)]),
        "sorf_server_query": (i32, [P, i64]),
        "sorf_server_energies": (ctypes.POINTER(ctypes.c_float), [P, i64]),
        "sorf_server_forces": (ctypes.POINTER(ctypes.c_float), [P, i64]),
        "sorf_server_stop": (ctypes.c_int, [P, ctypes.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(code: int) -> str:
    try:
        return load().sorf_status_string(code).decode()
    except Exception:  # pragma: no cover - only used for messages
        return str(code)


def check(fn: str, code: int) -> None:
    if code != SORF_OK:
        raise SorfError(fn, code)
