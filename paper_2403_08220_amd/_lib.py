"""ctypes declarations of the C ABI in include/dino.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdino.so")

DINO_OK = 0
STATUS_NAMES = {0: "DINO_OK", -1: "DINO_EINVAL", -2: "DINO_ENOMEM", -3: "DINO_EDEVICE", -4: "DINO_ESTATE",
                -5: "DINO_ENUMERIC"}

LAYER_KINDS = {"linear": 0, "act": 1, "resid": 2}
PRECISIONS = {"f64": 0, "bf16": 1, "fp8": 2, "fp8_single": 3}
FACTORIZATIONS = {"primal": 0, "dual": 1, "auto": 2}
TUNE_KINDS = {"chol": 0, "fwd64": 1, "fwd32": 2, "hess": 3, "fwdchain": 4, "dualsolve": 5}
LAUNCH_MODES = {"eager": 0, "graph": 1}
METHODS = {"mmala": 0, "pcn": 1, "mala": 2, "lapcn": 3, "da_mmala": 4, "dis_mmala": 5}


class DinoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class ProblemDesc(ct.Structure):
    _fields_ = [
        ("n_chains", ct.c_int32),
        ("d_y", ct.c_int32),
        ("precision", ct.c_int32),
        ("track_complement", ct.c_int32),
        ("trace_capacity", ct.c_int32),
        ("factorization", ct.c_int32),
        ("dt", ct.c_double),
        ("seed", ct.c_uint64),
        ("request_id", ct.c_uint64),
        ("method", ct.c_int32),
    ]


MAX_BUCKETS = 8


class ServerCfg(ct.Structure):
    _fields_ = [
        ("n_buckets", ct.c_int32),
        ("bucket_dy", ct.c_int32 * MAX_BUCKETS),
        ("bucket_slots", ct.c_int32 * MAX_BUCKETS),
        ("max_requests", ct.c_int32),
        ("steps_per_quantum", ct.c_int32),
        ("precision", ct.c_int32),
        ("track_complement", ct.c_int32),
        ("factorization", ct.c_int32),
        ("dt", ct.c_double),
        ("hbm_budget_bytes", ct.c_double),
    ]


class Request(ct.Structure):
    _fields_ = [
        ("seed", ct.c_uint64),
        ("request_id", ct.c_uint64),
        ("d_y", ct.c_int32),
        ("n_chains", ct.c_int32),
        ("n_steps", ct.c_int64),
        ("y", ct.POINTER(ct.c_double)),
        ("noise_var", ct.POINTER(ct.c_double)),
        ("arrival", ct.c_double),
    ]


class Result(ct.Structure):
    _fields_ = [
        ("request_id", ct.c_uint64),
        ("d_y", ct.c_int32),
        ("n_chains", ct.c_int32),
        ("n_steps", ct.c_int64),
        ("arrival", ct.c_double),
        ("admitted", ct.c_double),
        ("finished", ct.c_double),
        ("accepts", ct.c_int64),
        ("failures", ct.c_int64),
    ]


_P = ct.c_void_p
_D = ct.POINTER(ct.c_double)
_F = ct.POINTER(ct.c_float)
_I32 = ct.POINTER(ct.c_int32)
_I64 = ct.POINTER(ct.c_int64)

SIGNATURES = {
    "dino_last_error": (ct.c_char_p, []),
    "dino_version": (ct.c_char_p, []),
    "dino_ctx_create": (ct.c_int32, [ct.c_int, ct.POINTER(_P)]),
    "dino_ctx_destroy": (ct.c_int32, [_P]),
    "dino_load_prior": (ct.c_int32, [_P, ct.c_int, ct.c_double, ct.c_double, ct.c_int]),
    "dino_read_basis": (ct.c_int32, [_P, _D, _D, _D, _I32]),
    "dino_load_basis": (ct.c_int32, [_P, ct.c_int, _D, _D]),
    "dino_load_network": (ct.c_int32, [_P, ct.c_int, _I32, _I32, _I32, ct.POINTER(_D), ct.POINTER(_D)]),
    "dino_load_true_model": (ct.c_int32, [_P, ct.c_int, _I32, _I32, _I32, ct.POINTER(_D), ct.POINTER(_D)]),
    "dino_read_delayed": (ct.c_int32, [_P, _D, _I64]),
    "dino_eval_true_misfit": (ct.c_int32, [_P, ct.c_int, _P, _P, _P]),
    "dino_problem_workspace_bytes": (ct.c_int32, [_P, ct.POINTER(ProblemDesc), ct.POINTER(ct.c_size_t)]),
    "dino_problem_create": (ct.c_int32, [_P, ct.POINTER(ProblemDesc), _D, _D, _P, ct.c_size_t, ct.POINTER(_P)]),
    "dino_problem_destroy": (ct.c_int32, [_P]),
    "dino_chains_init": (ct.c_int32, [_P, _D, _F, _P]),
    "dino_step": (ct.c_int32, [_P, ct.c_int, _P]),
    "dino_set_fixed_metric": (ct.c_int32, [_P, _D, _D]),
    "dino_read_states": (ct.c_int32, [_P, _D, _F]),
    "dino_read_cache": (ct.c_int32, [_P, _D, _D, _D]),
    "dino_read_diagnostics": (ct.c_int32, [_P, _I64, _I64, _I64]),
    "dino_read_trace": (ct.c_int32, [_P, _F, _D, _I64]),
    "dino_posterior": (ct.c_int32, [_P, ct.c_int, _D, _D, _D, _D]),
    "dino_ess": (ct.c_int32, [_P, ct.c_int, _D]),
    "dino_eval_geometry": (ct.c_int32, [_P, ct.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dino_eval_propose": (ct.c_int32, [_P, ct.c_int, _P, _P, _P, _P, _P, _P]),
    "dino_eval_log_rho": (ct.c_int32, [_P, ct.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dino_eval_normals": (ct.c_int32, [_P, ct.c_int, ct.c_int, ct.c_int64, ct.c_int, _P, _P]),
    "dino_eval_jacobian": (ct.c_int32, [_P, ct.c_int, _P, _P, _P]),
    "dino_jacobian_ld": (ct.c_int32, [_P, _I32]),
    "dino_eval_propose_dual": (ct.c_int32, [_P, ct.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dino_eval_log_rho_dual": (ct.c_int32, [_P, ct.c_int] + [_P] * 13 + [_P]),
    "dino_set_profiling": (ct.c_int32, [_P, ct.c_int]),
    "dino_set_launch_mode": (ct.c_int32, [_P, ct.c_int, ct.c_int]),
    "dino_autotune": (ct.c_int32, [_P, _P, _I32]),
    "dino_tune_set": (ct.c_int32, [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32]),
    "dino_tuning_table": (ct.c_int32, [ct.c_char_p, ct.c_size_t, ct.POINTER(ct.c_size_t)]),
    "dino_read_profile": (ct.c_int32, [_P, _D, _I32, _I64]),
    "dino_stage_name": (ct.c_char_p, [ct.c_int]),
    "dino_encode": (ct.c_int32, [_P, ct.c_int, _P, _P, _P, _P]),
    "dino_decode": (ct.c_int32, [_P, ct.c_int, _P, _P, _P, _P]),
    "dino_encode_noalloc": (ct.c_int32, [_P, ct.c_int, _P, _P, _P, _P]),
    "dino_server_create": (ct.c_int32, [_P, ct.POINTER(ServerCfg), ct.POINTER(_P)]),
    "dino_server_destroy": (ct.c_int32, [_P]),
    "dino_server_clock": (ct.c_int32, [_P, ct.POINTER(ct.c_double)]),
    "dino_server_submit": (ct.c_int32, [_P, ct.POINTER(Request)]),
    "dino_server_run": (ct.c_int32, [_P, ct.c_double, ct.POINTER(ct.c_int)]),
    "dino_server_poll": (ct.c_int32, [_P, ct.c_int, ct.POINTER(Result), _D, ct.POINTER(ct.c_int)]),
    "dino_server_stats": (ct.c_int32, [_P, _I64, _I64, _I64]),
}

N_STAGES = 10

_lib = None


def load():
    """Load libdino.so from the package directory. Fails loudly when it is missing:
    there is no other implementation of the path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2403_08220_amd.build` "
                          "(hipcc for gfx950); there is no fallback path")
    # torch first: torch's bundled HIP runtime and the one libdino.so links against share
    # a soname, so whichever is loaded first serves the whole process. Loading torch's
    # first gives the library and torch one runtime (the one torch was built with)
    # whatever the caller imported before.
    import torch  # noqa: F401

    lib = ct.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != DINO_OK:
        msg = load().dino_last_error().decode()
        raise DinoError(status, msg)


def dptr(a):
    """ctypes double* of a C-contiguous float64 numpy array (or None)."""
    return None if a is None else a.ctypes.data_as(_D)


def fptr(a):
    return None if a is None else a.ctypes.data_as(_F)


def i32ptr(a):
    return None if a is None else a.ctypes.data_as(_I32)


def i64ptr(a):
    return None if a is None else a.ctypes.data_as(_I64)
