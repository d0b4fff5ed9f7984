"""ctypes binding of the C ABI declared in include/ohm.h.

Argument marshalling only: every computation runs in the HIP library.  The
functions keep the C names; fields are torch tensors on the GPU (their device
pointers are passed), streams default to torch's current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libohm.so")

OHM_OK, OHM_ERR_ARG, OHM_ERR_LAYOUT, OHM_ERR_NOMEM, OHM_ERR_HIP, OHM_ERR_NOCONV, OHM_ERR_NONFINITE = range(7)
OHM_F64, OHM_F32 = 0, 1
MAX_LEVELS = 8
STATUS_NAMES = {0: "OHM_OK", 1: "OHM_ERR_ARG", 2: "OHM_ERR_LAYOUT", 3: "OHM_ERR_NOMEM", 4: "OHM_ERR_HIP",
                5: "OHM_ERR_NOCONV", 6: "OHM_ERR_NONFINITE"}

EXPORTS = ["ohm_hier_create", "ohm_hier_destroy", "ohm_hier_level_info", "ohm_hier_problem_info",
           "ohm_hier_device_bytes",
           "ohm_last_error", "ohm_fill_ghosts", "ohm_apply", "ohm_residual", "ohm_smooth", "ohm_restrict",
           "ohm_prolong", "ohm_reflux", "ohm_cn_default_opts", "ohm_cn_workspace_size", "ohm_cn_step",
           "ohm_explicit_workspace_size", "ohm_explicit_step", "ohm_residual_noalloc"]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int32), ("base_blocks", ctypes.c_int32 * 3), ("dx0", ctypes.c_double),
                ("nblocks", ctypes.c_int32 * MAX_LEVELS),
                ("block_ijk", ctypes.POINTER(ctypes.c_int32) * MAX_LEVELS)]


class CnOpts(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("rtol", ctypes.c_double), ("max_iters", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32), ("n_vcycles", ctypes.c_int32),
                ("cycle", ctypes.c_int32), ("outer", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("coarse_sweeps", ctypes.c_int32), ("nu_coarse", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("ordering", ctypes.c_int32), ("amr_fmg", ctypes.c_int32),
                ("amr_vcycles", ctypes.c_int32), ("amr_mlat", ctypes.c_int32), ("nu_amr", ctypes.c_int32)]


class CnStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("mg_apps", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("max_res", ctypes.c_double * 3)]


class OhmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libohm.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        # torch carries its own HIP runtime with the same soname as the system
        # one; load it first so that libohm.so binds to that single runtime
        # (two runtimes in one process cannot share devices, memory or streams)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1009_0798_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        DP = ctypes.POINTER(ctypes.c_double)
        sig = {
            "ohm_hier_create": [ctypes.POINTER(ProblemDesc), I32, P, ctypes.POINTER(P)],
            "ohm_hier_destroy": [P],
            "ohm_hier_level_info": [P, I32, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)],
            "ohm_hier_problem_info": [P, I32, I32, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I32)],
            "ohm_hier_device_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
            "ohm_fill_ghosts": [P, I32, P, P, I32, I32, P],
            "ohm_apply": [P, I32, P, P, P, P, DP, P, I32, P],
            "ohm_residual": [P, I32, P, P, P, P, P, DP, P, DP, I32, P],
            "ohm_residual_noalloc": [P, I32, P, P, P, P, P, DP, P, P, I32, P],
            "ohm_smooth": [P, I32, P, P, P, P, P, DP, I32, I32, P, I32, P],
            "ohm_restrict": [P, I32, P, P, I32, I32, P],
            "ohm_prolong": [P, I32, P, P, I32, I32, I32, P],
            "ohm_reflux": [P, I32, P, P, P, P, P, P, DP, P, I32, I32, P],
            "ohm_cn_default_opts": [ctypes.POINTER(CnOpts)],
            "ohm_cn_workspace_size": [P, ctypes.POINTER(CnOpts), ctypes.POINTER(ctypes.c_size_t)],
            "ohm_cn_step": [P, ctypes.POINTER(P), ctypes.POINTER(P), DP, ctypes.POINTER(CnOpts), P,
                            ctypes.c_size_t, ctypes.POINTER(CnStats), P],
            "ohm_explicit_workspace_size": [P, ctypes.POINTER(ctypes.c_size_t)],
            "ohm_explicit_step": [P, ctypes.POINTER(P), ctypes.POINTER(P), DP, I32, P, ctypes.c_size_t, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int if name != "ohm_cn_default_opts" else None
        L.ohm_last_error.argtypes = []
        L.ohm_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(status: int) -> int:
    if status != OHM_OK:
        raise OhmError(status, lib().ohm_last_error().decode())
    return status


def dptr(t) -> ctypes.c_void_p:
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(t.data_ptr())


def stream_ptr(stream=None) -> ctypes.c_void_p:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def host_doubles(vals) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(vals, dtype=np.float64).ravel())
    return (ctypes.c_double * len(a))(*a)
