"""ctypes binding of libftdmrg.so (include/ftdmrg.h).

Argument marshalling only: every step of the computation runs in the native
library.  PyTorch supplies the HIP stream (the current torch stream) and,
optionally, device memory through its caching allocator.  If the shared
library is missing this module raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libftdmrg.so")

FTD_OK, FTD_EINVAL, FTD_ENOMEM, FTD_EDEVICE, FTD_ENOCONV, FTD_ESTATE = range(6)
PRECISION = {"c128": 0, "c64": 1, "bf16x3": 2}


class FtdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ftdmrg error {code}: {msg}")
        self.code = code


class Model(C.Structure):
    _fields_ = [("n_mol", C.c_int32), ("n_loc", C.c_int32), ("n_nl", C.c_int32),
                ("periodic", C.c_int32), ("levels_loc", C.c_int32), ("levels_nl", C.c_int32),
                ("omega_loc", C.POINTER(C.c_double)), ("g_loc", C.POINTER(C.c_double)),
                ("omega_nl", C.POINTER(C.c_double)), ("g_nl", C.POINTER(C.c_double)),
                ("V", C.c_double), ("R", C.c_double), ("e0", C.c_double)]


class KrylovOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("mmax", C.c_int32)]


class SweepPoint(C.Structure):
    _fields_ = [("beta", C.c_double), ("V", C.c_double), ("omega_scale", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("heff_launches", C.c_int64), ("heff_ms", C.c_double),
                ("heff_flops", C.c_double), ("dom_launches", C.c_int64),
                ("dom_ms", C.c_double), ("dom_flops", C.c_double), ("dom_bytes", C.c_double),
                ("matvecs", C.c_int64), ("krylov_vectors", C.c_int64),
                ("expm_calls", C.c_int64), ("krylov_max", C.c_int64),
                ("dom_kind", C.c_int32), ("all_flops", C.c_double),
                ("kind_launches", C.c_int64 * 32), ("kind_ms", C.c_double * 32),
                ("kind_flops", C.c_double * 32), ("kind_bytes", C.c_double * 32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
D = C.c_double
DP = C.POINTER(C.c_double)
I32 = C.c_int32
I32P = C.POINTER(C.c_int32)

SIGNATURES = {
    "ftd_last_error": (C.c_char_p, []),
    "ftd_ctx_create": (I32, [I32, P, C.POINTER(Allocator), PP]),
    "ftd_ctx_destroy": (None, [P]),
    "ftd_ctx_set_verbose": (I32, [P, I32]),
    "ftd_ctx_set_timing": (I32, [P, I32]),
    "ftd_ctx_stats": (I32, [P, C.POINTER(Stats)]),
    "ftd_ctx_stats_reset": (I32, [P]),
    "ftd_ctx_synchronize": (I32, [P]),
    "ftd_mpo_build": (I32, [P, C.POINTER(Model), PP, PP]),
    "ftd_mpo_destroy": (None, [P]),
    "ftd_mpo_info": (I32, [P, I32P, I32P, I32P]),
    "ftd_mps_destroy": (None, [P]),
    "ftd_mps_copy": (I32, [P, P, PP]),
    "ftd_mps_info": (I32, [P, I32P, I32P, DP, I32P]),
    "ftd_mps_get_site": (I32, [P, P, I32, DP, C.c_int64]),
    "ftd_mps_from_host": (I32, [P, I32, I32P, DP, D, I32, PP]),
    "ftd_mps_norm": (I32, [P, P, DP]),
    "ftd_mps_set_precision": (I32, [P, I32]),
    "ftd_mps_set_site": (I32, [P, P, I32, DP, C.c_int64]),
    "ftd_mps_save": (I32, [P, P, C.c_char_p]),
    "ftd_mps_load": (I32, [P, C.c_char_p, PP]),
    "ftd_thermal_prep": (I32, [P, P, D, I32, I32, I32, D, D, I32, C.POINTER(KrylovOpts), PP,
                               DP]),
    "ftd_tdvp_step_expand": (I32, [P, P, P, D, D, I32, D, C.POINTER(KrylovOpts)]),
    "ftd_tdvp_pair": (I32, [P, P, P, P, D, D, C.POINTER(KrylovOpts)]),
    "ftd_tdvp_step": (I32, [P, P, P, D, D, C.POINTER(KrylovOpts)]),
    "ftd_apply_compress": (I32, [P, P, P, I32, D, PP]),
    "ftd_overlap": (I32, [P, P, P, P, DP]),
    "ftd_pc_stage": (I32, [P, P, P, P, DP, I32, D, PP]),
    "ftd_corr_current": (I32, [P, P, P, P, I32, D, D, I32, C.POINTER(KrylovOpts), DP]),
    "ftd_mobility": (I32, [DP, I32, D, D, D, DP, DP]),
    "ftd_mean_free_path": (I32, [DP, I32, D, D, DP, DP, DP]),
    "ftd_fgr_corr": (I32, [DP, I32, DP, DP, I32, D, D, D, D, DP]),
    "ftd_mobility_sweep": (I32, [P, P, P, I32, I32, I32, I32, D, D, I32, I32, P, DP, DP]),
    "ftd_mobility_grad": (I32, [P, P, D, I32, I32, I32, D, D, I32, I32, P, D, DP, DP, DP, DP,
                                DP]),
    "ftd_reduced_density": (I32, [P, P, P, DP]),
    "ftd_coherent_length": (I32, [DP, I32, DP]),
    "ftd_heff_apply": (I32, [P, P, P, I32, DP, DP, I32]),
    "ftd_heff_expm": (I32, [P, P, P, I32, DP, DP, D, D, C.POINTER(KrylovOpts), I32, I32P]),
    "ftd_svd_trunc": (I32, [P, I32, I32, DP, I32, D, I32, DP, DP, I32P]),
    "ftd_qr": (I32, [P, I32, I32, DP, I32, DP, DP]),
    "ftd_gemm": (I32, [P, I32, I32, I32, I32, I32, I32, DP, DP, DP]),
    "ftd_gemm_noalloc": (I32, [P, I32, I32, I32, I32, I32, I32, P, P, P]),
}


def _load():
    # torch ships its own HIP runtime under the same soname as the system one;
    # loading torch first makes this library bind to that single runtime, so
    # torch streams and allocations are valid handles here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2003_13245_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(code):
    if code != FTD_OK:
        raise FtdError(code, lib.ftd_last_error().decode())


def exported_symbols():
    return sorted(SIGNATURES)


def _dptr(a):
    return a.ctypes.data_as(DP)


def _krylov(tol, mmax):
    return KrylovOpts(float(tol), int(mmax))
