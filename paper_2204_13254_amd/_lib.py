"""ctypes declarations of the C ABI in include/ddfem.h (argument marshalling
only; every step of the solve runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddfem.so")

DD_OK = 0
DD_ERR = {
    -1: "DD_ERR_ARG", -2: "DD_ERR_MESH", -3: "DD_ERR_PARTITION", -4: "DD_ERR_NOT_SPD",
    -5: "DD_ERR_NO_CONVERGENCE", -6: "DD_ERR_STATE", -7: "DD_ERR_HIP", -8: "DD_ERR_OOM",
    -9: "DD_ERR_NONFINITE",
}
DD_FP64, DD_FP32_REFINE = 0, 1


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("nrhs", C.c_int), ("cg_tol", C.c_double),
                ("cg_max_iter", C.c_int), ("refine_tol", C.c_double), ("refine_max", C.c_int),
                ("warm_start", C.c_int), ("use_graph", C.c_int), ("check_every", C.c_int),
                ("stream", C.c_void_p), ("precond", C.c_int), ("method", C.c_int),
                ("robin_alpha", C.c_double), ("diagnostics", C.c_int), ("tune_cache", C.c_char_p)]


class Tuning(C.Structure):
    _fields_ = [("chunk", C.c_int), ("coarse_chunk", C.c_int), ("full_chunk", C.c_int),
                ("full_bucket", C.c_int), ("full_persist", C.c_int), ("full_pair", C.c_int),
                ("full_quarter", C.c_int), ("from_cache", C.c_int),
                ("full_ms", C.c_double),
                ("full_ms_default", C.c_double), ("coarse_ms", C.c_double), ("coarse_ms_default", C.c_double),
                ("trailing_ms", C.c_double), ("trailing_ms_default", C.c_double),
                ("sym_persist", C.c_int), ("local_ms", C.c_double), ("local_ms_default", C.c_double),
                ("sym_pw", C.c_int)]


DD_DIAG_GAUSS, DD_DIAG_ENERGY = 1, 2


class Stats(C.Structure):
    _fields_ = [("cg_iters", C.c_int * 32), ("refine_sweeps", C.c_int), ("dd_solves", C.c_int),
                ("cg_relres", C.c_double * 32), ("global_relres", C.c_double * 32),
                ("solve_iters", C.c_int * 4), ("diagnostics", C.c_int),
                ("gauss_residual", C.c_double * 32), ("charge_max", C.c_double * 32),
                ("energy", C.c_double * 32)]


class Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("coords", C.c_void_p), ("n_tets", C.c_int64),
                ("tets", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("n_edges", C.c_int64), ("n_interior", C.c_int64), ("n_tets", C.c_int64),
                ("n_vertices", C.c_int64), ("n_sub", C.c_int32), ("n_lambda", C.c_int32),
                ("n_corner", C.c_int32), ("nrhs", C.c_int32), ("precision", C.c_int32),
                ("tile", C.c_int32), ("factor_bytes", C.c_int64), ("trailing_bytes", C.c_int64),
                ("schur_bytes", C.c_int64), ("corner_bytes", C.c_int64), ("coarse_bytes", C.c_int64),
                ("full_bytes", C.c_int64), ("cross_bytes", C.c_int64)]


class Analysis(C.Structure):
    _fields_ = [("n_edges", C.c_int64), ("n_interior", C.c_int64), ("n_sub", C.c_int32),
                ("n_lambda", C.c_int32), ("n_corner", C.c_int32), ("max_multiplicity", C.c_int32),
                ("sum_nr3", C.c_int64)]


P = C.c_void_p
I64 = C.c_int64
D = C.c_double

SIGNATURES = {
    "dd_default_options": (None, [C.POINTER(Options)]),
    "dd_setup": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Mesh), P, P, P, D, D, C.POINTER(Options)]),
    "dd_get_info": (C.c_int, [P, C.POINTER(Info)]),
    "dd_get_edges": (C.c_int, [P, P, P]),
    "dd_num_edges": (C.c_int, [P, P]),
    "dd_set_eps": (C.c_int, [P, P, C.c_int]),
    "dd_set_charge": (C.c_int, [P, P]),
    "dd_factor": (C.c_int, [P]),
    "dd_autotune": (C.c_int, [P, C.c_char_p, C.POINTER(Tuning)]),
    "dd_step": (C.c_int, [P, P, P, P, P, P, C.POINTER(Stats)]),
    "dd_state_set": (C.c_int, [P, P, P, P]),
    "dd_step_resident": (C.c_int, [P, P, P, C.POINTER(Stats)]),
    "dd_solve": (C.c_int, [P, P, P, C.POINTER(Stats)]),
    "dd_adjoint_step": (C.c_int, [P, P, P, P, P, P, P, P, P, P, P, C.POINTER(Stats)]),
    "dd_charge_update": (C.c_int, [P, P, P]),
    "dd_gauss_residual": (C.c_int, [P, P, P, P]),
    "dd_energy": (C.c_int, [P, P, P, P]),
    "dd_profile": (C.c_int, [P, C.c_int, P, P]),
    "dd_pic_status": (C.c_int, [P, P, C.c_int]),
    "dd_mixed_faces": (C.c_int, [P, P, P]),
    "dd_step_mixed": (C.c_int, [P, P, P, P, P, P, C.POINTER(Stats)]),
    "dd_pic_locate": (C.c_int, [P, I64, P, P]),
    "dd_pic_deposit": (C.c_int, [P, I64, P, P, P, P, P]),
    "dd_pic_faraday": (C.c_int, [P, C.c_int, P, D, P]),
    "dd_pic_sort": (C.c_int, [P, I64, P, P]),
    "dd_pic_sort_noalloc": (C.c_int, [P, I64, P, P]),
    "dd_pic_permute": (C.c_int, [P, I64, P, C.c_int, P, P]),
    "dd_pic_push": (C.c_int, [P, I64, P, P, P, P, P, P, P, P, C.c_int]),
    "dd_destroy": (None, [P]),
    "dd_last_error": (C.c_char_p, []),
    "dd_analyze": (C.c_int, [C.POINTER(Mesh), P, C.POINTER(Analysis), P]),
    "dd_analyze_lambda": (C.c_int, [C.POINTER(Mesh), P, P, P, P, P, P]),
}

_lib = None


def load():
    """Load libddfem.so; raise (never fall back) if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2204_13254_amd/build.py "
                               "(or __graft_entry__.build()) first")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class DDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{DD_ERR.get(code, code)}: {msg}")
        self.code = code


def check(rc):
    if rc != DD_OK:
        raise DDError(rc, load().dd_last_error().decode())
    return rc
