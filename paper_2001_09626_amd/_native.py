"""ctypes declarations of the C ABI in include/afieti.h (argument marshalling
only; every step of the method runs in the native library)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("AFIETI_LIBRARY") or os.path.join(HERE, "libafieti.so")

OK = 0
NOT_CONVERGED = 1
EBREAKDOWN = -4
ERRORS = {-1: "EINVAL", -2: "EGEOM", -3: "ESINGULAR", -4: "EBREAKDOWN",
          -5: "ENOMEM", -6: "EHIP", -7: "EUNSUPPORTED"}

FD_PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "fp32_valu": 3, "fp64_valu": 4}
PS_VARIANT = {"nr": 0, "plain": 1}
PRECOND = {"fd": 0, "geo": 1}
STIFFNESS = {"auto": 0, "assembled": 1, "matrix_free": 2}

OPS = {"stiffness": 0, "B": 1, "Bt": 2, "P_u": 3, "P_chi": 4, "Shat": 5, "P_S": 6,
       "prec": 7, "saddle": 8, "fd_interior": 9, "Ahat": 10, "mass": 11, "load": 12,
       "dirichlet_lift": 13}

EXPORT = {"B": 0, "eig": 1, "H": 2, "GtG": 3, "fixed_load": 4, "dirichlet_c": 5, "eigvec": 6,
          "geo_scale": 7, "geo_eig": 8, "glue": 9}


class Patch(C.Structure):
    _fields_ = [("p", C.c_int), ("reg", C.c_int), ("n_el", C.c_int * 3),
                ("corners", C.c_double * 24), ("lam", C.c_double), ("mu", C.c_double),
                ("face_bc", C.c_int * 6), ("knots", C.POINTER(C.c_double) * 3), ("n_knots", C.c_int * 3),
                ("ctrl", C.POINTER(C.c_double))]


class LoadMode(C.Structure):
    _fields_ = [("comp", C.c_int), ("amp", C.c_double), ("k", C.c_int * 3),
                ("phase", C.c_double * 3)]


FIELD_FN = C.CFUNCTYPE(None, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)
TRACTION_FN = C.CFUNCTYPE(None, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                          C.POINTER(C.c_double), C.c_void_p)


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_patches", C.c_int), ("patches", C.POINTER(Patch)),
                ("n_load_modes", C.c_int), ("load_modes", C.POINTER(LoadMode)),
                ("body_force", FIELD_FN), ("traction", TRACTION_FN), ("dirichlet", FIELD_FN),
                ("ctx", C.c_void_p), ("n_interfaces", C.c_int), ("interfaces", C.POINTER(C.c_int))]


class Options(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("fd_precision", C.c_int),
                ("ps_variant", C.c_int), ("check_every", C.c_int), ("host_only", C.c_int),
                ("use_graph", C.c_int), ("stiffness", C.c_int), ("fd_tune", C.c_int),
                ("ps_weight", C.c_double), ("precond", C.c_int),
                ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p), ("alloc_ctx", C.c_void_p)]


DEV_ALLOC_FN = C.CFUNCTYPE(C.c_uint64, C.c_size_t, C.c_void_p)  # returns the device address
DEV_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class Info(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_c", C.c_int64), ("n_problems", C.c_int),
                ("n_patches_total", C.c_int), ("stiffness_bytes", C.c_int64),
                ("device_bytes", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int),
                ("rel_residual", C.c_double), ("ms_solve", C.c_double)]


SYMBOLS = {
    "afieti_default_options": (None, [C.POINTER(Options)]),
    "afieti_setup": (C.c_int, [C.POINTER(Problem), C.c_int, C.POINTER(Options), C.c_void_p,
                               C.POINTER(C.c_void_p)]),
    "afieti_get_info": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "afieti_get_problem_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double),
                                           C.POINTER(C.c_int)]),
    "afieti_get_offsets": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "afieti_apply_fd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "afieti_apply_fd_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "afieti_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(Stats), C.c_void_p]),
    "afieti_solve_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.c_int, C.c_void_p, C.POINTER(C.c_double),
                                       C.POINTER(Stats), C.c_void_p]),
    "afieti_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "afieti_set_parameters": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.c_void_p]),
    "afieti_export": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "afieti_export_size": (C.c_int64, [C.c_void_p, C.c_int]),
    "afieti_destroy": (None, [C.c_void_p]),
    "afieti_strerror": (C.c_char_p, [C.c_int]),
    "afieti_last_error": (C.c_char_p, [C.c_void_p]),
}

_lib = None


def lib():
    """Load the in-tree native library; fail loudly if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"native library missing: {LIB_PATH} (run python -m paper_2001_09626_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
