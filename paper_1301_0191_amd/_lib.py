"""ctypes binding of libambddc.so (argument marshalling only).

Every numeric step runs in the HIP library; this module only converts
Python/numpy/torch arguments into the C ABI declared in include/ambddc.h.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libambddc.so")

STATUS = {0: "OK", 1: "E_INVALID_ARG", 2: "E_NOT_SPD", 3: "E_ASSUMPTION",
          4: "E_NO_CONVERGENCE", 5: "E_OOM", 6: "E_DEVICE", 7: "E_STATE"}


class AmbddcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("dof_per_node", C.c_int32),
                ("coords", C.POINTER(C.c_double)), ("elem_nodes", C.POINTER(C.c_int32)),
                ("dirichlet", C.POINTER(C.c_uint8))]


class Decomp(C.Structure):
    _fields_ = [("levels", C.c_int32), ("elem_to_sub", C.POINTER(C.c_int32)),
                ("parents", C.POINTER(C.POINTER(C.c_int32)))]


class Options(C.Structure):
    _fields_ = [("tau", C.c_double), ("nev_max", C.c_int32), ("lobpcg_maxit", C.c_int32),
                ("lobpcg_block", C.c_int32), ("lobpcg_tol", C.c_double),
                ("precision", C.c_int32), ("initial_constraints", C.c_int32),
                ("keep_edges", C.c_int32), ("fixed_per_face", C.c_int32),
                ("seed", C.c_uint64), ("stream", C.c_void_p)]


# initial constraint sets (AMBDDC_INIT_*)
INITIAL = {"c+e": 0, "c+e+f": 1, "c": 2}


class Stats(C.Structure):
    _fields_ = [("levels", C.c_int32), ("n_free", C.c_int32), ("n_sub", C.c_int32 * 8),
                ("n_pairs", C.c_int32 * 8), ("n_coarse", C.c_int32 * 8),
                ("n_adaptive", C.c_int32 * 8), ("lobpcg_iters", C.c_int32 * 8),
                ("lobpcg_iters_fp32", C.c_int32 * 8),
                ("n_unconverged", C.c_int32 * 8), ("omega_tilde", C.c_double * 8),
                ("t_phase", C.c_double * 16), ("pcg_replacements", C.c_int32),
                ("pcg_stalled", C.c_int32)]


class Analysis(C.Structure):
    _fields_ = [("n_free", C.c_int32), ("n_sub", C.c_int32), ("n_interface", C.c_int32),
                ("n_faces", C.c_int32), ("n_edges", C.c_int32), ("n_corners", C.c_int32),
                ("n_coarse_initial", C.c_int32), ("n_pairs", C.c_int32)]


_lib = None

_SIGS = {
    "ambddc_default_options": (None, [C.POINTER(Options)]),
    "ambddc_analyze": (C.c_int, [C.POINTER(Mesh), C.POINTER(Decomp), C.c_int32,
                                 C.POINTER(Analysis), C.c_void_p, C.c_int32]),
    "ambddc_create": (C.c_int, [C.POINTER(Mesh), C.POINTER(Decomp), C.POINTER(Options),
                                C.POINTER(C.c_void_p)]),
    "ambddc_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ambddc_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int32,
                               C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "ambddc_solve_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                       C.c_int32, C.c_void_p, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double)]),
    "ambddc_element_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                          C.c_void_p]),
    "ambddc_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "ambddc_level_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
    "ambddc_sub_dofs": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ambddc_get_schur": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "ambddc_pair_info": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ambddc_get_pair_result": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                         C.POINTER(C.c_int32), C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ambddc_get_face_constraints": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                              C.c_void_p]),
    "ambddc_get_coarse_element": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                            C.POINTER(C.c_int32)]),
    "ambddc_get_top_coarse": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "ambddc_last_residual": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "ambddc_setup_log10": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ambddc_misfit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                C.POINTER(C.c_double)]),
    "ambddc_timing_enable": (C.c_int, [C.c_void_p, C.c_char_p]),
    "ambddc_set_graphs": (C.c_int, [C.c_void_p, C.c_int32]),
    "ambddc_timing_read": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
    "ambddc_last_error": (C.c_char_p, []),
    "ambddc_destroy": (None, [C.c_void_p]),
}

EXPORTED = tuple(_SIGS.keys())


def load(path: str = LIB_PATH):
    """Load libambddc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built: run __graft_entry__.build() or "
                           "python -m paper_1301_0191_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != 0:
        msg = load().ambddc_last_error()
        raise AmbddcError(code, msg.decode() if msg else "")
