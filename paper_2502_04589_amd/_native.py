"""ctypes declarations of the C ABI in include/pase.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpase.so")

MAX_LEVELS = 8
MAX_NEV = 256

STATUS = {0: "PASE_OK", 1: "PASE_E_ARG", 2: "PASE_E_HIP", 3: "PASE_E_NOMEM", 4: "PASE_E_NOTCONV",
          5: "PASE_E_BREAKDOWN", 6: "PASE_E_UNSUPPORTED"}
PREC = {"fp64": 0, "mixed": 1, "learned": 2}


class Csr(C.Structure):
    _fields_ = [("rows", C.c_int), ("cols", C.c_int), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("val", C.c_void_p)]


class HierarchyCsr(C.Structure):
    _fields_ = [("nlevels", C.c_int), ("A", Csr * MAX_LEVELS), ("M", Csr * MAX_LEVELS), ("P", Csr * MAX_LEVELS),
                ("R", Csr * MAX_LEVELS)]


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("nlevels", C.c_int), ("n", C.c_int * MAX_LEVELS), ("kappa", C.c_void_p),
                ("tensor", C.c_void_p), ("reaction", C.c_void_p), ("csr", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("nev_max", C.c_int), ("cg_steps", C.c_int), ("max_outer", C.c_int),
                ("nu", C.c_int), ("omega", C.c_double), ("small_solver", C.c_int), ("locking", C.c_int),
                ("guard", C.c_int), ("start", C.c_int), ("fallback_ratio", C.c_double),
                ("coarse_level", C.c_int), ("aug_rtol", C.c_double)]


class Report(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("n_converged", C.c_int), ("res_host", C.c_void_p),
                ("res_literal_host", C.c_void_p), ("ritz_history_host", C.c_void_p),
                ("ritz_history_rows", C.c_int), ("t_solve_ms", C.c_double), ("small_fast_iters", C.c_int),
                ("small_path_host", C.c_void_p), ("learned_fallbacks", C.c_int),
                ("lowprec_projection_iters", C.c_int), ("fine_solve_columns", C.c_int),
                ("t_phase_ms", C.c_double * 6), ("aug_iters", C.c_int),
                ("aug_restarts", C.c_int)]

# names of pase_report.t_phase_ms's entries, in order
PHASES = ("start", "residual", "fine_solves", "projection", "small_problem", "prolongation")


# (name, restype, argtypes) for every entry point of include/pase.h
SIGNATURES = [
    ("pase_options_default", None, [C.POINTER(Options)]),
    ("pase_workspace_bytes", C.c_int, [C.POINTER(Problem), C.POINTER(Options), C.POINTER(C.c_size_t)]),
    ("pase_setup", C.c_int, [C.POINTER(Problem), C.POINTER(Options), C.c_void_p, C.c_size_t, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    ("pase_solve", C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.POINTER(Report)]),
    ("pase_solve_batch", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_int,
                                   C.POINTER(Report)]),
    ("pase_solve_batches", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                     C.POINTER(Report)]),
    ("pase_destroy", C.c_int, [C.c_void_p]),
    ("pase_status_string", C.c_char_p, [C.c_int]),
    ("pase_last_error", C.c_char_p, [C.c_void_p]),
    ("pase_level_size", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_longlong)]),
    ("pase_apply", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_vcycle", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    ("pase_pcg", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_restrict", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    ("pase_prolong", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    ("pase_gram", C.c_int, [C.c_void_p, C.c_longlong, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_gram_bf16x3", C.c_int, [C.c_void_p, C.c_longlong, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_gram_noalloc", C.c_int, [C.c_longlong, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_small_eig", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_small_eig_max_n", C.c_int, [C.c_void_p]),
    ("pase_correction", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    ("pase_time_kernel", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    ("pase_export_csr", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                  C.POINTER(C.c_int), C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_unet_param_count", C.c_int, [C.POINTER(C.c_int), C.POINTER(C.c_size_t)]),
    ("pase_unet_workspace_bytes", C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_size_t)]),
    ("pase_unet_create", C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int), C.c_void_p, C.c_size_t, C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    ("pase_unet_destroy", C.c_int, [C.c_void_p]),
    ("pase_unet_last_error", C.c_char_p, [C.c_void_p]),
    ("pase_unet_set_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pase_unet_get_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pase_unet_save", C.c_int, [C.c_void_p, C.c_char_p]),
    ("pase_unet_load", C.c_int, [C.c_void_p, C.c_char_p]),
    ("pase_unet_apply", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_unet_loss_grad", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_double), C.c_void_p]),
    ("pase_unet_adam_step", C.c_int, [C.c_void_p, C.c_float]),
    ("pase_unet_fit_scale", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_double)]),
    ("pase_attach_unet", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pase_harvest", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pase_node_logk", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pase_fine_diag_inverse", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pase_unet_set_output_scale", C.c_int, [C.c_void_p, C.c_void_p]),
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpase.so and declare its signatures.  Raises if the library was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpase.so not found at {path}: run paper_2502_04589_amd.build.build() first")
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
