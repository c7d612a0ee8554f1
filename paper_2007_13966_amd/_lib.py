"""ctypes declarations of libnks (include/nks.h).  Argument marshalling only.

The shared library is built in-tree by ``paper_2007_13966_amd.build``; if it
is missing this module raises ImportError: there is no CPU fallback.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libnks.so")

NKS_OK = 0
ERRORS = {-1: "NKS_EINVAL", -2: "NKS_EHIP", -3: "NKS_EZEROPIVOT", -4: "NKS_ENONPHYSICAL",
          -5: "NKS_ENOTCONVERGED", -6: "NKS_ENOMEM"}
NKS_LEFT_RAS, NKS_AS, NKS_RIGHT_RAS = 0, 1, 2
NKS_VCYCLE, NKS_LEFT_KASKADE, NKS_RIGHT_KASKADE, NKS_ADDITIVE, NKS_COARSE_ONLY = 0, 1, 2, 3, 4
NKS_FP64, NKS_FP32, NKS_BF16 = 0, 1, 2

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class nks_fluid(C.Structure):
    _fields_ = [("Tc", C.c_double), ("pc", C.c_double), ("omega", C.c_double), ("T", C.c_double),
                ("W", C.c_double), ("R", C.c_double), ("mu", C.c_double), ("Tb", C.c_double)]


class nks_reservoir_desc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("kx", C.c_void_p), ("ky", C.c_void_p), ("kz", C.c_void_p), ("phi", C.c_void_p),
                ("nwells", C.c_int), ("well_cell", C.POINTER(C.c_int)),
                ("well_rate", C.POINTER(C.c_double)),
                ("bc_type", C.POINTER(C.c_int)), ("bc_value", C.POINTER(C.c_double))]


class nks_grid_desc(C.Structure):
    _fields_ = [("nres", C.c_int), ("res", C.POINTER(nks_reservoir_desc)), ("fluid", nks_fluid),
                ("gravity", C.c_int), ("g", C.c_double), ("stream", C.c_void_p),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p), ("accum", C.c_int)]


ACCUM_FORMS = {"conservative": 0, "chain_rule": 1}
COARSE_KERNELS = {"auto": 0, "chunked": 1, "persistent": 2}


class nks_ras_desc(C.Structure):
    _fields_ = [("px", C.c_int), ("py", C.c_int), ("pz", C.c_int), ("levels", C.c_int),
                ("overlap", C.c_int * 8), ("variant", C.c_int), ("interp_order", C.c_int),
                ("cycle", C.c_int), ("mu", C.c_int), ("nu", C.c_int),
                ("coarse_rtol", C.c_double), ("coarse_maxit", C.c_int),
                ("coarse_restart", C.c_int), ("precision", C.c_int),
                ("tx", C.c_int), ("ty", C.c_int), ("tz", C.c_int), ("fill", C.c_int),
                ("ratio", C.c_int), ("coarse_op", C.c_int), ("coarse_kernel", C.c_int)]


class nks_gmres_desc(C.Structure):
    _fields_ = [("restart", C.c_int), ("rtol", C.c_double), ("atol", C.c_double),
                ("maxit", C.c_int), ("flexible", C.c_int), ("transpose", C.c_int)]


class nks_gmres_stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("total_iterations", C.c_int), ("residual", C.c_double),
                ("converged", C.c_int), ("its", C.POINTER(C.c_int)),
                ("res", C.POINTER(C.c_double))]


class nks_newton_desc(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("eps_a", C.c_double), ("eta_r", C.c_double),
                ("eta_a", C.c_double), ("restart", C.c_int), ("maxit", C.c_int),
                ("flexible", C.c_int), ("alpha", C.c_double), ("max_newton", C.c_int),
                ("max_backtracks", C.c_int), ("stol", C.c_double), ("floor_test", C.c_int),
                ("lag", C.c_int)]


class nks_newton_stats(C.Structure):
    _fields_ = [("newton_its", C.c_int), ("linear_its", C.c_int), ("status", C.c_int),
                ("fnorm0", C.c_double), ("fnorm", C.c_double), ("fnorms", C.c_double * 64),
                ("lits", C.c_int * 64), ("lambdas", C.c_double * 64),
                ("t_residual", C.c_double), ("t_jacobian", C.c_double), ("t_setup", C.c_double),
                ("t_gmres", C.c_double), ("t_linesearch", C.c_double),
                ("stop_reason", C.POINTER(C.c_int)), ("rel_res", C.POINTER(C.c_double)),
                ("host_waits", C.c_int), ("graph_chunk", C.c_int)]


STOP_REASONS = {0: "none", 1: "tolerance", 2: "floor", 3: "step"}


class nks_adjoint_stats(C.Structure):
    _fields_ = [("linear_its", C.c_int * 64), ("total_linear_its", C.c_int), ("status", C.c_int),
                ("t_total", C.c_double)]


class nks_autotune_entry(C.Structure):
    _fields_ = [("tile", C.c_int), ("overlap", C.c_int), ("ok", C.c_int), ("iterations", C.c_int),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("ratio", C.c_int)]


_P = C.c_void_p
_D = C.c_double
_I = C.c_int
_IP = C.POINTER(C.c_int)
_DP = C.POINTER(C.c_double)

PROTOTYPES = {
    "nks_setup_grid": [C.POINTER(nks_grid_desc), C.POINTER(C.c_void_p)],
    "nks_destroy_grid": [_P],
    "nks_grid_info": [_P, _IP, _IP, _IP],
    "nks_hydrostatic_init": [_P, _D, _P],
    "nks_residual": [_P, _P, _P, _P, _D, _I, _P],
    "nks_matrix_create": [_P, C.POINTER(C.c_void_p)],
    "nks_destroy_matrix": [_P],
    "nks_jacobian": [_P, _P, _P, _P, _D, _I, _P, _P],
    "nks_matrix_nnz": [_P, _IP],
    "nks_matrix_export_csr": [_P, _IP, _IP, _DP],
    "nks_matrix_apply": [_P, _P, _P],
    "nks_jacobian_transpose_apply": [_P, _P, _P],
    "nks_residual_dlogk_transpose_apply": [_P, _P, _P, _P],
    "nks_ras_setup": [_P, C.POINTER(nks_ras_desc), C.POINTER(C.c_void_p)],
    "nks_destroy_ras": [_P],
    "nks_ras_apply": [_P, _P, _P],
    "nks_ras_apply_level": [_P, _I, _P, _P],
    "nks_ras_coarse_solve": [_P, _P, _P],
    "nks_ras_coarse_stats": [_P, _IP, _DP],
    "nks_ras_apply_transpose": [_P, _P, _P],
    "nks_ras_level_info": [_P, _I, _IP],
    "nks_ras_level_sweep": [_P, _I, _IP, _IP],
    "nks_ras_level_export": [_P, _I, _IP, _IP, _DP],
    "nks_ras_restrict": [_P, _I, _P, _P],
    "nks_ras_prolong_add": [_P, _I, _P, _P],
    "nks_gmres_solve": [_P, _P, _P, _P, C.POINTER(nks_gmres_desc), C.POINTER(nks_gmres_stats)],
    "nks_newton_step": [_P, _P, _P, _P, _D, _I, C.POINTER(nks_newton_desc),
                        C.POINTER(nks_ras_desc), C.POINTER(nks_newton_stats)],
    "nks_residual_noalloc": [_P, _P, _P, _P, _D, _I, _P],
    "nks_matrix_transpose": [_P, _P],
    "nks_adjoint": [_P, _I, C.POINTER(C.c_void_p), _IP, _D, C.POINTER(C.c_void_p),
                    C.POINTER(nks_ras_desc), C.POINTER(nks_gmres_desc), _P, C.POINTER(C.c_void_p),
                    C.POINTER(nks_adjoint_stats)],
    "nks_ras_autotune": [_P, _P, _P, _P, _D, _I, C.POINTER(nks_ras_desc), _IP, _I, _IP, _I, _IP, _I,
                         C.POINTER(nks_gmres_desc), _I, C.POINTER(nks_ras_desc),
                         C.POINTER(nks_autotune_entry)],
    "nks_profile_enable": [_I],
    "nks_profile_filter": [C.c_char_p],
    "nks_profile_query": [C.c_char_p, _IP, _DP],
    "nks_profile_durations": [C.c_char_p, _DP, _I, _IP],
    "nks_profile_units": [C.c_char_p, _DP],
    "nks_last_error": [],
    "nks_version": [],
}


def load():
    if not os.path.exists(LIBPATH):
        raise ImportError(
            f"libnks.so not found at {LIBPATH}: build it with `python -m paper_2007_13966_amd.build` "
            "(hipcc, gfx950); there is no CPU fallback")
    lib = C.CDLL(LIBPATH)
    for name, args in PROTOTYPES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_char_p if name in ("nks_last_error", "nks_version") else C.c_int
    return lib


class NksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(lib, code):
    if code != NKS_OK:
        raise NksError(code, lib.nks_last_error().decode(errors="replace"))
    return code
