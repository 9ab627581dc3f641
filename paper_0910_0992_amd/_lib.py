"""ctypes declarations of the C ABI in include/tprec.h.

Loads the in-tree libtprec.so; raises if it has not been built.  No compute
happens here: every function is a direct call into the HIP library.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtprec.so")

# status codes
TP_OK, TP_EINVAL, TP_EDIMS, TP_ESINGULAR, TP_ENOCONV, TP_EBREAKDOWN, TP_ENOMEM, TP_EHIP = (
    0, -1, -2, -3, -4, -5, -6, -7)
TP_HOST, TP_DEVICE = 0, 1
SCHEMES = {"UNPREC": 0, "SCHUR4D": 1, "TEMPORAL": 2, "TEMPORAL_SCHUR": 3, "TEMPORAL_SCHUR3D": 4,
           "TEMPORAL_FULLSW": 5}
SOLVERS = {"CGNR": 0, "BICGSTAB": 1}
PRECS = {"F64": 0, "F32": 1, "F16N": 2}
LAYOUTS = {"CANONICAL": 0, "P3": 1, "P4": 2}
SUBSETS = {"FULL": 0, "EVEN": 1, "ODD": 2}


class TpField(C.Structure):
    _fields_ = [("data", C.c_void_p), ("layout", C.c_int32), ("prec", C.c_int32),
                ("subset", C.c_int32), ("nrhs", C.c_int32)]


class SolveParams(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("solver", C.c_int32), ("prec", C.c_int32),
                ("max_iter", C.c_int32), ("max_restarts", C.c_int32), ("use_x0", C.c_int32),
                ("estimate_kappa", C.c_int32), ("dagger", C.c_int32),
                ("tol", C.c_double), ("inner_tol", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("applies", C.c_int32),
                ("restarts", C.c_int32), ("true_rel_resid", C.c_double),
                ("prec_rel_resid", C.c_double), ("kappa_est", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TprecError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_P = C.c_void_p
_I = C.c_int32
_D = C.c_double

# tp_alloc_fn and tp_free_fn
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)

# (name, argtypes, restype)
SIGNATURES = [
    ("tp_ctx_create", [C.POINTER(C.c_int32), _I, _I, C.POINTER(_P)], _I),
    ("tp_ctx_destroy", [_P], _I),
    ("tp_ctx_set_stream", [_P, _P], _I),
    ("tp_ctx_set_allocator", [_P, ALLOC_FN, FREE_FN, _P], _I),
    ("tp_ctx_device_bytes", [_P, C.POINTER(C.c_size_t)], _I),
    ("tp_gauge_create", [_P, _P, _I, C.POINTER(_P)], _I),
    ("tp_gauge_destroy", [_P], _I),
    ("tp_gauge_plaquette", [_P, C.POINTER(_D), C.POINTER(_D)], _I),
    ("tp_clover_create", [_P, _D, _D, C.POINTER(_P)], _I),
    ("tp_clover_destroy", [_P], _I),
    ("tp_op_create", [_P, _P, _D, _D, C.POINTER(_P)], _I),
    ("tp_op_destroy", [_P], _I),
    ("tp_op_mass", [_P, C.POINTER(_D)], _I),
    ("tp_op_set_cutoff", [_P, _D, C.POINTER(C.c_int32)], _I),
    ("tp_apply_M", [_P, _I, _P, _P, _I], _I),
    ("tp_apply_Ds", [_P, _I, _P, _P], _I),
    ("tp_apply_clover", [_P, _I, _P, _P, _I], _I),
    ("tp_apply_Tinv", [_P, _I, _P, _P, _I], _I),
    ("tp_apply_CL", [_P, _I, _P, _P], _I),
    ("tp_apply_CR", [_P, _I, _P, _P], _I),
    ("tp_apply_prec", [_P, _I, _I, _P, _P, _I], _I),
    ("tp_apply_prec_noalloc", [_P, _I, _I, _P, _P, _I], _I),
    ("tp_prepare_source", [_P, _I, _I, _P, _P], _I),
    ("tp_reconstruct", [_P, _I, _I, _P, _P], _I),
    ("tp_field_bytes", [_P, _I, _I, _I, C.POINTER(C.c_size_t)], _I),
    ("tp_field_convert", [_P, C.POINTER(TpField), C.POINTER(TpField)], _I),
    ("tp_apply_prec_field", [_P, _I, C.POINTER(TpField), C.POINTER(TpField), _I], _I),
    ("tp_prepare_source_field", [_P, _I, C.POINTER(TpField), C.POINTER(TpField)], _I),
    ("tp_reconstruct_field", [_P, _I, C.POINTER(TpField), C.POINTER(TpField)], _I),
    ("tp_solve", [_P, C.POINTER(SolveParams), _P, _P, C.POINTER(SolveInfo)], _I),
    ("tp_solve_multi", [_P, C.POINTER(SolveParams), _I, C.POINTER(_P), C.POINTER(_P), C.POINTER(SolveInfo)], _I),
    ("tp_force", [_P, _P, _P, _P, _I], _I),
    ("tp_status_string", [_I], C.c_char_p),
    ("tp_last_error", [], C.c_char_p),
    ("tp_prof_enable", [_P, _I], _I),
    ("tp_prof_select", [_P, C.c_uint32], _I),
    ("tp_prof_reset", [_P], _I),
    ("tp_prof_count", [], _I),
    ("tp_prof_name", [_I], C.c_char_p),
    ("tp_prof_get", [_P, _I, C.POINTER(C.c_int64), C.POINTER(_D), C.POINTER(_D)], _I),
]

_lib = None


def load():
    """The loaded library (ctypes.CDLL) with argument types declared."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libtprec.so is not built: run `python -m paper_0910_0992_amd.build` "
                "(or __graft_entry__.build()) first")
        lib = C.CDLL(LIB_PATH)
        for name, args, res in SIGNATURES:
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(status):
    if status != TP_OK:
        lib = load()
        msg = lib.tp_last_error().decode() or lib.tp_status_string(status).decode()
        raise TprecError(status, msg)
    return status
