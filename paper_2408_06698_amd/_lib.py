"""ctypes binding of libhopu.so (argument marshalling only).

Every computation runs in the library's HIP kernels; PyTorch provides device
memory and the stream.  Importing this module does not touch the GPU; loading
the library fails loudly if it has not been built.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhopu.so")

HOPU_OK, HOPU_EINVAL, HOPU_EMESH, HOPU_ENOMEM, HOPU_EHIP, HOPU_ENOCONV, HOPU_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_MFMA, BF16X2, BF16X3 = 0, 1, 2, 3
TERM_VOLUME, TERM_CENTRAL, TERM_UPWIND, TERM_ALL = 1, 2, 4, 7
HOPU_STOKES_CONVECTION, HOPU_STOKES_GUESS = 1, 2
HOPU_STOKES_FP32_PRECOND = 1

STATUS_NAMES = {0: "HOPU_OK", -1: "HOPU_EINVAL", -2: "HOPU_EMESH", -3: "HOPU_ENOMEM",
                -4: "HOPU_EHIP", -5: "HOPU_ENOCONV", -6: "HOPU_EUNSUPPORTED"}

# name -> (restype, argtypes)
_p, _i, _d, _i64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
SIGNATURES = {
    "hopu_create": (_i, [C.POINTER(C.c_void_p), _i, _i, _i64, _p, _p, _p]),
    "hopu_sizes": (_i, [_p, _p, _p, _p, _p, _p, _p]),
    "hopu_set_upwind": (_i, [_p, _i, _p]),
    "hopu_set_solver": (_i, [_p, _d, _i, _i]),
    "hopu_jump_indicator": (_i, [_p, _p, _p]),
    "hopu_set_adaptive": (_i, [_p, _i, _i, _p, _i]),
    "hopu_adapt_upwind": (_i, [_p, _p]),
    "hopu_get_facet_orders": (_i, [_p, _p]),
    "hopu_convection_apply": (_i, [_p, _p, _p, _i, _i]),
    "hopu_mass_apply": (_i, [_p, _p, _p]),
    "hopu_mass_solve": (_i, [_p, _p, _p, _d, _i, _p]),
    "hopu_project": (_i, [_p, _p, _p, _d, _i, _p]),
    "hopu_mfma_f64_rate": (_i, [_i, _p]),
    "hopu_substeps": (_i, [_p, _p, _d, _i, _i, _p]),
    "hopu_set_warm_start": (_i, [_p, _i]),
    "hopu_convection_vjp": (_i, [_p, _p, _p, _p, _i]),
    "hopu_substeps_vjp_workspace": (_i64, [_p, _i, _i]),
    "hopu_substeps_vjp": (_i, [_p, _p, _d, _i, _i, _p, _p, _i, _p, _i64]),
    "hopu_diagnostics": (_i, [_p, _p, _p, _p, _p]),
    "hopu_energy": (_i, [_p, _p, _p]),
    "hopu_count_nonfinite": (_i, [_p, _p, _p]),
    "hopu_interp_points": (_i, [_p, _i, _p, _p]),
    "hopu_interpolate": (_i, [_p, _i, _p, _p, _p]),
    "hopu_eval": (_i, [_p, _p, _i, _p, _p]),
    "hopu_eval_noalloc": (_i, [_p, _p, _i, _p, _p]),
    "hopu_profile_enable": (_i, [_p, _i, _i]),
    "hopu_profile_read": (_i, [_p, _i, _p, _p]),
    "hopu_last_error": (C.c_char_p, [_p]),
    "hopu_destroy": (None, [_p]),
    "hopu_host_tables": (_i64, [_i, _i, _i, _p, _i64]),
    "hopu_host_mesh": (_i64, [_i, _i64, _p, _p, _i, _p, _i64]),
    "hopu_host_sizes": (_i64, [_i, _i, _i]),
    "hopu_stokes_sizes": (_i, [_p, _p, _p, _p]),
    "hopu_stokes_setup": (_i, [_p, _d, _d, _i]),
    "hopu_stokes_apply": (_i, [_p, _p, _p]),
    "hopu_stokes_precond": (_i, [_p, _p, _p]),
    "hopu_stokes_step": (_i, [_p, _p, _i, _p, _d, _i, _p]),
}

_lib = None


class HopuError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2408_06698_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, ctx=None):
    if status != HOPU_OK:
        msg = lib().hopu_last_error(ctx)
        raise HopuError(status, msg.decode() if msg else "")
