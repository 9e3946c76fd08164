"""ctypes mirror of include/waveholtz.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwaveholtz.so")

WH_OK, WH_ENOCONV = 0, 1
WH_EINVAL, WH_EUNSUPPORTED, WH_EHIP, WH_EWORKSPACE, WH_EUNSTABLE, WH_EBREAKDOWN, WH_EHOST = -1, -2, -3, -4, -5, -6, -7
WH_F64, WH_MIXED = 0, 1
WH_FPI, WH_CG, WH_DCG, WH_GMRES, WH_BICGSTAB = 0, 1, 2, 3, 4
WH_DEFL_NONE, WH_DEFL_SINE, WH_DEFL_DENSE_EXACT, WH_DEFL_DENSE, WH_DEFL_FACTORED = 0, 1, 2, 3, 4


class WhGrid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32), ("order", C.c_int32)]


class WhParams(C.Structure):
    _fields_ = [
        ("omega", C.c_double), ("n_periods", C.c_int32), ("cfl", C.c_double),
        ("steps_per_period", C.c_int32), ("freq_correction", C.c_int32), ("c_max", C.c_double),
        ("precision", C.c_int32), ("solver", C.c_int32), ("restart", C.c_int32),
        ("tol", C.c_double), ("max_iters", C.c_int32), ("inner_tol", C.c_double),
        ("max_outer", C.c_int32), ("k_fuse", C.c_int32), ("reproject", C.c_int32),
        ("check_every", C.c_int32), ("mixed_form", C.c_int32), ("devd", C.c_int32), ("k_shape", C.c_int32),
    ]


class WhDeflation(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n_d", C.c_int32), ("modes", C.POINTER(C.c_int32)),
        ("V", C.c_void_p), ("ldv", C.c_int64), ("lambda2", C.POINTER(C.c_double)),
        ("n_terms", C.c_int32), ("term_mode", C.POINTER(C.c_int32)), ("fx", C.c_void_p), ("fy", C.c_void_p),
    ]


class WhInfo(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("iters", C.c_int32), ("wave_solves", C.c_int32),
        ("wave_solves_f32", C.c_int32), ("outer", C.c_int32), ("nt", C.c_int32), ("m", C.c_int32),
        ("k_fuse", C.c_int32), ("rel_res", C.c_double), ("true_rel_res", C.c_double),
        ("omega_tilde", C.c_double), ("dt", C.c_double), ("c_max", C.c_double), ("ms", C.c_double),
        ("k_rows", C.c_int32), ("k_waves", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class WhProblem(C.Structure):
    _fields_ = [("grid", WhGrid), ("c2", C.c_void_p), ("f", C.c_void_p), ("omega", C.c_double),
                ("u", C.c_void_p), ("n_defl", C.c_int32)]


P = C.POINTER
_SIGS = {
    "wh_params_default": (None, [P(WhParams)]),
    "wh_create": (C.c_int, [P(C.c_void_p), C.c_int, C.c_void_p]),
    "wh_destroy": (C.c_int, [C.c_void_p]),
    "wh_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "wh_last_error": (C.c_char_p, [C.c_void_p]),
    "wh_coeff_bound": (C.c_int, [C.c_void_p, P(WhGrid), C.c_void_p, P(C.c_double)]),
    "wh_status_string": (C.c_char_p, [C.c_int]),
    "wh_time_params": (C.c_int, [P(WhGrid), P(WhParams), C.c_double, P(C.c_int32), P(C.c_int32),
                                 P(C.c_double), P(C.c_double)]),
    "wh_transfer": (C.c_int, [P(WhGrid), P(WhParams), C.c_double, C.c_int32, P(C.c_double),
                              P(C.c_double)]),
    "wh_select_sine_modes": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int32, P(C.c_int32),
                                       P(C.c_double)]),
    "wh_workspace_bytes": (C.c_size_t, [P(WhGrid), P(WhParams), P(WhDeflation)]),
    "wh_apply_filter": (C.c_int, [C.c_void_p, P(WhGrid), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, P(WhParams), C.c_void_p, C.c_size_t, P(WhInfo)]),
    "wh_solve": (C.c_int, [C.c_void_p, P(WhGrid), C.c_void_p, C.c_void_p, P(WhDeflation),
                           P(WhParams), C.c_void_p, C.c_void_p, C.c_size_t, P(WhInfo)]),
    "wh_helmholtz_residual": (C.c_int, [C.c_void_p, P(WhGrid), C.c_void_p, C.c_void_p, C.c_double,
                                        C.c_void_p, C.c_void_p, C.c_size_t, P(C.c_double)]),
}

# entry points added as they are built (declared in include/waveholtz.h)
_OPTIONAL = {
    "wh_workspace_bytes_adjoint": (C.c_size_t, [P(WhGrid), P(WhParams), C.c_int32]),
    "wh_solve_vjp": (C.c_int, [C.c_void_p, P(WhGrid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               P(WhParams), C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, P(WhInfo)]),
    "wh_adjoint_grad": (C.c_int, [C.c_void_p, P(WhGrid), C.c_void_p, C.c_int32, P(C.c_void_p), C.c_int32,
                                  C.c_void_p, C.c_void_p, P(WhParams), C.c_int32, C.c_void_p,
                                  P(C.c_double), C.c_void_p, C.c_size_t, P(WhInfo)]),
    "wh_workspace_bytes_batched": (C.c_size_t, [C.c_int32, P(WhProblem), P(WhParams)]),
    "wh_solve_batched": (C.c_int, [C.c_void_p, C.c_int32, P(WhProblem), P(WhParams), C.c_void_p, C.c_size_t,
                                   P(WhInfo)]),
    "wh_time_batch_kernel": (C.c_int, [C.c_void_p, C.c_int32, P(WhProblem), P(WhParams), C.c_int32, C.c_void_p,
                                       C.c_size_t, P(C.c_double), P(C.c_int64)]),
    "wh_apply_filter_noalloc": (C.c_int, [C.c_void_p, P(WhGrid), C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, P(WhParams), P(WhInfo)]),
    "wh_time_step_kernel": (C.c_int, [C.c_void_p, P(WhGrid), C.c_void_p, P(WhParams), C.c_int32, C.c_void_p,
                                      C.c_size_t, P(C.c_double), P(C.c_int32), P(C.c_int32),
                                      P(C.c_int32)]),
}

_lib = None


def load():
    """Load the in-tree libwaveholtz.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libwaveholtz.so not built ({LIB_PATH}); run __graft_entry__.build()")
    # torch first: its HIP runtime (libamdhip64.so.7 and the HSA runtime it names) must be
    # the one in the process.  Loading the library first would bring in the system copies,
    # after which torch's own HSA runtime is mapped a second time and the library's HIP
    # calls see no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in {**_SIGS, **_OPTIONAL}.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return sorted(list(_SIGS) + list(_OPTIONAL))
