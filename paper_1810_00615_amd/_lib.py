"""ctypes binding of libaao.so (argument marshalling only).

The library is loaded after ``import torch`` so that it binds to the HIP
runtime torch already loaded (same SONAME), i.e. one runtime per process and
device pointers shared with torch tensors."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaao.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int_p = ctypes.POINTER(ctypes.c_int)


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_resid_est", ctypes.c_double), ("rel_resid_true", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> argtypes; every entry point returns an int status unless listed in _RET
SIGNATURES = {
    "aao_create": [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                   ctypes.POINTER(ctypes.c_void_p)],
    "aao_create_2d": [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                      ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)],
    "aao_destroy": [ctypes.c_void_p],
    "aao_set_stream": [ctypes.c_void_p, ctypes.c_void_p],
    "aao_set_kappa": [ctypes.c_void_p, ctypes.c_double],
    "aao_set_steps": [ctypes.c_void_p, ctypes.c_void_p],
    "aao_set_precision": [ctypes.c_void_p, ctypes.c_int],
    "aao_set_neumann_order": [ctypes.c_void_p, ctypes.c_int],
    "aao_project_sine": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_void_p],
    "aao_build_rhs": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "aao_apply_A": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "aao_apply_Pinv": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                       ctypes.c_int],
    "aao_apply_Pinv_noalloc": [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int, ctypes.c_void_p],
    "aao_gmres": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                  ctypes.c_double, ctypes.c_int, ctypes.POINTER(Info)],
    "aao_gmres_ex": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Info)],
    "aao_adjoint_solve": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                          ctypes.c_double, ctypes.c_int, ctypes.POINTER(Info)],
    "aao_grad": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _c_double_p],
    "aao_grad_checkpointed": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_void_p],
    "aao_set_timing": [ctypes.c_void_p, ctypes.c_int],
    "aao_get_timing": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_int64)],
    "aao_set_timing_mask": [ctypes.c_void_p, ctypes.c_uint],
    "aao_get_timing_ex": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
    "aao_tune": [ctypes.c_void_p, ctypes.c_int],
    "aao_set_tune_cache": [ctypes.c_char_p],
    "aao_get_config": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "aao_set_config": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int],
    "aao_config_shape": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "aao_batch_create": [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                         ctypes.POINTER(ctypes.c_void_p)],
    "aao_batch_destroy": [ctypes.c_void_p],
    "aao_batch_offsets": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)],
    "aao_batch_set_graph": [ctypes.c_void_p, ctypes.c_int],
    "aao_batch_get_config": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "aao_batch_set_config": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int],
    "aao_batch_tune": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                       ctypes.c_int, ctypes.c_int],
    "aao_batch_project_sine": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p],
    "aao_batch_build_rhs": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "aao_batch_apply_A": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "aao_batch_apply_Pinv": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "aao_batch_gmres": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                        ctypes.c_double, ctypes.c_int, ctypes.c_void_p],
    "aao_batch_gmres_ex": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                           ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p],
    "aao_batch_last_error": [ctypes.c_void_p],
    "aao_status_string": [ctypes.c_int],
    "aao_last_error": [ctypes.c_void_p],
}
_RET = {"aao_status_string": ctypes.c_char_p, "aao_last_error": ctypes.c_char_p,
        "aao_batch_last_error": ctypes.c_char_p}

_lib = None


def lib():
    """Load libaao.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (bind to torch's HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _RET.get(name, ctypes.c_int)
        _lib = L
    return _lib


class AAOError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        msg = lib().aao_status_string(status).decode()
        super().__init__(f"{where}: {msg} ({status}) {detail}".strip())


def check(status, where, ctx=None):
    if status < 0:
        detail = lib().aao_last_error(ctx).decode() if ctx else ""
        raise AAOError(status, where, detail)
    return status

GMRES_ZERO_GUESS, GMRES_TRANSPOSE, GMRES_CGS2_CLASSIC, GMRES_EARLY_CHECK = 1, 2, 4, 8
CONFIG_KINDS = ["fft_fwd", "shifted_solve", "fft_inv", "matvec"]
BATCH_CONFIG_KINDS = ["slab", "matvec_rows", "graph_span"]
KERNELS = ["fft_fwd", "shifted_solve", "fft_inv", "matvec", "cgs_dot", "cgs_update_dot",
           "cgs_update_norm", "axpy", "arnoldi_update", "sine_y"]
