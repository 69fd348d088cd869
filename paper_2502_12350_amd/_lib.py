"""ctypes declarations of include/wfd.h (argument marshalling only).

Loading fails loudly when the in-tree library has not been built: there is
no CPU fallback anywhere in the package.
"""

from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# WFD_LIB may name another build of the same library (used to compare builds)
LIB_PATH = os.environ.get("WFD_LIB") or os.path.join(_PKG, "libwfd.so")

WFD_OK = 0
STATUS_NAMES = {0: "WFD_OK", -1: "WFD_E_ARG", -2: "WFD_E_CFL", -3: "WFD_E_RANGE",
                -4: "WFD_E_NOMEM", -5: "WFD_E_HIP", -6: "WFD_E_STATE"}
CKPT_FULL = 0
CKPT_REVOLVE = 1
CKPT_HOST = 2
K_FORWARD, K_ADJOINT, K_OTHER = 0, 1, 2
CNN_REDUCE_BYTES = 8192
NOALLOC_SCRATCH_BYTES = 64 << 20
SMOOTH_LAPLACE, SMOOTH_BESSEL = 1, 2
RESAMPLE_NEAREST, RESAMPLE_SINC = 1, 2


class wfd_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("ox", C.c_double), ("oy", C.c_double), ("oz", C.c_double),
                ("border", C.c_int32), ("dt", C.c_double), ("nt", C.c_int32),
                ("free_surface", C.c_int32), ("cpml", C.c_int32), ("fpeak", C.c_double),
                ("cpml_vmax", C.c_double)]


class wfd_ckpt(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_snapshots", C.c_int32), ("mem_fraction", C.c_double),
                ("host_store", C.c_void_p), ("host_bytes", C.c_uint64)]


class wfd_tuning(C.Structure):
    _fields_ = [("fwd_variant", C.c_int32), ("fwd_rounds", C.c_int32),
                ("adj_variant", C.c_int32), ("adj_rounds", C.c_int32)]


class wfd_gradient_opts(C.Structure):
    _fields_ = [("wavelet_grad_dev", C.c_void_p), ("out_exp2", C.c_int32),
                ("field_exp2_dev", C.c_void_p)]


class WfdError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


_P = C.c_void_p
_D3 = C.POINTER(C.c_double)
_SIGS = {
    "wfd_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, _P]),
    "wfd_set_stream": (C.c_int, [_P, _P]),
    "wfd_destroy": (C.c_int, [_P]),
    "wfd_model_bytes": (C.c_int, [C.POINTER(wfd_grid), C.c_int32, C.POINTER(C.c_size_t)]),
    "wfd_set_model": (C.c_int, [_P, C.POINTER(wfd_grid), _P, _P, _P, C.c_size_t]),
    "wfd_workspace_bytes": (C.c_int, [_P, C.c_int32, C.POINTER(wfd_ckpt), C.POINTER(C.c_size_t)]),
    "wfd_host_store_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "wfd_forward": (C.c_int, [_P, _P, _D3, C.c_int32, _D3, _P, _P, _P, C.c_size_t]),
    "wfd_forward_noalloc": (C.c_int, [_P, _P, _D3, C.c_int32, _D3, _P, _P]),
    "wfd_forward_misfit": (C.c_int, [_P, _P, _D3, C.c_int32, _D3, _P, _P, _P, _P, C.c_size_t]),
    "wfd_misfit_workspace_bytes": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_size_t)]),
    "wfd_gradient": (C.c_int, [_P, _P, _D3, C.c_int32, _D3, _P, C.POINTER(wfd_ckpt), _P, _P,
                               _P, _P, _P, C.c_size_t]),
    "wfd_gradient_ex": (C.c_int, [_P, _P, _D3, C.c_int32, _D3, _P, C.POINTER(wfd_ckpt), _P, _P,
                                  _P, _P, C.POINTER(wfd_gradient_opts), _P, C.c_size_t]),
    "wfd_gradient_finish": (C.c_int, [_P, _P, C.c_int32]),
    "wfd_set_tuning": (C.c_int, [_P, C.POINTER(wfd_tuning)]),
    "wfd_get_tuning": (C.c_int, [_P, C.POINTER(wfd_tuning)]),
    "wfd_autotune": (C.c_int, [_P, C.c_int32, _P, C.c_size_t, C.POINTER(wfd_tuning),
                               C.POINTER(C.c_double)]),
    "wfd_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p), _P,
                                   _D3, C.POINTER(C.c_int32), C.POINTER(_D3),
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_size_t)]),
    "wfd_batch_run": (C.c_int, [_P, C.c_int32]),
    "wfd_gbatch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p), _P,
                                    _D3, C.POINTER(C.c_int32), C.POINTER(_D3),
                                    C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_void_p), C.POINTER(C.c_size_t)]),
    "wfd_gbatch_run": (C.c_int, [_P, C.c_int32]),
    "wfd_gbatch_destroy": (C.c_int, [_P]),
    "wfd_batch_destroy": (C.c_int, [_P]),
    "wfd_cnn_packed_elems": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]),
    "wfd_cnn_pack_weights": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P]),
    "wfd_cnn_conv": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P,
                               C.c_int32, _P, _P, C.c_int32, _P, _P, _P]),
    "wfd_cnn_wgrad_workspace_bytes": (C.c_int, [C.c_int32, C.c_int32, C.c_int32,
                                                C.POINTER(C.c_size_t)]),
    "wfd_cnn_wgrad": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                _P, _P, _P, C.c_size_t, _P]),
    "wfd_cnn_mse": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, C.c_size_t, _P]),
    "wfd_cnn_adam": (C.c_int, [_P, _P, _P, _P, C.c_int32, C.c_float, C.c_float, C.c_float,
                               C.c_float, C.c_int32, _P]),
    "wfd_cnn_pack_input": (C.c_int, [_P, _P, C.c_int64, C.c_float, _P, _P, C.c_size_t, _P]),
    "wfd_smooth_workspace_bytes": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                             C.POINTER(C.c_size_t)]),
    "wfd_smooth": (C.c_int, [C.c_int32, _P, _P, C.c_int32, C.c_int32, C.c_int32, _D3, _D3,
                             C.c_double, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_int32), _P]),
    "wfd_resample": (C.c_int, [C.c_int32, _P, C.c_int32, C.c_int32, C.c_double, _P, C.c_int32,
                               C.c_double, _P]),
    "wfd_map_position": (C.c_int, [C.POINTER(wfd_grid), _D3, C.POINTER(C.c_int32)]),
    "wfd_cfl_ratio": (C.c_int, [C.POINTER(wfd_grid), C.c_double, C.c_double, _D3]),
    "wfd_checkpoint_plan": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.c_int64,
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "wfd_set_profiling": (C.c_int, [_P, C.c_int32]),
    "wfd_kernel_stats": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "wfd_last_error": (C.c_char_p, []),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_2502_12350_amd.build or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def check(status: int) -> None:
    if status != WFD_OK:
        msg = lib().wfd_last_error()
        raise WfdError(status, msg.decode() if msg else "")
