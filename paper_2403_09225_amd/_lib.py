"""ctypes declarations of the C ABI in include/pwa.h and include/pwa_mlp.h.

Loading imports torch first so that libpwa.so binds to the HIP runtime torch
already loaded (both carry the soname libamdhip64.so.7): device pointers and
streams from torch are then valid inside the library.  There is no fallback:
if the library is missing, loading raises.
"""

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpwa.so")

PWA_MAX_RES = 64
PWA_OK = 0
PWA_E_INVALID = -1
PWA_E_WORKSPACE = -2
PWA_E_HIP = -3
PWA_E_DOMAIN = -4
PWA_E_NOCONV = -5
PWA_E_STATE = -6
PWA_PREC_F64 = 0
PWA_PREC_F32 = 1
PWA_STREAM_F64 = 1
PWA_STREAM_F32 = 2
PWA_LINESHAPE_BREIT_WIGNER = 0
PWA_LINESHAPE_FLATTE = 1
OPERANDS = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "f16s": 4}

c_double, c_int32, c_int64, c_size_t, c_void_p = (
    ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p)


class PwaModel(ctypes.Structure):
    _fields_ = [("parent_mass", c_double), ("masses", c_double * 3), ("r", c_double),
                ("n_res", c_int32), ("width_mode", c_int32),
                ("channel", c_int32 * PWA_MAX_RES), ("spin", c_int32 * PWA_MAX_RES),
                ("lineshape", c_int32 * PWA_MAX_RES), ("flatte_masses", c_double * 2),
                ("flatte_ratio", c_double), ("parent_spin", c_int32), ("reserved", c_int32)]


class PwaFitOpts(ctypes.Structure):
    _fields_ = [("xtol", c_double), ("maxiter", c_int32), ("cg_maxiter", c_int32),
                ("time_cap_s", c_double), ("hvp_precision", c_int32),
                ("free_mask_set", c_int32), ("free_mask", ctypes.c_uint8 * (4 * PWA_MAX_RES)),
                ("forcing", c_int32), ("precondition", c_int32), ("reconjugate", c_int32)]


class PwaMlpDims(ctypes.Structure):
    _fields_ = [("n_in", c_int32), ("n_h1", c_int32), ("n_h2", c_int32), ("n_out", c_int32)]


class PwaFitReport(ctypes.Structure):
    _fields_ = [("nll", c_double), ("grad_max", c_double), ("seconds", c_double),
                ("iterations", c_int32), ("n_nll", c_int32), ("n_grad", c_int32),
                ("n_hvp", c_int32), ("status", c_int32), ("converged", c_int32)]


_P = c_void_p
SIGNATURES = {
    "pwa_create": (c_int32, [ctypes.POINTER(PwaModel), c_int32, ctypes.POINTER(_P)]),
    "pwa_destroy": (None, [_P]),
    "pwa_workspace_bytes": (c_size_t, [_P, c_int64, c_int64]),
    "pwa_bind": (c_int32, [_P, _P, _P, c_int64, _P, _P, c_int64, _P, c_size_t, _P]),
    "pwa_bind_oriented": (c_int32, [_P, _P, _P, _P, _P, c_int64, _P, _P, _P, _P, c_int64, _P,
                                    c_size_t, _P]),
    "pwa_set_precision": (c_int32, [_P, c_int32]),
    "pwa_nll": (c_int32, [_P, _P, _P, _P]),
    "pwa_grad": (c_int32, [_P, _P, _P, _P, _P]),
    "pwa_hvp": (c_int32, [_P, _P, _P, _P, _P, _P, _P]),
    "pwa_partials": (c_int32, [_P, _P, _P, _P, _P]),
    "pwa_hvp_reuse": (c_int32, [_P, _P, _P, _P, _P, _P]),
    "pwa_partials_reuse": (c_int32, [_P, _P, _P, _P]),
    "pwa_intensity": (c_int32, [_P, _P, c_int32, _P, _P]),
    "pwa_combine": (c_int32, [c_int32, c_int32, _P, c_int64, c_int64, _P, _P, _P, _P, _P]),
    "pwa_fit": (c_int32, [_P, _P, ctypes.POINTER(PwaFitOpts), ctypes.POINTER(PwaFitReport), _P]),
    "pwa_fit_bfgs": (c_int32, [_P, _P, ctypes.POINTER(PwaFitOpts), ctypes.POINTER(PwaFitReport), _P]),
    "pwa_device_status": (c_int32, [_P, _P]),
    "pwa_status_str": (ctypes.c_char_p, [c_int32]),
    "pwa_n_par": (c_int32, [_P]),
    "pwa_stream_fields": (c_int32, [_P]),
    "pwa_set_launch_shape": (c_int32, [_P, c_int32, c_int32, c_int32]),
    "pwa_grid_blocks": (c_int32, [_P]),
    "pwa_set_kernel_timing": (c_int32, [_P, c_int32]),
    "pwa_kernel_time": (c_int32, [_P, ctypes.POINTER(c_double), ctypes.POINTER(c_int64)]),
    "pwa_batched_workspace_bytes": (c_size_t, [_P, c_int64, c_int32, c_int32]),
    "pwa_freeze": (c_int32, [_P, _P, c_int32, c_int32, _P, c_size_t, _P]),
    "pwa_nll_batched": (c_int32, [_P, _P, c_int32, _P, _P]),
    "pwa_gram": (c_int32, [_P, _P, _P]),
    "pwa_hessian": (c_int32, [_P, _P, _P, _P]),
    "pwa_fit_fractions": (c_int32, [_P, _P, _P, _P, _P]),
    "pwa_covariance": (c_int32, [c_int32, _P, _P, _P]),
    "pwa_fraction_matrix_workspace_bytes": (c_size_t, [_P]),
    "pwa_fraction_matrix": (c_int32, [_P, _P, _P, c_size_t, _P, _P]),
    "pwa_propagate": (c_int32, [c_int32, c_int32, _P, _P, _P]),
    # include/pwa_mlp.h
    "pwa_hist2d": (c_int32, [_P, _P, _P, c_int32, c_double, ctypes.POINTER(c_double), _P, _P]),
    "pwa_mlp_n_params": (c_int64, [ctypes.POINTER(PwaMlpDims)]),
    "pwa_mlp_n_transposed": (c_int64, [ctypes.POINTER(PwaMlpDims)]),
    "pwa_mlp_workspace_bytes": (c_size_t, [ctypes.POINTER(PwaMlpDims), c_int32]),
    "pwa_mlp_cast": (c_int32, [ctypes.POINTER(PwaMlpDims), _P, _P, _P, _P]),
    "pwa_mlp_forward": (c_int32, [ctypes.POINTER(PwaMlpDims), _P, _P, _P, c_int32, _P, _P,
                                  c_size_t, _P]),
    "pwa_mlp_forward_noalloc": (c_int32, [ctypes.POINTER(PwaMlpDims), _P, _P, _P, c_int32, _P,
                                          _P]),
    "pwa_mlp_backward": (c_int32, [ctypes.POINTER(PwaMlpDims), _P, _P, _P, c_int32, _P, c_size_t,
                                   _P, _P, _P]),
    "pwa_mlp_adam": (c_int32, [ctypes.POINTER(PwaMlpDims), _P, _P, _P, _P, c_int32, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               _P, _P, _P]),
}

_lib = None


def load(path=LIB_PATH):
    """Load libpwa.so (after torch) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime shared with torch)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2403_09225_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PwaError(RuntimeError):
    def __init__(self, fn, code):
        msg = load().pwa_status_str(code).decode()
        super().__init__(f"{fn} failed: {msg} ({code})")
        self.code = code


def check(fn, code):
    if code != PWA_OK:
        raise PwaError(fn, code)
    return code
