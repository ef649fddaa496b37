"""ctypes binding of libpdmi.so (include/pd.h), one Python function per C
entry point with the same name.  Argument marshalling only: every step of the
solve runs in the library's HIP kernels.  Device buffers are passed as raw
pointers (e.g. torch.Tensor.data_ptr()) and streams as hipStream_t handles
(torch.cuda.Stream.cuda_stream)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PDMI_LIB selects another build of the same library (the sanitizer build)
LIB_PATH = os.environ.get("PDMI_LIB") or os.path.join(HERE, "libpdmi.so")

PD_OK, PD_EINVAL, PD_ENOMEM, PD_EDEVICE, PD_EUNSTABLE, PD_ENONFINITE, PD_ESTATE = 0, -1, -2, -3, -4, -5, -6
PD_LAW_EXPLIN, PD_LAW_TRILINEAR = 0, 1
PD_FP32, PD_FP64 = 0, 1
PD_ACC_KAHAN, PD_ACC_PLAIN, PD_ACC_STATE_ONLY, PD_ACC_FORCES_ONLY = 0, 1, 2, 3
PD_FIELD_S0, PD_FIELD_C, PD_FIELD_GF = 0, 1, 2
PD_DTYPE_F32, PD_DTYPE_F64 = 0, 1
PD_SHAPE_AUTO, PD_SHAPE_LDS_16x4x4, PD_SHAPE_LDS_8x8x4, PD_SHAPE_LDS_12x4x4, PD_SHAPE_GLOBAL_256 = -1, 0, 1, 2, 3
PD_N_SHAPES = 4
PD_MAX_CDF_LEVELS = 8
PD_COV_SQEXP, PD_COV_EXP = 0, 1


class PdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pd error {code}: {msg}")
        self.code = code


class pd_mesh_desc(C.Structure):
    _fields_ = [("extent", C.c_double * 3), ("dx", C.c_double), ("m_ratio", C.c_double),
                ("span", C.c_double), ("notch_depth", C.c_double), ("pad_width", C.c_double),
                ("thickness", C.c_double), ("plane_strain", C.c_int32)]


class pd_params(C.Structure):
    _fields_ = [("E", C.c_double), ("rho", C.c_double), ("GF", C.c_double), ("s0", C.c_double),
                ("k", C.c_double), ("alpha", C.c_double), ("law", C.c_int32),
                ("damping", C.c_double), ("dt", C.c_double), ("du", C.c_double),
                ("n_steps", C.c_int64), ("precision", C.c_int32), ("accumulate", C.c_int32),
                ("record_history", C.c_int32), ("checkpoint_every", C.c_int32)]


class pd_mesh_info_t(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("n_nodes", C.c_int64),
                ("n_bonds", C.c_int64), ("n_cut", C.c_int64), ("n_support", C.c_int32),
                ("n_load", C.c_int32), ("n_stencil", C.c_int32), ("delta", C.c_double)]


class pd_fib_params(C.Structure):
    _fields_ = [("fcm", C.c_double), ("weibull_m", C.c_double), ("alpha_E", C.c_double),
                ("delta_f", C.c_double), ("fck_min", C.c_double)]


class pd_batch_item(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("params", C.POINTER(pd_params)), ("n_samples", C.c_int64),
                ("s0", C.c_void_p), ("c", C.c_void_p), ("gf", C.c_void_p), ("field_dtype", C.c_int32),
                ("qoi", C.c_void_p), ("nstar", C.c_void_p), ("status", C.c_void_p), ("u_out", C.c_void_p)]


_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_P = C.POINTER

# name -> (argtypes) ; every function returns int except pd_last_error
SIGNATURES = {
    "pd_build_mesh": [_P(pd_mesh_desc), _P(_vp)],
    "pd_build_bonds": [_vp, _P(_i64)],
    "pd_mesh_get_info": [_vp, _P(pd_mesh_info_t)],
    "pd_mesh_get_pads": [_vp, _vp, _vp],
    "pd_set_material_field": [_vp, _i32, _i64, _vp, _i32, _i32, _vp],
    "pd_force_eval": [_vp, _P(pd_params), _i64, _vp, _vp, _vp],
    "pd_run": [_vp, _P(pd_params), _vp, _P(_vp)],
    "pd_qoi": [_vp, _P(_d), _P(_i64), _vp],
    "pd_run_state": [_vp, _vp, _vp],
    "pd_free_run": [_vp],
    "pd_run_batch": [_P(pd_batch_item), _i32, _vp],
    "pd_run_batch_static": [_P(pd_batch_item), _i32, _vp],
    "pd_batch_sync": [_vp],
    "pd_autotune": [_vp, _P(pd_params), _i64, _vp, _P(_i32), _vp],
    "pd_set_launch_shape": [_vp, _i32],
    "pd_qoi_grad": [_vp, _P(pd_params), _vp, _vp, _vp, _vp, _P(_d), _P(_i64), _vp],
    "pd_kl_build": [_vp, _d, _i32, _i32, _P(_vp)],
    "pd_kl_eigenvalues": [_vp, _vp],
    "pd_kl_field": [_vp, _vp, _i64, _d, _d, _vp, _i32, _vp],
    "pd_kl_free": [_vp],
    "pd_kl_build_exp": [_vp, _d, _i32, _P(_vp)],
    "pd_kl_extend": [_vp, _vp, _P(_vp)],
    "pd_kl_n_modes": [_vp, _P(_i32)],
    "pd_kl_gaussian": [_vp, _vp, _i64, _vp, _vp],
    "pd_fib_fields": [_vp, _vp, _i64, _P(pd_fib_params), _vp, _vp, _vp, _i32, _vp],
    "pd_level_stats": [_vp, _vp, _i64, _vp, _vp],
    "pd_mlmc_estimate": [_vp, _i32, _vp, _vp],
    "pd_mlmc_cdf": [_vp, _vp, _vp, _i32, _vp, _i64, _vp, _vp, _i64, _vp, _vp],
    "pd_mlmc_allocation": [_vp, _vp, _i32, _d, _vp, _vp],
    "pd_mlmc_bias": [_d, _d, _d, _d, _P(_d)],
    "pd_mlmc_fit_rate": [_vp, _vp, _i32, _P(_d), _P(_d)],
    "pd_free_mesh": [_vp],
    "pd_last_error": [],
}

_lib = None


def lib():
    """Load libpdmi.so; raises if it has not been built (there is no CPU
    fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2212_04415_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, argt in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = argt
            f.restype = C.c_char_p if name == "pd_last_error" else C.c_int
        _lib = L
    return _lib


def check(rc):
    if rc != PD_OK:
        raise PdError(rc, lib().pd_last_error().decode())
    return rc


def _wrap(name):
    def f(*args):
        return check(getattr(lib(), name)(*args))
    f.__name__ = name
    f.__doc__ = f"Calls {name} from libpdmi.so; raises PdError on a negative return code."
    return f


pd_build_mesh = _wrap("pd_build_mesh")
pd_build_bonds = _wrap("pd_build_bonds")
pd_mesh_get_info = _wrap("pd_mesh_get_info")
pd_mesh_get_pads = _wrap("pd_mesh_get_pads")
pd_set_material_field = _wrap("pd_set_material_field")
pd_force_eval = _wrap("pd_force_eval")
pd_run = _wrap("pd_run")
pd_qoi = _wrap("pd_qoi")
pd_run_state = _wrap("pd_run_state")
pd_free_run = _wrap("pd_free_run")
pd_run_batch = _wrap("pd_run_batch")
pd_run_batch_static = _wrap("pd_run_batch_static")
pd_batch_sync = _wrap("pd_batch_sync")
pd_autotune = _wrap("pd_autotune")
pd_set_launch_shape = _wrap("pd_set_launch_shape")
pd_qoi_grad = _wrap("pd_qoi_grad")
pd_kl_build = _wrap("pd_kl_build")
pd_kl_eigenvalues = _wrap("pd_kl_eigenvalues")
pd_kl_field = _wrap("pd_kl_field")
pd_kl_free = _wrap("pd_kl_free")
pd_kl_build_exp = _wrap("pd_kl_build_exp")
pd_kl_extend = _wrap("pd_kl_extend")
pd_kl_n_modes = _wrap("pd_kl_n_modes")
pd_kl_gaussian = _wrap("pd_kl_gaussian")
pd_fib_fields = _wrap("pd_fib_fields")
pd_level_stats = _wrap("pd_level_stats")
pd_mlmc_estimate = _wrap("pd_mlmc_estimate")
pd_mlmc_cdf = _wrap("pd_mlmc_cdf")
pd_mlmc_allocation = _wrap("pd_mlmc_allocation")
pd_mlmc_bias = _wrap("pd_mlmc_bias")
pd_mlmc_fit_rate = _wrap("pd_mlmc_fit_rate")
pd_free_mesh = _wrap("pd_free_mesh")


def pd_last_error():
    return lib().pd_last_error().decode()
