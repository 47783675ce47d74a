"""ctypes binding of libfil.so (argument marshalling only).

Every numerical step runs in the HIP library.  If the library has not been
built this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfil.so")

FIL_OK = 0
STATUS = {0: "FIL_OK", -1: "FIL_EINVAL", -2: "FIL_EHIP", -3: "FIL_ENOCONV", -4: "FIL_ENONFINITE", -5: "FIL_ENOMEM"}
PREC = {"f64": 0, "f32tile": 1}


class FilError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


_lib = None
_vp = C.c_void_p
_i64 = C.c_int64
_d = C.c_double
_i = C.c_int


class Params(C.Structure):
    _fields_ = [("a", _d), ("eta", _d), ("dL", _d), ("KB", _d), ("KT", _d), ("chi", _d), ("FS", _d),
                ("grav", _d * 3), ("dt", _d), ("tol", _d), ("kmax", C.c_int32), ("prec", C.c_int32),
                ("j0_mode", C.c_int32), ("j0_factor", C.c_int32),
                ("K0", _d), ("kw", _d), ("omega", _d)]


class StepReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("mobility_applies", C.c_int32), ("converged", C.c_int32),
                ("applies_f64", C.c_int32), ("resid", _d), ("used_learned", C.c_int32), ("pad", C.c_int32)]


class JfnkReport(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("krylov_iters", C.c_int32), ("mobility_applies", C.c_int32),
                ("converged", C.c_int32), ("resid", _d)]


def _declare(L):
    L.fil_last_error.restype = C.c_char_p
    L.fil_rpy_workspace_bytes.argtypes = [_i64, _i]
    L.fil_rpy_workspace_bytes.restype = _i64
    L.fil_rpy_mobility_apply.argtypes = [_i64, _vp, _vp, _vp, _d, _d, _i, _vp, _vp, _vp, _i64, _vp]
    L.fil_rpy_mobility_apply_noalloc.argtypes = [_i64, _vp, _vp, _vp, _d, _d, _i, _vp, _vp, _vp]
    L.fil_rpy_noalloc_scratch_bytes.argtypes = []
    L.fil_rpy_noalloc_scratch_bytes.restype = _i64
    L.fil_rpy_mobility_apply_timed.argtypes = [_i64, _vp, _vp, _vp, _d, _d, _i, _vp, _vp, _vp, _i64, _vp, _vp, _vp]
    L.fil_filament_internal_forces.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp, _d, _d, _d, _vp, _vp, _vp]
    L.fil_rpy_batch_create.argtypes = [_i64, _vp, _i, C.POINTER(_vp)]
    L.fil_rpy_batch_workspace_bytes.argtypes = [_vp]
    L.fil_rpy_batch_workspace_bytes.restype = _i64
    L.fil_rpy_mobility_apply_batched.argtypes = [_vp, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp, _i64, _vp]
    L.fil_rpy_batch_destroy.argtypes = [_vp]
    L.fil_rpy_batch_destroy.restype = None
    if hasattr(L, "fil_create"):
        L.fil_create.argtypes = [C.POINTER(Params), _i64, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)]
        L.fil_destroy.argtypes = [_vp]
        L.fil_destroy.restype = None
        L.fil_bdf2_step.argtypes = [_vp, _vp]
        L.fil_broyden_begin.argtypes = [_vp, _vp, _vp]
        L.fil_broyden_update.argtypes = [_vp, _vp, _vp]
        L.fil_residual.argtypes = [_vp, _vp, _vp]
        L.fil_get_state.argtypes = [_vp, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp),
                                    C.POINTER(_i64), C.POINTER(_d), C.POINTER(_i64)]
        L.fil_read_state.argtypes = [_vp, _vp, _vp, _vp]
        L.fil_checkpoint.argtypes = [_vp, C.c_char_p]
        L.fil_restore.argtypes = [_vp, C.c_char_p]
        L.fil_set_stream.argtypes = [_vp, _vp]
        L.fil_set_suspension_params.argtypes = [_vp, _vp, _vp, _vp]
        L.fil_set_external_forces.argtypes = [_vp, _vp]
        L.fil_set_periodic_fcm.argtypes = [_vp, _vp, _vp, _d]
        L.fil_set_wall.argtypes = [_vp]
        L.fil_set_motor.argtypes = [_vp, _d, _d]
        L.fil_set_geometric_switch.argtypes = [_vp, _vp, _vp, _d, _d, _d, _i]
        L.fil_read_switch.argtypes = [_vp, _vp]
        L.fil_rpy_wall_workspace_bytes.argtypes = [_i64]
        L.fil_rpy_wall_workspace_bytes.restype = _i64
        L.fil_rpy_wall_apply.argtypes = [_i64, _vp, _vp, _vp, _d, _d, _i, _vp, _vp, _vp, _i64, _vp]
        L.fil_fcm_create.argtypes = [_vp, _vp, _d, _d, _d, _vp]
        L.fil_fcm_apply.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]
        L.fil_fcm_destroy.argtypes = [_vp]
        L.fil_fcm_destroy.restype = None
        L.fil_jfnk_step.argtypes = [_vp, C.c_int, _d, _d, C.c_int, _vp]
        L.fil_jfb_step.argtypes = [_vp, C.c_int, _d, _d, C.c_int, _vp]
        L.fil_set_graph.argtypes = [_vp, _i]
        L.fil_sim_features.argtypes = [_vp, _vp]
        L.fil_sim_step_target.argtypes = [_vp, _vp]
        L.fil_sim_set_mlp.argtypes = [_vp, _vp, _i]
        L.fil_sim_fallbacks.argtypes = [_vp, C.POINTER(_i64)]
    if hasattr(L, "fil_mlp_create"):
        _i32 = C.c_int32
        L.fil_mlp_create.argtypes = [_i32, _i32, _i32, _i32, C.c_uint64, C.POINTER(_vp)]
        L.fil_mlp_destroy.argtypes = [_vp]
        L.fil_mlp_destroy.restype = None
        L.fil_mlp_dims.argtypes = [_vp, _vp, C.POINTER(_i64)]
        L.fil_mlp_set_params.argtypes = [_vp, _vp]
        L.fil_mlp_get_params.argtypes = [_vp, _vp]
        L.fil_mlp_set_norm.argtypes = [_vp, _vp]
        L.fil_mlp_get_norm.argtypes = [_vp, _vp]
        L.fil_mlp_save.argtypes = [_vp, C.c_char_p]
        L.fil_mlp_load.argtypes = [_vp, C.c_char_p]
        L.fil_mlp_fit_norm.argtypes = [_vp, _i64, _vp, _vp, _vp]
        L.fil_mlp_standardize.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp, _vp]
        L.fil_mlp_forward.argtypes = [_vp, _i32, _vp, _vp, _vp]
        L.fil_mlp_backward.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
        L.fil_mlp_adam_step.argtypes = [_vp, C.c_float, _vp]
        L.fil_mlp_train_step.argtypes = [_vp, _i32, _vp, _vp, _vp, C.c_float, _vp, _vp]
        L.fil_set_timing.argtypes = [_vp, _i]
        L.fil_get_timing.argtypes = [_vp, C.POINTER(_d), C.POINTER(_i64)]


def lib():
    """Load libfil.so; raises if it is missing (build it with paper_1903_12609_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfil.so is not built (run `python -m paper_1903_12609_amd.build`); "
                               "there is no fallback path")
        # torch carries its own HIP runtime; it must bring the device up before
        # the library's runtime makes its first call, or torch no longer finds it
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def check(rc):
    if rc != FIL_OK:
        raise FilError(rc, lib().fil_last_error().decode())
    return rc
