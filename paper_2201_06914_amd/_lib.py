"""ctypes declarations of librtm.so (include/rtm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtm.so")

RTM_F64, RTM_F32, RTM_BF16, RTM_BF16X2, RTM_I8, RTM_F16S = 0, 1, 2, 3, 4, 5
RTM_PROBE_U, RTM_PROBE_UTT = 0, 1
RTM_E_NONFINITE = 9

# every symbol include/rtm.h declares
EXPORTS = (
    "rtm_plan_create", "rtm_plan_destroy", "rtm_plan_workspace_bytes", "rtm_cfl_bound",
    "rtm_status_str", "rtm_set_stencil_variant", "rtm_last_error", "rtm_forward_probe",
    "rtm_adjoint_probe", "rtm_image", "fwi_gradient", "rtm_dot", "rtm_profile_enable",
    "rtm_profile_read", "rtm_bar_to_rows", "rtm_exact_workspace_bytes", "fwi_gradient_exact",
    "rtm_adjoint_image", "rtm_set_stencil_blocks", "rtm_autotune_stencil",
    "rtm_batch_create", "rtm_batch_destroy", "rtm_batch_workspace_bytes", "fwi_gradient_batched",
    "rtm_tti_workspace_bytes", "rtm_tti_forward_probe", "rtm_tti_adjoint_probe",
    "fwi_gradient_tti", "rtm_set_exact_fused", "rtm_set_tti_shape", "rtm_rf_workspace_bytes",
    "rtm_sketch", "rtm_orthonormalize", "fwi_gradient_rf", "rtm_offset_gathers",
    "rtm_stream_status", "rtm_forward_probe_range", "fwi_gradient_noalloc",
    "rtm_device_copy", "rtm_residual", "rtm_batch_stream_status", "rtm_tti_spectral_radius",
    "rtm_set_stencil_alternate", "rtm_set_probe_nt", "rtm_set_probe_grid", "rtm_set_graph", "rtm_set_tti_blocks",
)

RTM_NOALLOC_SCRATCH_BYTES = 256 << 20


class ShotIO(ctypes.Structure):
    _fields_ = [("m", ctypes.c_void_p), ("src_pos", ctypes.POINTER(ctypes.c_double)),
                ("q", ctypes.c_void_p), ("rec_pos", ctypes.POINTER(ctypes.c_double)),
                ("d_obs", ctypes.c_void_p), ("Z", ctypes.c_void_p), ("Ubar", ctypes.c_void_p),
                ("resid", ctypes.c_void_p), ("grad", ctypes.c_void_p)]


class RtmDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("nz", ctypes.c_int64), ("ny", ctypes.c_int64), ("nx", ctypes.c_int64),
        ("h", ctypes.c_double), ("dt", ctypes.c_double),
        ("nt", ctypes.c_int32), ("nb", ctypes.c_int32),
        ("c_ref", ctypes.c_double), ("R", ctypes.c_double), ("c_max", ctypes.c_double),
        ("field_dtype", ctypes.c_int), ("probe_dtype", ctypes.c_int),
        ("r", ctypes.c_int32), ("k_block", ctypes.c_int32),
        ("nsrc", ctypes.c_int32), ("nrec", ctypes.c_int32),
    ]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


def load() -> ctypes.CDLL:
    """Loads librtm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950); the library has no non-HIP fallback")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, sz, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    L.rtm_plan_create.argtypes = [ctypes.POINTER(RtmDesc), ctypes.POINTER(_vp)]
    L.rtm_plan_create.restype = ctypes.c_int
    L.rtm_plan_destroy.argtypes = [_vp]
    L.rtm_plan_destroy.restype = None
    L.rtm_plan_workspace_bytes.argtypes = [_vp, ctypes.POINTER(sz)]
    L.rtm_plan_workspace_bytes.restype = ctypes.c_int
    L.rtm_cfl_bound.argtypes = [i32]
    L.rtm_cfl_bound.restype = dbl
    L.rtm_status_str.argtypes = [ctypes.c_int]
    L.rtm_status_str.restype = ctypes.c_char_p
    L.rtm_last_error.argtypes = []
    L.rtm_last_error.restype = ctypes.c_char_p
    L.rtm_set_stencil_variant.argtypes = [ctypes.c_int]
    L.rtm_set_stencil_variant.restype = None
    L.rtm_forward_probe.argtypes = [_vp, _vp, _dp, _vp, _dp, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                    _vp, _vp, _vp, sz, _vp]
    L.rtm_forward_probe.restype = ctypes.c_int
    L.rtm_adjoint_probe.argtypes = [_vp, _vp, _dp, _vp, _dp, _vp, _vp, ctypes.c_int, _vp, _vp, sz,
                                    _vp]
    L.rtm_adjoint_probe.restype = ctypes.c_int
    L.rtm_image.argtypes = [_vp, _vp, _vp, dbl, _vp, _vp]
    L.rtm_image.restype = ctypes.c_int
    L.fwi_gradient.argtypes = [_vp, _vp, _dp, _vp, _dp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp,
                               _vp, _vp, sz, _vp]
    L.fwi_gradient.restype = ctypes.c_int
    L.fwi_gradient_noalloc.argtypes = [_vp, _vp, _dp, _vp, _dp, _vp, _vp, ctypes.c_int, _vp, _vp,
                                       _vp, _vp, _vp, _vp]
    L.fwi_gradient_noalloc.restype = ctypes.c_int
    L.rtm_tti_spectral_radius.argtypes = [_vp, _vp, _vp, i32, ctypes.c_uint64,
                                          ctypes.POINTER(dbl), _vp, sz, _vp]
    L.rtm_tti_spectral_radius.restype = ctypes.c_int
    L.rtm_residual.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, sz, _vp]
    L.rtm_residual.restype = ctypes.c_int
    L.rtm_batch_stream_status.argtypes = [_vp, _vp, _vp]
    L.rtm_batch_stream_status.restype = ctypes.c_int
    L.rtm_device_copy.argtypes = [_vp, _vp, sz, _vp]
    L.rtm_device_copy.restype = ctypes.c_int
    L.rtm_dot.argtypes = [_vp, _vp, _vp, i64, _vp, _vp, sz, _vp]
    L.rtm_dot.restype = ctypes.c_int
    L.rtm_exact_workspace_bytes.argtypes = [_vp, i32, ctypes.POINTER(sz)]
    L.rtm_exact_workspace_bytes.restype = ctypes.c_int
    L.fwi_gradient_exact.argtypes = [_vp, _vp, _dp, _vp, _dp, _vp, i32, _vp, _vp, _vp, _vp, sz, _vp]
    L.fwi_gradient_exact.restype = ctypes.c_int
    u64 = ctypes.c_uint64
    L.rtm_rf_workspace_bytes.argtypes = [_vp, ctypes.POINTER(sz)]
    L.rtm_rf_workspace_bytes.restype = ctypes.c_int
    L.rtm_sketch.argtypes = [_vp, _vp, _dp, _vp, u64, _vp, _vp, sz, _vp]
    L.rtm_sketch.restype = ctypes.c_int
    L.rtm_orthonormalize.argtypes = [_vp, _vp, _vp, _vp, sz, _vp]
    L.rtm_orthonormalize.restype = ctypes.c_int
    L.fwi_gradient_rf.argtypes = [_vp, _vp, _dp, _vp, _dp, _vp, u64, _vp, _vp, _vp, _vp, _vp,
                                  _vp, _vp, sz, _vp]
    L.fwi_gradient_rf.restype = ctypes.c_int
    L.rtm_offset_gathers.argtypes = [_vp, _vp, _vp, i32, i32, dbl, _vp, _vp]
    L.rtm_stream_status.argtypes = [_vp, _vp, _vp]
    L.rtm_forward_probe_range.argtypes = [_vp, _vp, _dp, _vp, _dp, _vp, _vp, i32, i32, _vp, i32,
                                          i32, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.rtm_offset_gathers.restype = ctypes.c_int
    L.rtm_adjoint_image.argtypes = [_vp, _vp, _dp, _vp, _vp, ctypes.c_int, _vp, dbl, _vp, _vp, sz,
                                    _vp]
    L.rtm_adjoint_image.restype = ctypes.c_int
    L.rtm_set_probe_nt.argtypes = [i32]
    L.rtm_set_probe_nt.restype = None
    L.rtm_set_probe_grid.argtypes = [i32, i32]
    L.rtm_set_tti_blocks.argtypes = [i32, i32]
    L.rtm_set_tti_blocks.restype = None
    L.rtm_set_probe_grid.restype = None
    L.rtm_set_graph.argtypes = [i32]
    L.rtm_set_graph.restype = None
    L.rtm_set_stencil_alternate.argtypes = [i32]
    L.rtm_set_stencil_alternate.restype = None
    L.rtm_set_stencil_blocks.argtypes = [i32]
    L.rtm_set_stencil_blocks.restype = None
    L.rtm_autotune_stencil.argtypes = [_vp, _vp, _vp, sz, i32, ctypes.POINTER(i32),
                                       ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i64), _vp]
    L.rtm_autotune_stencil.restype = ctypes.c_int
    L.rtm_batch_create.argtypes = [ctypes.POINTER(RtmDesc), i32, ctypes.POINTER(_vp)]
    L.rtm_batch_create.restype = ctypes.c_int
    L.rtm_batch_destroy.argtypes = [_vp]
    L.rtm_batch_destroy.restype = None
    L.rtm_batch_workspace_bytes.argtypes = [_vp, ctypes.POINTER(sz)]
    L.rtm_batch_workspace_bytes.restype = ctypes.c_int
    L.fwi_gradient_batched.argtypes = [_vp, ctypes.POINTER(ShotIO), _vp, i32, _vp, sz, _vp]
    L.fwi_gradient_batched.restype = ctypes.c_int
    L.rtm_set_exact_fused.argtypes = [i32]
    L.rtm_set_exact_fused.restype = None
    L.rtm_set_tti_shape.argtypes = [i32]
    L.rtm_set_tti_shape.restype = None
    L.rtm_tti_workspace_bytes.argtypes = [_vp, ctypes.POINTER(sz)]
    L.rtm_tti_workspace_bytes.restype = ctypes.c_int
    L.rtm_tti_forward_probe.argtypes = [_vp, _vp, _vp, _dp, _vp, _dp, _vp, _vp, ctypes.c_int, _vp,
                                        _vp, sz, _vp]
    L.rtm_tti_forward_probe.restype = ctypes.c_int
    L.rtm_tti_adjoint_probe.argtypes = [_vp, _vp, _vp, _dp, _vp, _dp, _vp, _vp, ctypes.c_int, _vp,
                                        _vp, sz, _vp]
    L.rtm_tti_adjoint_probe.restype = ctypes.c_int
    L.fwi_gradient_tti.argtypes = [_vp, _vp, _vp, _dp, _vp, _dp, _vp, _vp, ctypes.c_int, _vp, _vp,
                                   _vp, _vp, _vp, _vp, sz, _vp]
    L.fwi_gradient_tti.restype = ctypes.c_int
    L.rtm_bar_to_rows.argtypes = [_vp, _vp, _vp, _vp]
    L.rtm_bar_to_rows.restype = ctypes.c_int
    L.rtm_profile_enable.argtypes = [i32]
    L.rtm_profile_enable.restype = None
    L.rtm_profile_read.argtypes = [i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    L.rtm_profile_read.restype = ctypes.c_int
    _lib = L
    return L
