"""ctypes loader for libdcfbp.so and the C structures of include/dcfbp.h.

The library must have been built (``__graft_entry__.build()`` or
``python paper_2410_14900_amd/build.py``); there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_size_t, c_uint32, c_uint64, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdcfbp.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "dcfbp.h")

DC_OK, DC_EINVAL, DC_ESHAPE, DC_EDTYPE, DC_EALIGN, DC_EHIP, DC_ENOTSUP, DC_ENOMEM = range(8)
STATUS_NAMES = ["DC_OK", "DC_EINVAL", "DC_ESHAPE", "DC_EDTYPE", "DC_EALIGN", "DC_EHIP", "DC_ENOTSUP",
                "DC_ENOMEM"]
DC_F32, DC_BF16, DC_F16 = 0, 1, 2
DC_WEIGHT_ANALYTIC, DC_WEIGHT_RAW = 0, 1


class DcGrid(ctypes.Structure):
    _fields_ = [("nu", c_int32), ("nv", c_int32), ("du", c_double), ("dv", c_double),
                ("n_theta", c_int32), ("n_s", c_int32), ("ds", c_double),
                ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("vx", c_double), ("vy", c_double), ("vz", c_double),
                ("ox", c_double), ("oy", c_double), ("oz", c_double)]


class DcView(ctypes.Structure):
    _fields_ = [("src", c_double * 3), ("det_center", c_double * 3), ("ex", c_double * 3),
                ("ey", c_double * 3), ("tangent", c_double * 3)]


class DcOrbitSegment(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("start", c_int32), ("count", c_int32), ("closed", c_int32),
                ("p0", c_double), ("p1", c_double), ("phi_max", c_double), ("freq", c_double)]


DC_SEG_CIRCLE, DC_SEG_ARC, DC_SEG_LINE, DC_SEG_SINUSOID = 1, 2, 3, 4


class DcKnobs(ctypes.Structure):
    _fields_ = [("splat_angles", c_int32), ("interp_tile_u", c_int32), ("interp_angles", c_int32),
                ("bp_block_y", c_int32), ("fp_tile_u", c_int32)]


class DcBounds(ctypes.Structure):
    _fields_ = [("splat_angles", c_int32), ("splat_max_terms", c_int32), ("splat_checked", c_int32),
                ("interp_window", c_int32), ("interp_local", c_int32), ("cone_max_terms", c_int32),
                ("bp_stage", c_int32), ("cone_form", c_int32), ("bp_block", c_int32 * 3),
                ("interp_tile", c_int32 * 2), ("splat_qmax", c_float), ("cone_qmax", c_float),
                ("bp_pitch", c_int32)]


class DcError(RuntimeError):
    def __init__(self, status, where, msg):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__("%s failed with %s: %s" % (where, name, msg))


_i, _p, _vp = c_int32, c_void_p, c_void_p
SIGNATURES = {
    "dc_validate": (_i, [POINTER(DcGrid), POINTER(DcView), _i]),
    "dc_plan_create": (_i, [POINTER(DcGrid), POINTER(DcView), _i, c_uint32, POINTER(c_void_p)]),
    "dc_plan_create_batched": (_i, [POINTER(DcGrid), POINTER(DcView), _i, POINTER(c_int32), _i, c_uint32,
                                   POINTER(c_void_p)]),
    "dc_plan_destroy": (_i, [_p]),
    "dc_plan_bounds": (_i, [POINTER(DcGrid), POINTER(DcView), _i, POINTER(DcBounds)]),
    "dc_plan_get_knobs": (_i, [_p, POINTER(DcKnobs)]),
    "dc_plan_set_knobs": (_i, [_p, POINTER(DcKnobs)]),
    "dc_plan_autotune": (_i, [_p, c_uint32, _vp, POINTER(DcKnobs), POINTER(c_double), POINTER(c_int32)]),
    "dc_last_error": (c_char_p, []),
    "dc_plan_n_views": (_i, [_p]),
    "dc_plan_n_samples": (_i, [_p]),
    "dc_plan_grid": (_i, [_p, POINTER(DcGrid)]),
    "dc_weight_radon": (_i, [_p, _vp, _vp, _i, _i, _i, _vp]),
    "dc_weight_radon_noalloc": (_i, [_p, _vp, _vp, _i, _i, _i, _vp]),
    "dc_weight_radon_adjoint": (_i, [_p, _vp, _i, _vp, _i, _i, _vp]),
    "dc_filter": (_i, [_p, _vp, _i, _vp, _i, _vp, _i, _i, _i, _vp]),
    "dc_filter_adjoint": (_i, [_p, _vp, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, _i, _vp]),
    "dc_detector_bp": (_i, [_p, _vp, _i, _vp, _i, _i, _i, _vp]),
    "dc_detector_bp_adjoint": (_i, [_p, _vp, _i, _vp, _i, _i, _i, _vp]),
    "dc_cone_bp": (_i, [_p, _vp, _i, _vp, _i, _i, _i, _i, _vp]),
    "dc_cone_bp_adjoint": (_i, [_p, _vp, _vp, _vp, _i, _i, _i, _vp]),
    "dc_smooth_weights": (_i, [_p, _vp, _vp, c_double, _i, _i, _i, _vp]),
    "dc_smooth_weights_adjoint": (_i, [_p, _vp, _vp, c_double, _i, _i, _i, _vp]),
    "dc_project": (_i, [_p, _vp, _vp, _i, _i, _vp]),
    "dc_crofton_workspace_bytes": (c_size_t, [POINTER(DcOrbitSegment), _i, _i]),
    "dc_crofton_weights": (_i, [_p, POINTER(DcOrbitSegment), _i, c_double, _i, c_double, c_double, _i, _vp, _i, _i,
                                _vp, c_size_t, _vp]),
    "dc_poisson_noise": (_i, [_vp, _vp, _vp, c_size_t, c_double, c_double, c_uint64, c_uint64, _vp]),
    "dc_adam_step": (_i, [_vp, _vp, _vp, _vp, c_size_t, _vp, c_double, c_double, c_double, c_double, c_double, _vp]),
    "dc_ssim_workspace_bytes": (c_size_t, [_i, _i, _i]),
    "dc_ssim": (_i, [_vp, _vp, _i, _i, _i, c_float, _vp, _vp, _vp, c_size_t, _vp]),
}

_LIB = None


def header_symbols(path=HEADER):
    """Names of the functions declared in include/dcfbp.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dc_[a-z0-9_]+)\s*\(", text)))


def lib():
    """The loaded library (loaded once).  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # torch ships its own libamdhip64.so.7; loading it first makes this
        # library bind to the same HIP runtime (same soname) instead of pulling in
        # a second copy from /opt/rocm, which would leave torch without a device.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdcfbp.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def last_error():
    return lib().dc_last_error().decode()


def check(status, where):
    if status != DC_OK:
        raise DcError(status, where, last_error())
