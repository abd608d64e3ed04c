"""MI355X (gfx950) Defrise-Clack shift-variant FBP: HIP kernels behind a C ABI.

The library (libdcfbp.so, built from csrc/ by build.py) implements the four
stages of the paper's eq. 12 and their exact transposes; this package binds
them for torch tensors (``ops``) and wraps the chain as a differentiable
function of the redundancy weight M (``autograd``).  Importing the package
loads the library and fails if it has not been built.
"""
from . import _lib
from ._lib import DcError, header_symbols

_lib.lib()   # fail loudly at import time when the HIP library is missing

from .ops import (Plan, validate, plan_bounds, dc_weight_radon, dc_weight_radon_adjoint, dc_filter,  # noqa: E402
                  dc_filter_adjoint, dc_detector_bp, dc_detector_bp_adjoint, dc_cone_bp,
                  dc_cone_bp_adjoint, dc_smooth_weights, dc_smooth_weights_adjoint, dc_ssim, dc_project,
                  dc_crofton_weights, dc_poisson_noise, dc_adam_step)
from .autograd import DCFBP, reconstruct, sinogram  # noqa: E402
from . import train  # noqa: E402,F401

__all__ = ["Plan", "validate", "plan_bounds", "DcError", "header_symbols", "DCFBP", "reconstruct", "sinogram",
           "dc_weight_radon", "dc_weight_radon_adjoint", "dc_filter", "dc_filter_adjoint",
           "dc_detector_bp", "dc_detector_bp_adjoint", "dc_cone_bp", "dc_cone_bp_adjoint",
           "dc_smooth_weights", "dc_smooth_weights_adjoint", "dc_ssim", "dc_project", "dc_crofton_weights",
           "dc_poisson_noise", "dc_adam_step"]
