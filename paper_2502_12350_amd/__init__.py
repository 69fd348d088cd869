"""MI355X-native acoustic finite-difference library (arXiv 2502.12350 hot path).

Forward modeling, the discrete adjoint and the FWI velocity gradient of the
3-D acoustic wave equation (constant or variable density), eighth order in
space and second order in time, as hand-written HIP kernels for gfx950
behind a C ABI (include/wfd.h).  PyTorch supplies device memory and streams.
"""

from ._lib import (WfdError, LIB_PATH, CKPT_FULL, CKPT_REVOLVE, CKPT_HOST, K_FORWARD, K_ADJOINT,
                   K_OTHER)
from .api import (GridSpec, Propagator, ShotBatch, GradientBatch, smooth, resample, map_position,
                  cfl_ratio, checkpoint_plan, model_bytes)

__all__ = ["WfdError", "LIB_PATH", "CKPT_FULL", "CKPT_REVOLVE", "CKPT_HOST", "K_FORWARD",
           "K_ADJOINT", "K_OTHER", "GridSpec", "Propagator", "ShotBatch", "GradientBatch", "smooth",
           "resample",
           "map_position", "cfl_ratio", "checkpoint_plan", "model_bytes"]
