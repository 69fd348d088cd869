"""Seeded synthetic inputs for the acoustic finite-difference path.

This package only *generates inputs*: velocity and density volumes, source
wavelets and acquisition geometries.  It contains none of the propagation,
misfit, adjoint or gradient arithmetic, so both the FP64 CPU oracle and the
GPU library can be fed from it without sharing any of the method's code.

Conventions shared with the rest of the repository (paper §2.2.2, data
format): volumes are C-order ``[z][y][x]`` with x fastest, positions are
metres in ``(x, y, z)`` order, seismograms are trace-major ``[rec][ns]``.
"""

from .models import layered_model, gardner_density, blob_anomalies, smooth_noise
from .wavelet import ricker
from .configs import Workload, workload, WORKLOADS, shot_window, c5_model

__all__ = [
    "layered_model",
    "gardner_density",
    "blob_anomalies",
    "smooth_noise",
    "ricker",
    "Workload",
    "workload",
    "WORKLOADS",
    "shot_window",
    "c5_model",
]
