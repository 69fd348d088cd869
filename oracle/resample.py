"""FP64 oracle of seismic-data time resampling (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product library.

The paper resamples seismic data in time by nearest-neighbour or sinc
interpolation (§2.1).  Reading (R25): a trace of nt samples at step dt has
sample k at time (k + 1) dt (the recorded-trace convention, R10);
  nearest: out[m] = in[n], n = round-half-up(t_m / dt_in) - 1, clamped to the
           trace;
  sinc:    out[m] = sum_n in[n] sinc((t_m - t_n) / dt_in)  (Whittaker-Shannon
           over the whole trace), sinc(x) = sin(pi x) / (pi x).
"""

from __future__ import annotations

import math

import numpy as np


def resample(traces, dt_in: float, nt_out: int, dt_out: float, mode: str) -> np.ndarray:
    d = np.asarray(traces, dtype=np.float64)
    nrec, nt_in = d.shape
    t_out = (np.arange(nt_out) + 1.0) * dt_out
    if mode == "nearest":
        idx = np.array([min(max(math.floor(t / dt_in + 0.5) - 1, 0), nt_in - 1) for t in t_out])
        return d[:, idx]
    if mode == "sinc":
        t_in = (np.arange(nt_in) + 1.0) * dt_in
        kern = np.sinc((t_out[:, None] - t_in[None, :]) / dt_in)   # [nt_out][nt_in]
        return d @ kern.T
    raise ValueError(mode)
