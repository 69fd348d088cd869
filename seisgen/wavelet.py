"""Source signatures (inputs only).

The paper's examples use a Ricker wavelet with a peak frequency and a maximum
amplitude (§2.2.1 parameters ``fpeak``/``amplitude``; §3, Ricker figure).
Sample n of the wavelet belongs to time t_n = n * dt.
"""

from __future__ import annotations

import numpy as np


def ricker(nt: int, dt: float, fpeak: float, t0: float | None = None,
           amplitude: float = 1.0) -> np.ndarray:
    """amplitude * (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0.

    t0 defaults to 1 / fpeak so that the wavelet starts close to zero.
    Returns float32 of length nt; its peak value is ``amplitude`` at t = t0.
    """
    if t0 is None:
        t0 = 1.0 / fpeak
    t = np.arange(nt, dtype=np.float64) * dt
    a = (np.pi * fpeak * (t - t0)) ** 2
    return (amplitude * (1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)
