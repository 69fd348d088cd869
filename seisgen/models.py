"""Synthetic velocity / density volumes (inputs only, no propagation arithmetic).

The paper works with synthetic models only (constant, sphere, sphere with a
Gaussian perturbation, and Gardner density; §2.2.2 and §3).  The generators
here follow the same spirit at the sizes of the benchmark workloads:

* ``layered_model`` — 8 flat layers whose velocities grow with depth from
  1500 to 4500 m/s, Gaussian-smoothed, times (1 + p) with p a smooth seeded
  random field of prescribed peak amplitude, clipped to [1500, 4500] m/s.
* ``gardner_density`` — rho = 310 * v**0.25 (Gardner's relation, cited in
  §2.2.2 for the density script).
* ``blob_anomalies`` — smooth Gaussian blobs of +/- a few percent on top of a
  background (the FWI "true model").

Every volume is returned as float32, C-order ``[z][y][x]``.
"""

from __future__ import annotations

import numpy as np
from scipy import ndimage

VMIN = 1500.0
VMAX = 4500.0
N_LAYERS = 8


def _shape3(n):
    """Accept an int (cube) or an (nx, ny, nz) tuple; return (nz, ny, nx)."""
    if np.isscalar(n):
        n = int(n)
        return (n, n, n)
    nx, ny, nz = (int(v) for v in n)
    return (nz, ny, nx)


def _interfaces(rng: np.random.Generator, nz: int, n_if: int) -> np.ndarray:
    """Sorted interface depths (cells) with a minimum spacing.

    The spacing is 16 cells when the model is deep enough, else nz // (n_if + 2)
    so that small test models still hold all eight layers.
    """
    gap = max(1, min(16, nz // (n_if + 2)))
    lo, hi = gap, nz - gap
    for _ in range(10000):
        d = np.sort(rng.integers(lo, hi + 1, size=n_if))
        if np.all(np.diff(d) >= gap):
            return d
    # deterministic fallback: even spacing
    return np.linspace(lo, hi, n_if).round().astype(np.int64)


def layered_model(seed: int, n, sigma_p: float) -> np.ndarray:
    """Smooth layered velocity model with seeded multiplicative perturbation.

    Parameters
    ----------
    seed : int      numpy Generator seed.
    n    : int or (nx, ny, nz)
    sigma_p : float peak |p| of the smooth perturbation field (0 disables it).
    """
    nz, ny, nx = _shape3(n)
    rng = np.random.default_rng(seed)
    depths = _interfaces(rng, nz, N_LAYERS - 1)
    layer_v = np.linspace(VMIN, VMAX, N_LAYERS)
    z = np.arange(nz)
    layer_of_z = np.searchsorted(depths, z, side="right")
    prof = layer_v[layer_of_z].astype(np.float64)
    prof = ndimage.gaussian_filter1d(prof, sigma=3.0, mode="nearest")
    v = np.broadcast_to(prof[:, None, None], (nz, ny, nx)).astype(np.float32)
    if sigma_p > 0:
        p = smooth_noise((nx, ny, nz), rng, sigma=8.0, max_abs=sigma_p)
        v = v * (np.float32(1.0) + p)
    np.clip(v, VMIN, VMAX, out=v)
    return np.ascontiguousarray(v, dtype=np.float32)


def smooth_noise(n, rng, sigma: float, max_abs: float) -> np.ndarray:
    """Standard-normal noise, Gaussian-smoothed, rescaled to max|p| = max_abs.

    ``rng`` may be a Generator or an int seed.  Returns float32 [z][y][x].
    """
    if not isinstance(rng, np.random.Generator):
        rng = np.random.default_rng(rng)
    shape = _shape3(n)
    p = rng.standard_normal(shape, dtype=np.float32)
    p = ndimage.gaussian_filter(p, sigma=sigma, mode="nearest", output=np.float32)
    peak = float(np.max(np.abs(p)))
    if peak > 0:
        p *= np.float32(max_abs / peak)
    return p


def gardner_density(v: np.ndarray) -> np.ndarray:
    """rho = 310 * v**0.25 (kg/m^3 with v in m/s); float32."""
    v64 = np.asarray(v, dtype=np.float64)
    return (310.0 * v64 ** 0.25).astype(np.float32)


def blob_anomalies(background: np.ndarray, seed: int, n_blobs: int, amp: float,
                   sigma_cells=(6.0, 12.0), centre_lo=(40, 40, 40),
                   centre_hi=(160, 160, 130)) -> np.ndarray:
    """background * (1 + sum_b A_b exp(-|x - c_b|^2 / (2 sigma_b^2))).

    A_b = +/- amp with a seeded sign; sigma_b uniform in ``sigma_cells``;
    centres c_b uniform in the (x, y, z) box [centre_lo, centre_hi] (cells).
    """
    bg = np.asarray(background, dtype=np.float32)
    nz, ny, nx = bg.shape
    rng = np.random.default_rng(seed)
    signs = rng.choice(np.array([-1.0, 1.0]), size=n_blobs)
    sig = rng.uniform(sigma_cells[0], sigma_cells[1], size=n_blobs)
    cx = rng.uniform(centre_lo[0], centre_hi[0], size=n_blobs)
    cy = rng.uniform(centre_lo[1], centre_hi[1], size=n_blobs)
    cz = rng.uniform(centre_lo[2], centre_hi[2], size=n_blobs)
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    pert = np.zeros((nz, ny, nx), dtype=np.float64)
    for b in range(n_blobs):
        r2 = (x - cx[b]) ** 2 + (y - cy[b]) ** 2 + (z - cz[b]) ** 2
        pert += amp * signs[b] * np.exp(-r2 / (2.0 * sig[b] ** 2))
    return (bg.astype(np.float64) * (1.0 + pert)).astype(np.float32)
