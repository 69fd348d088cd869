"""FP64 oracle of the CPML absorbing boundary (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product library.
It shares no code with the GPU path.

The paper offers two absorbing boundaries (§2.1): damping (the sponge of
oracle/wave.py) and the convolutional perfectly matched layer of Roden and
Gedney (2000), in a layer ``border`` cells thick.  It gives no formulas; the
reading (R26) is:

* Stretched coordinates.  In the layer each second derivative becomes
  d/dx~ (d/dx~ w) with d/dx~ = (1/s) d/dx and s = 1 + d(x)/(alpha(x) + i omega)
  (the complex-frequency-shifted stretch, kappa = 1).  Multiplying by 1/s is
  a convolution in time, done recursively (Roden and Gedney's recursive
  convolution): for a field f, (1/s) f = f + psi with
      psi^n = b psi^{n-1} + a f^n,   b = exp(-(d + alpha) dt),
      a = d (b - 1) / (d + alpha)    (a = 0 where d = 0).
  Applied twice, per axis d:
      psi_d^n  = b_d psi_d^{n-1}  + a_d D1_d w^n
      zeta_d^n = b_d zeta_d^{n-1} + a_d (D2_d w^n + D1_d psi_d^n)
      d2w/dx~_d^2 = D2_d w^n + D1_d psi_d^n + zeta_d^n
  with D2 the eighth-order second difference of L and D1 the eighth-order
  central first difference (4/5, -1/5, 4/105, -1/280), zero outside the grid.
  So L is replaced by L + C with the correction C^n = sum_d (D1_d psi_d^n +
  zeta_d^n), and the leapfrog step becomes (no sponge multiply)
      w^{n+1} = 2 w^n - k m^2 w^n + k (L w^n + C^n) + inj^n - w^{n-1}.
* Profiles.  delta = distance into the layer in cells (as for the sponge; no
  layer on the free-surface side), N = border:
      d(delta)     = d0 (delta / N)^2,  d0 = -3 vmax ln(R0) / (2 N h),
      alpha(delta) = pi fpeak (1 - delta / N) inside the layer,
  R0 = 1e-3 the nominal reflection coefficient, vmax the largest velocity
  (a fixed parameter of the boundary, not differentiated), fpeak the
  source's peak frequency (0 gives the plain PML, alpha = 0).
* Free surface.  As in wave.py (R23): the planes at and above it are held at
  zero after the step; there is no layer on that side.

Adjoint (exact transpose; checked by the dot test).  With lambda the
multiplier of w, mu_d of psi_d, nu_d of zeta_d, and phi = k lambda:
      nu_d^n  = phi^{n+1} + b_d nu_d^{n+1}
      mu_d^n  = b_d mu_d^{n+1} - D1_d (a_d nu_d^n + phi^{n+1})
      phi^n   = 2 phi^{n+1} - k m^2 phi^{n+1} + k L phi^{n+1} - phi^{n+2}
                + k sum_d [D2_d (a_d nu_d^n) - D1_d (a_d mu_d^n)] + k e_n,
using D1^T = -D1 and D2^T = D2 (zero ghosts), and the held-zero planes as a
projection applied to every new phi.  The imaging condition is
      g = k dJ/dk = sum_{n=1}^{nt-1} phi^{n+1} (L w^n - m^2 w^n + C^n),
so the forward correction C^n is kept for the backward sweep.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

from . import wave

# Eighth-order central first-difference weights c1..c4 (c_-j = -c_j).
FD1 = (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0)
R0 = 1.0e-3


def first_derivative(u: np.ndarray, axis: int, h: float) -> np.ndarray:
    """Eighth-order central du/dx_axis with zero ghosts."""
    pad = [(0, 0)] * u.ndim
    pad[axis] = (wave.RADIUS, wave.RADIUS)
    up = np.pad(u, pad)
    n = u.shape[axis]

    def shifted(off):
        sl = [slice(None)] * u.ndim
        sl[axis] = slice(wave.RADIUS + off, wave.RADIUS + off + n)
        return up[tuple(sl)]

    out = np.zeros_like(u, dtype=np.float64)
    for j in range(1, wave.RADIUS + 1):
        out = out + FD1[j - 1] * (shifted(j) - shifted(-j))
    return out / h


def layer_depth(n: int, border: int, free_top: bool = False) -> np.ndarray:
    """delta_i: cells into the layer along one padded axis (0 in the model)."""
    i = np.arange(n + 2 * border)
    before = np.zeros_like(i) if free_top else border - i
    return np.maximum.reduce([before, np.zeros_like(i), i - (border + n - 1)])


def profile(n: int, border: int, h: float, dt: float, vmax: float, fpeak: float,
            free_top: bool = False, r0: float = R0) -> Tuple[np.ndarray, np.ndarray]:
    """Recursive-convolution coefficients (a, b) along one padded axis (R26)."""
    delta = layer_depth(n, border, free_top).astype(np.float64)
    if border == 0:
        return np.zeros(n), np.ones(n)
    d0 = -3.0 * vmax * math.log(r0) / (2.0 * border * h)
    d = d0 * (delta / border) ** 2
    alpha = np.where(delta > 0, math.pi * fpeak * (1.0 - delta / border), 0.0)
    b = np.exp(-(d + alpha) * dt)
    a = np.where(d > 0, d * (b - 1.0) / np.where(d + alpha > 0, d + alpha, 1.0), 0.0)
    return a, b


@dataclass
class Layer:
    a: List[np.ndarray]   # per axis (x, y, z), broadcastable to [z][y][x]
    b: List[np.ndarray]
    h: Tuple[float, float, float]
    axes: Tuple[int, int, int] = (2, 1, 0)   # array axis of x, y, z


def layer(grid: wave.Grid, vmax: float, fpeak: float, r0: float = R0) -> Layer:
    ax, bx = profile(grid.nx, grid.border, grid.dx, grid.dt, vmax, fpeak, r0=r0)
    ay, by = profile(grid.ny, grid.border, grid.dy, grid.dt, vmax, fpeak, r0=r0)
    az, bz = profile(grid.nz, grid.border, grid.dz, grid.dt, vmax, fpeak,
                     free_top=grid.free_surface, r0=r0)
    return Layer(a=[ax[None, None, :], ay[None, :, None], az[:, None, None]],
                 b=[bx[None, None, :], by[None, :, None], bz[:, None, None]],
                 h=grid.h)


def _d2(grid: wave.Grid, u: np.ndarray, d: int, h: float) -> np.ndarray:
    axis = (2, 1, 0)[d]
    return wave.second_derivative(u, axis, h, mirror_zs=grid.zs if axis == 0 else None)


def _d1(u: np.ndarray, d: int, h: float) -> np.ndarray:
    return first_derivative(u, (2, 1, 0)[d], h)


def _hold(grid: wave.Grid, u: np.ndarray) -> np.ndarray:
    if grid.free_surface:
        u[:grid.zs + 1] = 0.0
    return u


def forward_step(c: wave.Coefficients, grid: wave.Grid, lay: Layer, w, w_prev, inj,
                 psi: List[np.ndarray], zeta: List[np.ndarray]):
    """One CPML leapfrog step; updates psi/zeta in place, returns (w^{n+1}, C^n)."""
    C = np.zeros_like(w)
    for d in range(3):
        h = lay.h[d]
        psi[d] = lay.b[d] * psi[d] + lay.a[d] * _d1(w, d, h)
        d1psi = _d1(psi[d], d, h)
        zeta[d] = lay.b[d] * zeta[d] + lay.a[d] * (_d2(grid, w, d, h) + d1psi)
        C += d1psi + zeta[d]
    acc = 2.0 * w - c.k * c.m2 * w + c.k * (wave.grid_laplacian(grid, w) + C) + inj
    return _hold(grid, acc - w_prev), C


def adjoint_step(c: wave.Coefficients, grid: wave.Grid, lay: Layer, phi1, phi2, inj,
                 mu: List[np.ndarray], nu: List[np.ndarray]):
    """phi^m from phi^{m+1}, phi^{m+2}; updates mu/nu (m+1 -> m) in place."""
    corr = np.zeros_like(phi1)
    for d in range(3):
        h = lay.h[d]
        nu[d] = phi1 + lay.b[d] * nu[d]
        mu[d] = lay.b[d] * mu[d] - _d1(lay.a[d] * nu[d] + phi1, d, h)
        corr += _d2(grid, lay.a[d] * nu[d], d, h) - _d1(lay.a[d] * mu[d], d, h)
    acc = (2.0 * phi1 - c.k * c.m2 * phi1 + c.k * wave.grid_laplacian(grid, phi1)
           + c.k * corr + inj)
    return _hold(grid, acc - phi2)


@dataclass
class CpmlForward:
    seis: np.ndarray
    last: np.ndarray
    prev: np.ndarray
    states: Optional[List[np.ndarray]]   # w^0 .. w^nt
    corr: Optional[List[np.ndarray]]     # C^0 .. C^{nt-1}


def forward(grid: wave.Grid, vel, rho, wavelet, src_xyz, rec_xyz, *, vmax: float,
            fpeak: float, r0: float = R0, keep_states: bool = False,
            fp32_inputs: bool = True) -> CpmlForward:
    """Forward modelling with the CPML boundary (Alg. 1 with R26)."""
    c = wave.coefficients(grid, wave._as64(vel, fp32_inputs), wave._as64(rho, fp32_inputs))
    lay = layer(grid, vmax, fpeak, r0)
    geo = wave.geometry(grid, c, src_xyz, rec_xyz)
    f = wave._as64(wavelet, fp32_inputs)
    shape = grid.padded_shape
    w_prev, w = np.zeros(shape), np.zeros(shape)
    psi = [np.zeros(shape) for _ in range(3)]
    zeta = [np.zeros(shape) for _ in range(3)]
    seis = np.zeros((len(geo.rec), grid.nt))
    states = [w.copy()] if keep_states else None
    corr = [] if keep_states else None
    inj = np.zeros(shape)
    for n in range(grid.nt):
        inj[geo.src] = geo.sigma * f[n]
        w_new, C = forward_step(c, grid, lay, w, w_prev, inj, psi, zeta)
        inj[geo.src] = 0.0
        for r, node in enumerate(geo.rec):
            seis[r, n] = geo.rec_scale[r] * w_new[node]
        if keep_states:
            states.append(w_new.copy())
            corr.append(C)
        w_prev, w = w, w_new
    return CpmlForward(seis=seis, last=w, prev=w_prev, states=states, corr=corr)


def gradient(grid: wave.Grid, vel, rho, wavelet, src_xyz, rec_xyz, dobs, *, vmax: float,
             fpeak: float, r0: float = R0, illumination: bool = False,
             fp32_inputs: bool = True) -> wave.GradientResult:
    """Misfit and dJ/dv with the CPML boundary (Alg. 3 with R26): every forward
    state and correction is kept (small grids only)."""
    c = wave.coefficients(grid, wave._as64(vel, fp32_inputs), wave._as64(rho, fp32_inputs))
    lay = layer(grid, vmax, fpeak, r0)
    geo = wave.geometry(grid, c, src_xyz, rec_xyz)
    fw = forward(grid, vel, rho, wavelet, src_xyz, rec_xyz, vmax=vmax, fpeak=fpeak, r0=r0,
                 keep_states=True, fp32_inputs=fp32_inputs)
    J, res = wave.misfit(fw.seis, dobs, fp32_inputs)
    shape = grid.padded_shape
    phi1, phi2 = np.zeros(shape), np.zeros(shape)
    mu = [np.zeros(shape) for _ in range(3)]
    nu = [np.zeros(shape) for _ in range(3)]
    g = np.zeros(shape)
    illum = np.zeros(shape) if illumination else None
    for m in range(grid.nt, 0, -1):
        inj = wave._receiver_injection(shape, geo, c, res[:, m - 1])
        phi = adjoint_step(c, grid, lay, phi1, phi2, inj, mu, nu)
        wm = fw.states[m]
        if m < grid.nt:
            g += phi1 * (wave.grid_laplacian(grid, wm) - c.m2 * wm + fw.corr[m])
        if illum is not None:
            illum += wm * wm
        phi2, phi1 = phi1, phi
    grad_padded = 2.0 * g / c.V
    grad = wave.fold_padding(grad_padded, grid.border)
    if illum is not None and grid.border:
        N = grid.border
        illum = illum[N:N + grid.nz, N:N + grid.ny, N:N + grid.nx]
    return wave.GradientResult(misfit=J, grad=grad, grad_padded=grad_padded, g=g, seis=fw.seis,
                               illum=illum, psi_src=None)


def adjoint_source_transpose(grid: wave.Grid, vel, rho, src_xyz, rec_xyz, dprime, *,
                             vmax: float, fpeak: float, r0: float = R0,
                             fp32_inputs: bool = True) -> np.ndarray:
    """F^T d' for F: wavelet -> data with the CPML boundary:
    dJ/df[n] = sigma lambda^{n+1}[src] = sigma phi^{n+1}[src] / k_src."""
    c = wave.coefficients(grid, wave._as64(vel, fp32_inputs), wave._as64(rho, fp32_inputs))
    lay = layer(grid, vmax, fpeak, r0)
    geo = wave.geometry(grid, c, src_xyz, rec_xyz)
    d = np.asarray(dprime, dtype=np.float64)
    shape = grid.padded_shape
    phi1, phi2 = np.zeros(shape), np.zeros(shape)
    mu = [np.zeros(shape) for _ in range(3)]
    nu = [np.zeros(shape) for _ in range(3)]
    out = np.zeros(grid.nt)
    for m in range(grid.nt, 0, -1):
        inj = wave._receiver_injection(shape, geo, c, d[:, m - 1])
        phi = adjoint_step(c, grid, lay, phi1, phi2, inj, mu, nu)
        out[m - 1] = geo.sigma * phi[geo.src] / c.k[geo.src]
        phi2, phi1 = phi1, phi
    return out
