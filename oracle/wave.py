"""FP64 CPU oracle for the acoustic finite-difference path (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU library.

What it computes (paper references are to arXiv 2502.12350, "Mamute"):

* Eq. 1 (§2.1): constant density  p_tt = c^2 lap(p) + S  and variable density
  q_tt = c^2 (lap(q) - m^2 q) + S / sqrt(rho),  q = p / sqrt(rho),
  m^2 = lap(sqrt(rho)) / sqrt(rho),  S = f(t) delta(x - x_S).
* §2.1: second order in time, eighth order in space; absorbing boundary by
  damping (Cerjan-style sponge); the grid's sponge thickness is ``border``
  (§2.2.1 parameter table).
* Alg. 3 (§2.2, Adjoint::Run): forward sweep with receiver recording and
  wavefield saving, misfit, backward sweep with wavefield retrieval and the
  cross-correlation imaging condition, then the chain rule to the velocity
  gradient (MultiplyAdjoint) and zeroing of the top planes
  (ZeroesNearSurface).
* §2.2.2: volumes are [z][y][x] with x fastest; positions are metres in
  (x, y, z) order; seismograms are trace-major [rec][ns].

Readings taken where the paper is silent:

R1  8th-order central second-derivative weights (-205/72, 8/5, -1/5, 8/315,
    -1/560).
R2  leapfrog in time.
R3  sponge: g_d[i] = exp(-(0.4 * delta_i / N)^2) per axis, G = gz*gy*gx,
    applied as w^{n+1} = G (A w^n + inj - G w^{n-1}).
R4  the sponge is padded *outside* the model on all six faces with the
    model's edge values replicated into it.
R5  cells beyond the padded grid are zero (Dirichlet).
R7  the point source adds dt^2 f[n] / (hx hy hz sqrt(rho_src)) at its node.
R8  positions map to the nearest node, round half up; outside = error.
R9  recorded quantity: pressure p = sqrt(rho) q.
R10 wavelet sample n <-> t = n dt; trace sample n = w^{n+1} <-> t = (n+1) dt.
R13 m^2 is the same 8th-order Laplacian of sqrt(rho) (edge-replicated 4 more
    cells) divided by sqrt(rho).
R14 J = 1/2 sum (d - d_obs)^2, no dt weight.
R15 the adjoint is the exact discrete transpose of the forward recursion.
R17 the gradient is taken with respect to velocity: dJ/dv = 2 g / v with
    g = k dJ/dk and k = dt^2 v^2 (MultiplyAdjoint read as this chain rule).
R18 gradient cells in the sponge are folded back into the model-edge cells
    they replicate (transpose of R4).
R23 free surface (§2.1, an option that lets the surface reflect waves): a
    pressure-release surface at the top model plane zs.  Planes above it are
    read as the antisymmetric image, w(zs - k) = -w(zs + k) (the image
    method), sqrt(rho) is mirrored evenly about it for m^2, the planes at
    and above it are held at zero, and there is no sponge on that side.  The
    mirrored L is still symmetric, so the adjoint derivation below holds.

Adjoint derivation used here (written out so that it can be checked by eye).
Forward, with A = 2 I - K_m + K L, K = diag(k), K_m = diag(k m^2):
    w^{n+1} = G A w^n - G^2 w^{n-1} + G b_n,          w^0 = w^{-1} = 0.
With e_j = dJ/dw^j (receiver residuals) the Lagrange multipliers obey
    lambda^j = e_j + A^T G lambda^{j+1} - G^2 lambda^{j+2},
and L is symmetric (zero ghosts, or the free surface's antisymmetric image:
its (z, z') entry is c(z' - z) - c(2 zs - z - z'), symmetric in z and z'),
so A^T = 2 I - K_m + L K.  Substituting
psi^j = K G lambda^j gives exactly the forward recursion again:
    psi^j = G (2 psi^{j+1} - K_m psi^{j+1} + K L psi^{j+1} + K e_j - G psi^{j+2}).
Since dA/dk = diag(L w - m^2 w), the gradient is
    k dJ/dk = sum_{n} psi^{n+1} (L w^n - m^2 w^n),  n = 1 .. nt-1.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Eighth-order central weights of d^2/dx^2 (reading R1): a0, a1..a4.
FD8 = (-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)
RADIUS = 4
SPONGE_A = 0.4  # reading R3


# ----------------------------------------------------------------------------
# grid description
# ----------------------------------------------------------------------------
@dataclass
class Grid:
    """Model grid plus sponge (§2.2.1: nx/ny/nz, dx/dy/dz, ox/oy/oz, border, dt, ns)."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    ox: float = 0.0
    oy: float = 0.0
    oz: float = 0.0
    border: int = 0
    dt: float = 1.0e-3
    nt: int = 1
    free_surface: bool = False   # pressure-release surface at the top model plane (R23)

    @property
    def h(self) -> Tuple[float, float, float]:
        return (self.dx, self.dy, self.dz)

    @property
    def zs(self) -> Optional[int]:
        """Padded z index of the free surface (the top model plane), or None."""
        return self.border if self.free_surface else None

    @property
    def padded_shape(self) -> Tuple[int, int, int]:
        b = 2 * self.border
        return (self.nz + b, self.ny + b, self.nx + b)


# ----------------------------------------------------------------------------
# spatial operators
# ----------------------------------------------------------------------------
def second_derivative(u: np.ndarray, axis: int, h: float, periodic: bool = False,
                      mirror_zs: Optional[int] = None) -> np.ndarray:
    """8th-order central d^2u/dx_axis^2 with zero ghosts (R5) or periodic wrap.
    With mirror_zs (axis 0 only), every plane z < mirror_zs, including those
    above the array, reads -u[2 mirror_zs - z] (zero past the array's end):
    the antisymmetric image of a pressure-release surface at plane mirror_zs
    (R23)."""
    pad = [(0, 0)] * u.ndim
    pad[axis] = (RADIUS, RADIUS)
    up = np.pad(u, pad, mode="wrap" if periodic else "constant")
    n = u.shape[axis]
    if mirror_zs is not None and axis == 0:
        for e in range(0, mirror_zs + RADIUS):   # extended index e <-> plane z = e - RADIUS
            z = e - RADIUS
            zm = 2 * mirror_zs - z
            up[e] = -u[zm] if zm < n else 0.0

    def shifted(off):
        sl = [slice(None)] * u.ndim
        sl[axis] = slice(RADIUS + off, RADIUS + off + n)
        return up[tuple(sl)]

    out = FD8[0] * shifted(0)
    for j in range(1, RADIUS + 1):
        out = out + FD8[j] * (shifted(j) + shifted(-j))
    return out / (h * h)


def laplacian(u: np.ndarray, h: Sequence[float], periodic: bool = False,
              mirror_zs: Optional[int] = None) -> np.ndarray:
    """L u = d2/dx2 + d2/dy2 + d2/dz2 on a [z][y][x] array; h = (dx, dy, dz)."""
    dx, dy, dz = h
    return (second_derivative(u, 2, dx, periodic)
            + second_derivative(u, 1, dy, periodic)
            + second_derivative(u, 0, dz, periodic, mirror_zs))


def grid_laplacian(grid: "Grid", u: np.ndarray, periodic: bool = False) -> np.ndarray:
    """L on the padded grid with the grid's top boundary (zero ghosts, or the
    free surface's antisymmetric image)."""
    return laplacian(u, grid.h, periodic, grid.zs)


# ----------------------------------------------------------------------------
# model preparation
# ----------------------------------------------------------------------------
def pad_edge(vol: np.ndarray, n: int) -> np.ndarray:
    """Replicate the edge values ``n`` cells outward on all six faces (R4)."""
    return np.pad(np.asarray(vol, dtype=np.float64), n, mode="edge")


def fold_padding(gp: np.ndarray, n: int) -> np.ndarray:
    """Transpose of ``pad_edge``: add every padding cell into the model cell it
    copies, then crop (R18)."""
    out = np.asarray(gp, dtype=np.float64)
    if n == 0:
        return out.copy()
    for axis in range(3):
        m = out.shape[axis] - 2 * n
        lead = np.take(out, range(0, n + 1), axis=axis).sum(axis=axis, keepdims=True)
        trail = np.take(out, range(n + m - 1, out.shape[axis]), axis=axis).sum(axis=axis, keepdims=True)
        core = np.take(out, range(n, n + m), axis=axis).copy()
        idx_first = [slice(None)] * 3
        idx_first[axis] = slice(0, 1)
        idx_last = [slice(None)] * 3
        idx_last[axis] = slice(m - 1, m)
        if m == 1:
            core[tuple(idx_first)] = lead + trail - np.take(out, [n], axis=axis)
        else:
            core[tuple(idx_first)] = lead
            core[tuple(idx_last)] = trail
        out = core
    return out


def sponge_profile(n: int, border: int, a: float = SPONGE_A, free_top: bool = False) -> np.ndarray:
    """Per-axis damping g[i], i over the padded axis (R3): 1 inside the model,
    exp(-(a * delta / N)^2) at distance delta into the sponge; with free_top
    no damping before the model (the free surface's side, R23)."""
    total = n + 2 * border
    if border == 0:
        return np.ones(total)
    i = np.arange(total)
    before = np.zeros(total, dtype=np.int64) if free_top else border - i
    delta = np.maximum.reduce([before, np.zeros(total, dtype=np.int64), i - (border + n - 1)])
    return np.exp(-(a * delta / border) ** 2)


def sponge(grid: Grid) -> np.ndarray:
    gz = sponge_profile(grid.nz, grid.border, free_top=grid.free_surface)
    gy = sponge_profile(grid.ny, grid.border)
    gx = sponge_profile(grid.nx, grid.border)
    return gz[:, None, None] * gy[None, :, None] * gx[None, None, :]


@dataclass
class Coefficients:
    k: np.ndarray        # dt^2 v^2 on the padded grid
    m2: np.ndarray       # mass term m^2 (zeros for constant density)
    s: np.ndarray        # sqrt(rho) (ones for constant density)
    G: np.ndarray        # sponge
    V: np.ndarray        # padded velocity
    variable_density: bool


def coefficients(grid: Grid, vel: np.ndarray, rho: Optional[np.ndarray] = None) -> Coefficients:
    """Pad v (and rho) and build k = dt^2 V^2, s = sqrt(R), m^2 = L(s)/s (R13)."""
    N = grid.border
    V = pad_edge(vel, N)
    k = (grid.dt * V) ** 2
    if rho is None:
        m2 = np.zeros_like(k)
        s = np.ones_like(k)
    else:
        s_ext = np.sqrt(pad_edge(rho, N + RADIUS))
        if grid.free_surface:  # sqrt(rho) mirrored (even) about the surface, R23
            P = N + RADIUS
            for e in range(P):
                s_ext[e] = s_ext[P + min(P - e, grid.nz - 1)]
        lap_s = laplacian(s_ext, grid.h)
        core = (slice(RADIUS, -RADIUS),) * 3
        s = s_ext[core]
        m2 = lap_s[core] / s
    return Coefficients(k=k, m2=m2, s=s, G=sponge(grid), V=V, variable_density=rho is not None)


def node_index(grid: Grid, xyz) -> Tuple[int, int, int]:
    """Metres (x, y, z) -> padded-grid node (iz, iy, ix): nearest node, round
    half up (R8).  Raises ValueError outside the model."""
    out = []
    for x, o, h, n in zip(xyz, (grid.ox, grid.oy, grid.oz), grid.h, (grid.nx, grid.ny, grid.nz)):
        i = math.floor((x - o) / h + 0.5)
        if i < 0 or i >= n:
            raise ValueError(f"position {tuple(xyz)} outside the model")
        out.append(i + grid.border)
    ix, iy, iz = out
    return (iz, iy, ix)


# ----------------------------------------------------------------------------
# stability (ValidConditions, §2.2 table of Modeling methods)
# ----------------------------------------------------------------------------
def laplacian_symbol_max() -> float:
    """max over wavenumbers of -(a0 + 2 sum a_j cos(j theta)) (at theta = pi), h = 1."""
    return -(FD8[0] + 2.0 * sum(FD8[j] * (-1.0) ** j for j in range(1, RADIUS + 1)))


def cfl_ratio(grid: Grid, vmax: float, m2max: float = 0.0) -> float:
    """dt^2 vmax^2 (Lambda_max + max(m2, 0)) / 4; the scheme is stable when < 1."""
    lam = laplacian_symbol_max() * sum(1.0 / (h * h) for h in grid.h)
    return grid.dt ** 2 * vmax ** 2 * (lam + max(m2max, 0.0)) / 4.0


# ----------------------------------------------------------------------------
# time stepping
# ----------------------------------------------------------------------------
def step(c: Coefficients, grid: Grid, w: np.ndarray, w_prev: np.ndarray,
         inj: Optional[np.ndarray] = None, periodic: bool = False) -> np.ndarray:
    """One leapfrog step: G (2 w - k m2 w + k L w + inj - G w_prev); with a
    free surface the planes at and above it are held at zero (R23)."""
    acc = 2.0 * w - c.k * c.m2 * w + c.k * grid_laplacian(grid, w, periodic)
    if inj is not None:
        acc = acc + inj
    out = c.G * (acc - c.G * w_prev)
    if grid.free_surface:
        out[:grid.zs + 1] = 0.0
    return out


@dataclass
class Geometry:
    src: Tuple[int, int, int]
    rec: List[Tuple[int, int, int]]
    sigma: float          # source scale dt^2 / (hx hy hz s_src)
    rec_scale: np.ndarray  # s at each receiver (pressure = s * q)


def geometry(grid: Grid, c: Coefficients, src_xyz, rec_xyz) -> Geometry:
    src = node_index(grid, src_xyz)
    rec = [node_index(grid, r) for r in np.asarray(rec_xyz, dtype=np.float64).reshape(-1, 3)]
    sigma = grid.dt ** 2 / (grid.dx * grid.dy * grid.dz * c.s[src])
    rec_scale = np.array([c.s[r] for r in rec])
    return Geometry(src=src, rec=rec, sigma=sigma, rec_scale=rec_scale)


def _as64(a, fp32_inputs: bool = True):
    """Inputs as float64; by default first rounded to float32 (what the GPU sees)."""
    if a is None:
        return None
    if fp32_inputs:
        return np.asarray(a, dtype=np.float32).astype(np.float64)
    return np.asarray(a, dtype=np.float64)


@dataclass
class ForwardResult:
    seis: np.ndarray                    # [nrec][nt]
    last: np.ndarray                    # w^nt
    prev: np.ndarray                    # w^(nt-1)
    states: Optional[List[np.ndarray]]  # w^0 .. w^nt if requested
    illum: Optional[np.ndarray]         # sum_{n=1..nt} (w^n)^2 on the model grid


def forward(grid: Grid, vel, rho, wavelet, src_xyz, rec_xyz, *,
            keep_states: bool = False, illumination: bool = False,
            w0: Optional[np.ndarray] = None, w_m1: Optional[np.ndarray] = None,
            periodic: bool = False, coefs: Optional[Coefficients] = None,
            fp32_inputs: bool = True) -> ForwardResult:
    """Forward modeling (Alg. 1 / forward half of Alg. 3).

    Inputs are rounded to float32 and then used in float64, so the oracle sees
    exactly the values the GPU sees.  w0 / w_m1 override the zero initial
    states (used only by eigenmode tests).
    """
    c = coefs if coefs is not None else coefficients(
        grid, _as64(vel, fp32_inputs), _as64(rho, fp32_inputs))
    geo = geometry(grid, c, src_xyz, rec_xyz)
    f = _as64(wavelet, fp32_inputs)
    shape = grid.padded_shape
    w_prev = np.zeros(shape) if w_m1 is None else np.array(w_m1, dtype=np.float64)
    w = np.zeros(shape) if w0 is None else np.array(w0, dtype=np.float64)
    nrec = len(geo.rec)
    seis = np.zeros((nrec, grid.nt))
    states = [w.copy()] if keep_states else None
    illum = np.zeros(shape) if illumination else None
    inj = np.zeros(shape)
    for n in range(grid.nt):
        inj[geo.src] = geo.sigma * f[n]
        w_new = step(c, grid, w, w_prev, inj, periodic)
        inj[geo.src] = 0.0
        for r, node in enumerate(geo.rec):
            seis[r, n] = geo.rec_scale[r] * w_new[node]
        if illum is not None:
            illum += w_new * w_new
        if keep_states:
            states.append(w_new.copy())
        w_prev, w = w, w_new
    if illum is not None:
        N = grid.border
        illum = illum[N:N + grid.nz, N:N + grid.ny, N:N + grid.nx] if N else illum
    return ForwardResult(seis=seis, last=w, prev=w_prev, states=states, illum=illum)


def misfit(seis: np.ndarray, dobs: np.ndarray, fp32_inputs: bool = True) -> Tuple[float, np.ndarray]:
    """res = d - d_obs and J = 1/2 sum res^2 (SeismicData::Misfit, R14)."""
    res = np.asarray(seis, dtype=np.float64) - _as64(dobs, fp32_inputs)
    return 0.5 * float(np.sum(res * res)), res


def _receiver_injection(shape, geo: Geometry, c: Coefficients, res_col: np.ndarray) -> np.ndarray:
    """sum_r k_r s_r res[r] delta_r (duplicates add)."""
    inj = np.zeros(shape)
    for r, node in enumerate(geo.rec):
        inj[node] += c.k[node] * geo.rec_scale[r] * res_col[r]
    return inj


@dataclass
class GradientResult:
    misfit: float
    grad: np.ndarray          # dJ/dv on the model grid (after fold and zeroing)
    grad_padded: np.ndarray   # dJ/dV on the padded grid (before fold)
    g: np.ndarray             # k dJ/dk on the padded grid
    seis: np.ndarray
    illum: Optional[np.ndarray]
    psi_src: Optional[np.ndarray]  # psi^m at the source node, m = 1..nt


def _segment_states(c, grid, geo, f, K):
    """Forward sweep that keeps every K-th leapfrog pair (w^m, w^{m-1})."""
    shape = grid.padded_shape
    w_prev, w = np.zeros(shape), np.zeros(shape)
    nrec = len(geo.rec)
    seis = np.zeros((nrec, grid.nt))
    keep = {0: (w.copy(), w_prev.copy())}
    inj = np.zeros(shape)
    for n in range(grid.nt):
        inj[geo.src] = geo.sigma * f[n]
        w_new = step(c, grid, w, w_prev, inj)
        inj[geo.src] = 0.0
        for r, node in enumerate(geo.rec):
            seis[r, n] = geo.rec_scale[r] * w_new[node]
        w_prev, w = w, w_new
        if (n + 1) % K == 0:
            keep[n + 1] = (w.copy(), w_prev.copy())
    return seis, keep, (w, w_prev)


def _segment(c, grid, geo, f, keep, m0, m1):
    """States w^{m0} .. w^{m1-1}, recomputed from the pair stored at m0."""
    w, w_prev = (a.copy() for a in keep[m0])
    out = [w.copy()]
    inj = np.zeros(grid.padded_shape)
    for n in range(m0, m1 - 1):
        inj[geo.src] = geo.sigma * f[n]
        w_new = step(c, grid, w, w_prev, inj)
        inj[geo.src] = 0.0
        w_prev, w = w, w_new
        out.append(w.copy())
    return out


def gradient(grid: Grid, vel, rho, wavelet, src_xyz, rec_xyz, dobs, *,
             zero_top_planes: int = 0, illumination: bool = False,
             record_source: bool = False, segment: Optional[int] = None,
             fp32_inputs: bool = True) -> GradientResult:
    """Misfit and velocity gradient of one shot (Alg. 3 for a single shot).

    The backward sweep needs w^m in reverse order; the forward states are kept
    by plain segment checkpointing (every K-th pair stored, each K-step segment
    recomputed once), K = ceil(sqrt(nt)) unless given.
    """
    c = coefficients(grid, _as64(vel, fp32_inputs), _as64(rho, fp32_inputs))
    geo = geometry(grid, c, src_xyz, rec_xyz)
    f = _as64(wavelet, fp32_inputs)
    nt = grid.nt
    K = segment or max(1, int(math.ceil(math.sqrt(nt))))
    seis, keep, (w_last, _) = _segment_states(c, grid, geo, f, K)
    J, res = misfit(seis, dobs, fp32_inputs)

    shape = grid.padded_shape
    psi1 = np.zeros(shape)   # psi^{m+1}
    psi2 = np.zeros(shape)   # psi^{m+2}
    g = np.zeros(shape)
    illum = np.zeros(shape) if illumination else None
    psi_src = np.zeros(nt) if record_source else None
    if illum is not None:
        illum += w_last * w_last
    seg_states = {}
    for m in range(nt, 0, -1):
        inj = _receiver_injection(shape, geo, c, res[:, m - 1])
        psi = step(c, grid, psi1, psi2, inj)
        if m < nt:
            # w^m, from the segment that contains it
            m0 = (m // K) * K
            if m0 not in seg_states:
                seg_states = {m0: _segment(c, grid, geo, f, keep, m0, min(m0 + K, nt + 1))}
            wm = seg_states[m0][m - m0]
            g += psi1 * (grid_laplacian(grid, wm) - c.m2 * wm)
            if illum is not None:
                illum += wm * wm
        if psi_src is not None:
            psi_src[m - 1] = psi[geo.src]
        psi2, psi1 = psi1, psi
    grad_padded = 2.0 * g / c.V
    grad = fold_padding(grad_padded, grid.border)
    if zero_top_planes > 0:
        grad[:zero_top_planes] = 0.0
    if illum is not None and grid.border:
        N = grid.border
        illum = illum[N:N + grid.nz, N:N + grid.ny, N:N + grid.nx]
    return GradientResult(misfit=J, grad=grad, grad_padded=grad_padded, g=g, seis=seis,
                          illum=illum, psi_src=psi_src)


def adjoint_source_transpose(grid: Grid, vel, rho, src_xyz, rec_xyz, dprime,
                             fp32_inputs: bool = True) -> np.ndarray:
    """F^T d' for the linear map F: wavelet -> data (fixed model).

    dJ/df[n] = sigma * G_src lambda^{n+1}[src] = sigma * psi^{n+1}[src] / k_src.
    """
    c = coefficients(grid, _as64(vel, fp32_inputs), _as64(rho, fp32_inputs))
    geo = geometry(grid, c, src_xyz, rec_xyz)
    d = np.asarray(dprime, dtype=np.float64)
    shape = grid.padded_shape
    psi1 = np.zeros(shape)
    psi2 = np.zeros(shape)
    out = np.zeros(grid.nt)
    for m in range(grid.nt, 0, -1):
        inj = _receiver_injection(shape, geo, c, d[:, m - 1])
        psi = step(c, grid, psi1, psi2, inj)
        out[m - 1] = geo.sigma * psi[geo.src] / c.k[geo.src]
        psi2, psi1 = psi1, psi
    return out


def energy(c: Coefficients, grid: Grid, w_new: np.ndarray, w: np.ndarray) -> float:
    """Discrete energy E^{n+1/2} = 1/2 sum (w^{n+1}-w^n)^2 / k
    + 1/2 sum w^{n+1} (-L + m^2) w^n  (conserved without sponge and source)."""
    dw = w_new - w
    kin = 0.5 * np.sum(dw * dw / c.k)
    pot = 0.5 * np.sum(w_new * (-grid_laplacian(grid, w) + c.m2 * w))
    return float(kin + pot)


def illumination_gradient(grad: np.ndarray, illum: np.ndarray, eps: float = 1.0e-3) -> np.ndarray:
    """Illumination-compensated gradient g / (I + eps * max I)."""
    return grad / (illum + eps * float(np.max(illum)))
