"""Named synthetic workloads (inputs only).

Each workload fixes a model grid, the sponge width, dt, nt, a Ricker source
and an acquisition geometry.  Positions are produced in metres, (x, y, z)
order, from integer node indices: x = ox + i * dx (§2.2.2: coordinates in
metres, one (x, y, z) triple per source / receiver).

Workloads
---------
c1        64^3 constant velocity 2000 m/s, 8-cell sponge, 200 steps, 15 Hz,
          64 receivers on a line at depth index 4 (plain forward, constant
          density).
c1_long   c1 with 400 steps (the direct wave peak reaches the receivers
          after 0.2 s).
c2        512^3 layered model with +/-5 % smooth perturbation, Gardner
          density, 32-cell sponge, dt from Courant 0.4 at 4500 m/s, 2000
          steps, 10 Hz, 256 x 256 receiver grid (plain forward, variable
          density).
c2_small  the same generator on a small ragged grid (93 x 77 x 61, 16-cell
          sponge, 300 steps) for element-wise parity; extra["v_true"] adds
          three +/-8 % blobs to a 3 % faster background (the observed-data
          model of gradient parity).
c2_crop   a 128^3 crop of the c2 model (x, y in [192, 320), z in [0, 128)),
          c2's sponge, dt, wavelet, source node and receivers inside the crop,
          500 steps (element-wise parity on the c2 model itself).
c3        400 x 400 x 256 model from the c2 generator (seed 2503), 32-cell
          sponge, 1500 steps, 24 shots on a 6 x 4 surface grid at depth
          index 4; shot i runs on its own aperture window: a square in x-y of
          side s_i drawn from integers(160, 321) (seed 3), centred on the shot,
          clipped to the model, full depth, with receivers at every 2nd
          surface node of the window (depth index 2) (batched multi-shot).
c3_small  the same recipe on 96 x 80 x 48 with 4 shots (2 x 2), sides from
          integers(24, 49), 8-cell sponge, 250 steps (element-wise parity).
c3_narrow the same recipe with narrow apertures: 288 x 192 x 64, 24 shots
          (6 x 4), sides from integers(32, 65), 8-cell sponge, 500 steps
          (windows too small to fill the device on their own).
c4        200 x 200 x 160 smooth layered background + six +/-10 % blobs,
          20-cell sponge, 1200 steps, 8 shots, 2500 receivers (FWI gradient).
c4_fd     32^3 layered model, 8-cell sponge, 300 steps, one shot, 64
          receivers, plus a smooth 1 % velocity perturbation direction for
          finite-difference gradient checks.
c5_train  (function c5_model(seed)) training models of the learned
          preconditioner: 128^3 layered background L(seed, 0), 1-4 blobs of
          +/-10 % (sigma 4-10 cells) away from the faces, 16-cell sponge,
          1000 steps, 10 Hz, 4 shots at depth 4 on a 2 x 2 grid, 32 x 32
          receivers at depth 2; start model = background.
c5_eval   the same recipe at 256^3 (seed 5999), 20-cell sponge, 1600
          steps, 8 shots, 64 x 64 receivers.
example   the paper's illustrative 25^3 setup (§3): h = 10 m, border 25,
          500 steps, dt = 1 ms, 10 Hz Ricker with amplitude 1e5, Gaussian
          velocity blob.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from .models import layered_model, gardner_density, blob_anomalies, smooth_noise
from .wavelet import ricker


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    ox: float
    oy: float
    oz: float
    border: int
    dt: float
    nt: int
    vel: np.ndarray                      # float32 [nz][ny][nx]
    rho: Optional[np.ndarray]            # float32 [nz][ny][nx] or None
    wavelet: np.ndarray                  # float32 [nt]
    sources: np.ndarray                  # float64 [nshot][3] metres (x, y, z)
    receivers: np.ndarray                # float64 [nrec][3] metres (x, y, z)
    extra: Dict[str, np.ndarray] = field(default_factory=dict)

    @property
    def padded_shape(self):
        """(Nz, Ny, Nx) of the grid with the sponge added on every face."""
        b = 2 * self.border
        return (self.nz + b, self.ny + b, self.nx + b)

    @property
    def padded_points(self) -> int:
        nz, ny, nx = self.padded_shape
        return nz * ny * nx

    def grid_kwargs(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, dx=self.dx, dy=self.dy,
                    dz=self.dz, ox=self.ox, oy=self.oy, oz=self.oz,
                    border=self.border, dt=self.dt, nt=self.nt)

    def nodes_to_metres(self, nodes) -> np.ndarray:
        nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, 3)
        o = np.array([self.ox, self.oy, self.oz])
        h = np.array([self.dx, self.dy, self.dz])
        return o + nodes * h


def _metres(nodes, h, o=(0.0, 0.0, 0.0)) -> np.ndarray:
    nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, 3)
    return np.asarray(o, dtype=np.float64) + nodes * np.asarray(h, dtype=np.float64)


def _surface_grid(i0, di, ni, j0, dj, nj, z) -> np.ndarray:
    ii, jj = np.meshgrid(i0 + di * np.arange(ni), j0 + dj * np.arange(nj), indexing="xy")
    return np.stack([ii.ravel(), jj.ravel(), np.full(ii.size, z)], axis=1)


def _c1(nt: int = 200) -> Workload:
    n, h = 64, 10.0
    vel = np.full((n, n, n), 2000.0, dtype=np.float32)
    rec_nodes = np.stack([np.arange(64), np.full(64, 32), np.full(64, 4)], axis=1)
    return Workload("c1" if nt == 200 else f"c1_nt{nt}", n, n, n, h, h, h, 0.0, 0.0, 0.0,
                    8, 1.0e-3, nt, vel, None,
                    ricker(nt, 1.0e-3, 15.0, 1.0 / 15.0),
                    _metres([[32, 32, 32]], (h, h, h)), _metres(rec_nodes, (h, h, h)))


def _c2(nx=512, ny=512, nz=512, border=32, nt=2000, seed=2502, name="c2",
        src=None, rec=None) -> Workload:
    h = 10.0
    vel = layered_model(seed, (nx, ny, nz), 0.05)
    rho = gardner_density(vel)
    dt = 0.4 * h / 4500.0
    if src is None:
        src = [[nx // 2, ny // 2, 8]]
    if rec is None:
        rec = _surface_grid(1, 2, nx // 2, 1, 2, ny // 2, 4)
    return Workload(name, nx, ny, nz, h, h, h, 0.0, 0.0, 0.0, border, dt, nt, vel, rho,
                    ricker(nt, dt, 10.0, 0.1), _metres(src, (h, h, h)), _metres(rec, (h, h, h)))


def _c2_small() -> Workload:
    w = _c2(nx=93, ny=77, nz=61, border=16, nt=300, name="c2_small", src=[[46, 38, 8]])
    # A "true" model for gradient parity: three +/-8 % blobs inside the model
    # on a background 3 % faster.  The residual is then about 16 % of the
    # data (the blobs alone give 0.5 % in 300 steps), so that J's relative
    # error stays near the traces' (J amplifies trace error by |d| / |res|).
    blobs = blob_anomalies(w.vel, seed=2504, n_blobs=3, amp=0.08, sigma_cells=(4.0, 8.0),
                           centre_lo=(15, 15, 15), centre_hi=(78, 62, 50))
    w.extra["v_true"] = (blobs * np.float32(1.03)).astype(np.float32)
    return w


def _c2_crop(n: int = 128, nt: int = 500) -> Workload:
    """A 128^3 crop of the c2 model (same generator, seed and density): x, y
    in [192, 320), z in [0, 128), so the source node (256, 256, 8) and the
    receivers of c2 that fall inside it keep their positions; the c2 sponge
    (32 cells), dt and wavelet; 500 steps."""
    full = _c2()
    x0 = y0 = (512 - n) // 2
    vel = np.ascontiguousarray(full.vel[:n, y0:y0 + n, x0:x0 + n])
    rho = np.ascontiguousarray(full.rho[:n, y0:y0 + n, x0:x0 + n])
    h = full.dx
    src = [[256 - x0, 256 - y0, 8]]
    rec = _surface_grid(1, 2, n // 2, 1, 2, n // 2, 4)   # c2's odd nodes inside the crop
    return Workload("c2_crop", n, n, n, h, h, h, 0.0, 0.0, 0.0, full.border, full.dt, nt, vel,
                    rho, full.wavelet[:nt].copy(), _metres(src, (h, h, h)),
                    _metres(rec, (h, h, h)))


def _c3(nx=400, ny=400, nz=256, border=32, nt=1500, shots_xy=(6, 4), side=(160, 321),
        seed=2503, name="c3") -> Workload:
    h = 10.0
    vel = layered_model(seed, (nx, ny, nz), 0.05)
    rho = gardner_density(vel)
    dt = 0.4 * h / 4500.0
    sx, sy = shots_xy
    xs = [int(round((i + 0.5) * nx / sx)) for i in range(sx)]
    ys = [int(round((j + 0.5) * ny / sy)) for j in range(sy)]
    shots = [[x, y, 4] for y in ys for x in xs]
    sides = np.random.default_rng(3).integers(side[0], side[1], size=len(shots))
    win = []
    for (x, y, _), s_ in zip(shots, sides):
        ax, ay = x - s_ // 2, y - s_ // 2
        win.append([max(0, ax), min(nx, ax + s_), max(0, ay), min(ny, ay + s_)])
    w = Workload(name, nx, ny, nz, h, h, h, 0.0, 0.0, 0.0, border, dt, nt, vel, rho,
                 ricker(nt, dt, 10.0, 0.1), _metres(shots, (h, h, h)), np.zeros((0, 3)))
    w.extra["windows"] = np.asarray(win, dtype=np.int64)   # [shot] (x0, x1, y0, y1), nodes
    return w


def shot_window(w: Workload, i: int) -> Workload:
    """Shot i of a windowed workload on its own grid: the model restricted to
    its window (full depth), the origin moved to the window corner so that
    positions stay in model metres, receivers at every 2nd surface node."""
    x0, x1, y0, y1 = (int(v) for v in w.extra["windows"][i])
    vel = np.ascontiguousarray(w.vel[:, y0:y1, x0:x1])
    rho = None if w.rho is None else np.ascontiguousarray(w.rho[:, y0:y1, x0:x1])
    rec = _surface_grid(x0 + 1, 2, (x1 - x0) // 2, y0 + 1, 2, (y1 - y0) // 2, 2)
    return Workload(f"{w.name}_shot{i}", x1 - x0, y1 - y0, w.nz, w.dx, w.dy, w.dz,
                    w.ox + x0 * w.dx, w.oy + y0 * w.dy, w.oz, w.border, w.dt, w.nt, vel, rho,
                    w.wavelet, w.sources[i:i + 1].copy(),
                    _metres(rec, (w.dx, w.dy, w.dz), (w.ox, w.oy, w.oz)))


def _c4(variant: str = "true") -> Workload:
    nx, ny, nz, h = 200, 200, 160, 10.0
    bg = layered_model(4, (nx, ny, nz), 0.0)
    true = blob_anomalies(bg, seed=40, n_blobs=6, amp=0.10)
    dt = 0.4 * h / float(np.max(true))
    nt = 1200
    shots = [[x, y, 4] for y in (67, 133) for x in (25, 75, 125, 175)]
    rec = _surface_grid(2, 4, 50, 2, 4, 50, 4)
    vel = true if variant == "true" else bg
    w = Workload("c4" if variant == "true" else "c4_start", nx, ny, nz, h, h, h, 0.0, 0.0, 0.0,
                 20, dt, nt, vel, None, ricker(nt, dt, 10.0, 0.1),
                 _metres(shots, (h, h, h)), _metres(rec, (h, h, h)))
    w.extra["v_true"] = true
    w.extra["v_start"] = bg
    return w


def _c4_fd(variable_density: bool = False, nt: int = 300) -> Workload:
    n, h = 32, 10.0
    vel = layered_model(44, n, 0.05)
    rho = gardner_density(vel) if variable_density else None
    dt = 0.4 * h / float(np.max(vel))
    rec = _surface_grid(2, 4, 8, 2, 4, 8, 4)
    w = Workload("c4_fd_vd" if variable_density else "c4_fd", n, n, n, h, h, h, 0.0, 0.0, 0.0,
                 8, dt, nt, vel, rho, ricker(nt, dt, 15.0),
                 _metres([[16, 16, 4]], (h, h, h)), _metres(rec, (h, h, h)))
    dv = smooth_noise(n, 4401, sigma=3.0, max_abs=1.0)
    w.extra["dv"] = (0.01 * dv * vel).astype(np.float32)
    return w


def c5_model(seed: int, n: int = 128, border: int = 16, nt: int = 1000,
             shots_xy=(2, 2), rec_step: int = 4) -> Workload:
    """One model of the learned-preconditioner recipe (see the module notes)."""
    h = 10.0
    rng = np.random.default_rng(seed)
    bg = layered_model(seed, n, 0.0)
    n_blobs = int(rng.integers(1, 5))
    m = max(8, n // 8)
    true = blob_anomalies(bg, seed=seed + 100000, n_blobs=n_blobs, amp=0.10,
                          sigma_cells=(4.0, 10.0), centre_lo=(m, m, 2 * m),
                          centre_hi=(n - m, n - m, n - m))
    dt = 0.4 * h / (1.1 * 4500.0)
    sx, sy = shots_xy
    shots = [[int((i + 0.5) * n / sx), int((j + 0.5) * n / sy), 4]
             for j in range(sy) for i in range(sx)]
    k = n // rec_step
    rec = _surface_grid(rec_step // 2, rec_step, k, rec_step // 2, rec_step, k, 2)
    w = Workload(f"c5_{seed}", n, n, n, h, h, h, 0.0, 0.0, 0.0, border, dt, nt, bg, None,
                 ricker(nt, dt, 10.0, 0.1), _metres(shots, (h, h, h)), _metres(rec, (h, h, h)))
    w.extra["v_true"] = true
    return w


def _example() -> Workload:
    """Paper §3: 25^3 cells of 10 m, border 25, 500 steps of 1 ms, 10 Hz Ricker,
    amplitude 1e5; sources every 100 m from 20 m to 220 m, receivers every
    50 m from 10 m to 210 m.  The printed velocity formula is ambiguous; it is
    read as a 2500 m/s background with a +1000 m/s Gaussian blob of 5 cells."""
    n, h = 25, 10.0
    i = np.arange(n, dtype=np.float64)
    r2 = ((i[:, None, None] - n / 2) ** 2 + (i[None, :, None] - n / 2) ** 2
          + (i[None, None, :] - n / 2) ** 2)
    vel = (2500.0 + 1.0e3 * np.exp(-0.5 * r2 / 5.0 ** 2)).astype(np.float32)
    s = np.array([20.0, 120.0, 220.0])
    src = np.array([[x, y, z] for z in s for y in s for x in s])
    r = np.arange(10.0, 211.0, 50.0)
    rec = np.array([[x, y, 10.0] for y in r for x in r])
    return Workload("example", n, n, n, h, h, h, 0.0, 0.0, 0.0, 25, 1.0e-3, 500, vel, None,
                    ricker(500, 1.0e-3, 10.0, amplitude=1.0e5), src, rec)


WORKLOADS: Dict[str, Callable[[], Workload]] = {
    "c1": _c1,
    "c1_long": lambda: _c1(400),
    "c2": _c2,
    "c2_small": _c2_small,
    "c2_crop": _c2_crop,
    "c3": _c3,
    "c3_small": lambda: _c3(nx=96, ny=80, nz=48, border=8, nt=250, shots_xy=(2, 2),
                            side=(24, 49), name="c3_small"),
    "c3_narrow": lambda: _c3(nx=288, ny=192, nz=64, border=8, nt=500, shots_xy=(6, 4),
                             side=(32, 65), name="c3_narrow"),
    "c4": _c4,
    "c4_start": lambda: _c4("start"),
    "c4_fd": _c4_fd,
    "c4_fd_vd": lambda: _c4_fd(True),
    "example": _example,
    "c5_eval": lambda: c5_model(5999, n=256, border=20, nt=1600, shots_xy=(4, 2)),
}


def workload(name: str) -> Workload:
    """Build a named workload (deterministic; seeds are fixed per workload)."""
    try:
        return WORKLOADS[name]()
    except KeyError:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(WORKLOADS)}") from None
