"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test pins one part of the oracle to something other than itself:
closed forms, invariants, special cases and brute force.  Together they are
chosen so that a dropped term, a wrong sign, a swapped axis or a transposed
operand in any oracle function fails at least one of them.
"""

from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from oracle import wave
import seisgen

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------------------
# 1. the 1-D weights: moments fixed by an eighth-order second derivative
# ---------------------------------------------------------------------------
def test_fd8_moment_conditions_exact():
    """Taylor moments: a0 + 2 sum a_j = 0, 2 sum a_j j^2 = 2, 2 sum a_j j^p = 0
    for p = 4, 6, 8, and 2 sum a_j j^10 = -1152 (error -h^8 f^(10) / 3150)."""
    a = [Fraction(x).limit_denominator(10000) for x in oracle.FD8]
    assert [float(x) for x in a] == list(oracle.FD8)
    assert a[0] + 2 * sum(a[1:]) == 0
    mom = lambda p: 2 * sum(a[j] * j ** p for j in range(1, 5))
    assert mom(2) == 2
    assert mom(4) == 0 and mom(6) == 0 and mom(8) == 0
    assert mom(10) == -1152
    assert Fraction(-1152, math.factorial(10)) == Fraction(-1, 3150)


# ---------------------------------------------------------------------------
# 2. the 3-D Laplacian: exact on polynomials of degree <= 9 per axis
# ---------------------------------------------------------------------------
def _poly_grid(shape, h):
    nz, ny, nx = shape
    z = (np.arange(nz) - nz / 2) * h[2]
    y = (np.arange(ny) - ny / 2) * h[1]
    x = (np.arange(nx) - nx / 2) * h[0]
    return z[:, None, None], y[None, :, None], x[None, None, :]


@pytest.mark.parametrize("deg", [(2, 5, 9), (9, 0, 3), (4, 9, 7), (0, 0, 1)])
def test_laplacian_exact_on_polynomials(deg):
    a, b, c = deg                         # exponents of x, y, z
    h = (0.11, 0.07, 0.13)                # unequal spacings catch axis swaps
    shape = (14, 15, 16)
    z, y, x = _poly_grid(shape, h)
    u = x ** a * y ** b * z ** c
    lap = oracle.laplacian(u, h)
    exact = (a * (a - 1) * x ** max(a - 2, 0) * y ** b * z ** c
             + b * (b - 1) * x ** a * y ** max(b - 2, 0) * z ** c
             + c * (c - 1) * x ** a * y ** b * z ** max(c - 2, 0))
    core = (slice(4, -4),) * 3
    # round-off of the stencil sum scales with |u| / h^2
    scale = np.max(np.abs(exact[core])) + np.max(np.abs(u)) / min(h) ** 2
    assert np.max(np.abs(lap[core] - exact[core])) <= 1e-9 * scale


def test_laplacian_degree_ten_misses_by_closed_form():
    h = (0.1, 0.2, 0.3)
    shape = (12, 12, 12)
    z, y, x = _poly_grid(shape, h)
    u = x ** 10 + 2.0 * y ** 10 - z ** 10
    lap = oracle.laplacian(u, h)
    exact = 90 * x ** 8 + 180 * y ** 8 - 90 * z ** 8
    # truncation of the 8th-order stencil on t^10: -1152 h^8 per term
    miss = -1152 * (h[0] ** 8 + 2.0 * h[1] ** 8 - h[2] ** 8)
    core = (slice(4, -4),) * 3
    err = lap[core] - exact[core]
    assert np.allclose(err, miss, rtol=1e-6, atol=1e-9 * np.max(np.abs(exact[core])))


def test_spatial_order_of_convergence():
    """L sin(ax)sin(by)sin(cz) -> -(a^2+b^2+c^2) u with error ratio ~2^8 on halving h."""
    al, be, ga = 1.0, 1.3, 0.7
    errs = []
    for h in (0.4, 0.2):
        n = int(round(8.0 / h))
        z, y, x = _poly_grid((n, n, n), (h, h, h))
        u = np.sin(al * x + 0.3) * np.sin(be * y + 0.1) * np.sin(ga * z + 0.2)
        lap = oracle.laplacian(u, (h, h, h))
        core = (slice(4, -4),) * 3
        errs.append(np.max(np.abs(lap[core] + (al ** 2 + be ** 2 + ga ** 2) * u[core])))
    slope = math.log2(errs[0] / errs[1])
    assert slope >= 7.5, (errs, slope)


# ---------------------------------------------------------------------------
# 3. time stepping: exact discrete evolution of a periodic eigenmode
# ---------------------------------------------------------------------------
def _symbol(kh):
    a = oracle.FD8
    return -(a[0] + 2.0 * sum(a[j] * math.cos(j * kh) for j in range(1, 5)))


def test_periodic_eigenmode_evolves_as_cos_n_theta():
    nx, ny, nz = 16, 12, 10
    dx, dy, dz = 10.0, 12.0, 8.0
    c, dt, nt = 2500.0, 1.0e-3, 120
    jx, jy, jz = 2, 1, 3
    kx, ky, kz = (2 * math.pi * jx / (nx * dx), 2 * math.pi * jy / (ny * dy),
                  2 * math.pi * jz / (nz * dz))
    X = np.arange(nx)[None, None, :] * dx
    Y = np.arange(ny)[None, :, None] * dy
    Z = np.arange(nz)[:, None, None] * dz
    u = np.cos(kx * X + ky * Y + kz * Z + 0.4) * np.ones((nz, ny, nx))
    lam = _symbol(kx * dx) / dx ** 2 + _symbol(ky * dy) / dy ** 2 + _symbol(kz * dz) / dz ** 2
    cos_t = 1.0 - 0.5 * c * c * dt * dt * lam
    theta = math.acos(cos_t)
    g = oracle.Grid(nx, ny, nz, dx, dy, dz, border=0, dt=dt, nt=nt)
    vel = np.full((nz, ny, nx), c)
    rec = [[3 * dx, 5 * dy, 7 * dz]]
    r = oracle.forward(g, vel, None, np.zeros(nt), [0.0, 0.0, 0.0], rec, w0=u, w_m1=cos_t * u,
                       periodic=True, fp32_inputs=False)
    expect_last = math.cos(nt * theta) * u
    assert np.max(np.abs(r.last - expect_last)) <= 1e-11
    n = np.arange(1, nt + 1)
    expect_trace = np.cos(n * theta) * u[7, 5, 3]
    assert np.max(np.abs(r.seis[0] - expect_trace)) <= 1e-11


# ---------------------------------------------------------------------------
# 4. stability: closed-form CFL limit and behaviour just across it
# ---------------------------------------------------------------------------
def test_cfl_closed_form():
    lam1 = oracle.laplacian_symbol_max()
    assert abs(lam1 - 2048.0 / 315.0) < 1e-13
    limit = 2.0 / math.sqrt(3.0 * 2048.0 / 315.0)
    assert abs(limit - 0.45286) < 1e-5
    g = oracle.Grid(10, 10, 10, 10.0, 10.0, 10.0, dt=limit * 10.0 / 3000.0)
    assert abs(oracle.cfl_ratio(g, 3000.0) - 1.0) < 1e-12
    # a positive mass term tightens the bound
    assert oracle.cfl_ratio(g, 3000.0, 1e-3) > 1.0


@pytest.mark.parametrize("factor,grows", [(0.999, False), (1.001, True)])
def test_cfl_blowup_across_limit(factor, grows):
    n, h, c, nt = 8, 10.0, 3000.0, 400
    limit = 2.0 / math.sqrt(3.0 * 2048.0 / 315.0)
    dt = factor * limit * h / c
    i = np.arange(n)
    checker = (-1.0) ** (i[:, None, None] + i[None, :, None] + i[None, None, :])
    g = oracle.Grid(n, n, n, h, h, h, border=0, dt=dt, nt=nt)
    r = oracle.forward(g, np.full((n, n, n), c), None, np.zeros(nt), [0, 0, 0], [[0, 0, 0]],
                       w0=checker, w_m1=-checker, periodic=True, fp32_inputs=False)
    # near the limit theta ~ pi, so the start (1, -1) is almost a pure cos(n theta)
    peak = np.max(np.abs(r.seis))
    if grows:
        assert peak > 1e6
    else:
        assert peak <= 1.01


# ---------------------------------------------------------------------------
# 5. source normalisation and propagation: analytic 3-D Green's function
# ---------------------------------------------------------------------------
def _green_case(dt):
    n, h, c, f = 72, 10.0, 2000.0, 10.0
    T = 0.3
    nt = int(round(T / dt))
    g = oracle.Grid(n, n, n, h, h, h, border=0, dt=dt, nt=nt)
    vel = np.full((n, n, n), c)
    src = [36 * h, 36 * h, 36 * h]
    rec = [[(36 + 15) * h, 36 * h, 36 * h], [36 * h, (36 + 12) * h, 36 * h],
           [36 * h, 36 * h, (36 - 10) * h]]
    wav = seisgen.ricker(nt, dt, f, 0.1)
    r = oracle.forward(g, vel, None, wav.astype(np.float64), src, rec, fp32_inputs=False)
    t = (np.arange(nt) + 1) * dt            # trace sample n is time (n+1) dt
    err = []
    for i, dist in enumerate((150.0, 120.0, 100.0)):
        tau = t - dist / c - 0.1
        a = (math.pi * f * tau) ** 2
        exact = (1.0 - 2.0 * a) * np.exp(-a) / (4 * math.pi * c * c * dist)
        err.append(np.linalg.norm(r.seis[i] - exact) / np.linalg.norm(exact))
    return max(err)


@pytest.mark.slow
def test_greens_function_homogeneous():
    # 10-15 cells from a point source the h^8 / point-source floor (~2e-3) already
    # dominates the O(dt^2) error, which the eigenmode test pins exactly.
    e1 = _green_case(1.0e-3)
    assert e1 <= 5e-3, e1


# ---------------------------------------------------------------------------
# 6. energy conservation without sponge and source (CD and VD)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("vd", [False, True])
def test_energy_conserved(vd):
    n, h = 20, 10.0
    vel = seisgen.layered_model(7, n, 0.05).astype(np.float64)
    rho = seisgen.gardner_density(vel).astype(np.float64) if vd else None
    dt = 0.35 * h / vel.max()
    nt, n0 = 160, 40
    wav = np.zeros(nt)
    wav[:n0] = seisgen.ricker(n0, dt, 25.0, 0.02)
    g = oracle.Grid(n, n, n, h, h, h, border=0, dt=dt, nt=nt)
    r = oracle.forward(g, vel, rho, wav, [95.0, 100.0, 105.0], [[50.0, 50.0, 50.0]],
                       keep_states=True, fp32_inputs=False)
    c = oracle.coefficients(g, vel, rho)
    E = [oracle.energy(c, g, r.states[m + 1], r.states[m]) for m in range(n0 + 1, nt)]
    E = np.array(E)
    assert E[0] > 0
    assert np.max(np.abs(E - E[0])) <= 1e-10 * abs(E[0])


# ---------------------------------------------------------------------------
# 7. variable-density special cases
# ---------------------------------------------------------------------------
def test_constant_density_vd_equals_cd():
    w = seisgen.workload("c4_fd")
    g = oracle.Grid(**{**w.grid_kwargs(), "nt": 120})
    rho = np.full_like(w.vel, 2150.0)
    a = oracle.forward(g, w.vel, None, w.wavelet[:120], w.sources[0], w.receivers)
    b = oracle.forward(g, w.vel, rho, w.wavelet[:120], w.sources[0], w.receivers)
    c = oracle.coefficients(g, w.vel.astype(np.float64), rho.astype(np.float64))
    assert np.max(np.abs(c.m2)) <= 1e-13 * 1e-4
    assert np.max(np.abs(a.seis - b.seis)) <= 1e-13 * np.max(np.abs(a.seis))


def test_exponential_density_mass_term():
    """sqrt(rho) = exp(beta z) has m^2 = beta^2 exactly; the discrete error is O(h^8)."""
    n, h, beta = 24, 10.0, 2.0e-3
    z = np.arange(n) * h
    s = np.exp(beta * z)[:, None, None] * np.ones((n, n, n))
    rho = s * s
    g = oracle.Grid(n, n, n, h, h, h, border=3, dt=1e-3, nt=1)
    c = oracle.coefficients(g, np.full((n, n, n), 2000.0), rho)
    core = c.m2[3 + 4:-3 - 4, :, :]        # away from the edge-replicated z ends
    assert np.max(np.abs(core / beta ** 2 - 1.0)) <= 1e-8
    # x and y directions are constant, so even the replicated faces are exact there
    assert np.allclose(c.m2[7:-7, 0, 0], beta ** 2, rtol=1e-8)


# ---------------------------------------------------------------------------
# 8. adjoint: dot-product test and brute-force transpose
# ---------------------------------------------------------------------------
def _small_vd_case(n=12, border=4, nt=40, seed=3):
    vel = seisgen.layered_model(seed, n, 0.05).astype(np.float64)
    rho = seisgen.gardner_density(vel).astype(np.float64)
    dt = 0.4 * 10.0 / vel.max()
    g = oracle.Grid(n, n, n, 10.0, 10.0, 10.0, border=border, dt=dt, nt=nt)
    src = [55.0, 45.0, 30.0]
    rec = [[10.0, 20.0, 20.0], [90.0, 80.0, 40.0], [60.0, 30.0, 90.0], [60.0, 30.0, 90.0]]
    return g, vel, rho, src, rec


def test_adjoint_dot_product():
    g, vel, rho, src, rec = _small_vd_case()
    rng = np.random.default_rng(11)
    f = rng.standard_normal(g.nt)
    dp = rng.standard_normal((len(rec), g.nt))
    Ff = oracle.forward(g, vel, rho, f, src, rec, fp32_inputs=False).seis
    Ftd = oracle.adjoint_source_transpose(g, vel, rho, src, rec, dp, fp32_inputs=False)
    lhs = float(np.sum(Ff * dp))
    rhs = float(np.dot(f, Ftd))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), np.linalg.norm(Ff) * np.linalg.norm(dp))


def test_adjoint_brute_force_transpose():
    g, vel, rho, src, rec = _small_vd_case(n=8, border=2, nt=8, seed=5)
    src = [35.0, 45.0, 30.0]
    rec = [[10.0, 20.0, 20.0], [60.0, 50.0, 40.0], [30.0, 70.0, 60.0]]
    nt, nr = g.nt, len(rec)
    F = np.zeros((nr * nt, nt))
    for n in range(nt):
        e = np.zeros(nt)
        e[n] = 1.0
        F[:, n] = oracle.forward(g, vel, rho, e, src, rec, fp32_inputs=False).seis.ravel()
    FT = np.zeros((nt, nr * nt))
    for col in range(nr * nt):
        d = np.zeros(nr * nt)
        d[col] = 1.0
        FT[:, col] = oracle.adjoint_source_transpose(g, vel, rho, src, rec, d.reshape(nr, nt),
                                                     fp32_inputs=False)
    assert np.max(np.abs(F)) > 0
    assert np.max(np.abs(FT - F.T)) <= 1e-13 * np.max(np.abs(F))


# ---------------------------------------------------------------------------
# 9. gradient: central finite differences of J (FP64)
# ---------------------------------------------------------------------------
def _fd_case(vd):
    n, h = 16, 10.0
    vel = seisgen.layered_model(21, n, 0.05).astype(np.float64)
    true = seisgen.blob_anomalies(vel.astype(np.float32), seed=2, n_blobs=2, amp=0.05,
                                  sigma_cells=(2, 3), centre_lo=(5, 5, 5),
                                  centre_hi=(11, 11, 11)).astype(np.float64)
    rho = seisgen.gardner_density(vel).astype(np.float64) if vd else None
    dt = 0.4 * h / true.max()
    g = oracle.Grid(n, n, n, h, h, h, border=6, dt=dt, nt=150)
    wav = seisgen.ricker(150, dt, 20.0).astype(np.float64)
    src = [75.0, 80.0, 20.0]
    rec = [[x, y, 30.0] for x in (10.0, 50.0, 100.0, 140.0) for y in (20.0, 90.0, 150.0)]
    dobs = oracle.forward(g, true, rho, wav, src, rec, fp32_inputs=False).seis
    return g, vel, rho, wav, src, rec, dobs


def _J(g, vel, rho, wav, src, rec, dobs):
    s = oracle.forward(g, vel, rho, wav, src, rec, fp32_inputs=False).seis
    return oracle.misfit(s, dobs, fp32_inputs=False)[0]


@pytest.mark.parametrize("vd", [False, True])
def test_gradient_directional_fd(vd):
    g, vel, rho, wav, src, rec, dobs = _fd_case(vd)
    res = oracle.gradient(g, vel, rho, wav, src, rec, dobs, fp32_inputs=False)
    dv = seisgen.smooth_noise(16, 5, sigma=3.0, max_abs=1.0).astype(np.float64) * vel
    eps = 1e-4
    fd = (_J(g, vel + eps * dv, rho, wav, src, rec, dobs)
          - _J(g, vel - eps * dv, rho, wav, src, rec, dobs)) / (2 * eps)
    an = float(np.sum(res.grad * dv))
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    assert abs(res.misfit - _J(g, vel, rho, wav, src, rec, dobs)) <= 1e-14 * res.misfit


def test_gradient_pointwise_fd_including_edges():
    g, vel, rho, wav, src, rec, dobs = _fd_case(False)
    res = oracle.gradient(g, vel, rho, wav, src, rec, dobs, fp32_inputs=False)
    # interior, face, edge and corner cells (the last three gather sponge cells)
    for node in [(8, 7, 9), (5, 10, 4), (0, 8, 8), (15, 0, 7), (0, 0, 15)]:
        eps = 1e-4 * vel[node]
        vp, vm = vel.copy(), vel.copy()
        vp[node] += eps
        vm[node] -= eps
        fd = (_J(g, vp, rho, wav, src, rec, dobs) - _J(g, vm, rho, wav, src, rec, dobs)) / (2 * eps)
        an = res.grad[node]
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9 * np.max(np.abs(res.grad)), (node, fd, an)


def test_segment_checkpointing_is_exact():
    g, vel, rho, wav, src, rec, dobs = _fd_case(True)
    a = oracle.gradient(g, vel, rho, wav, src, rec, dobs, fp32_inputs=False, segment=1)
    b = oracle.gradient(g, vel, rho, wav, src, rec, dobs, fp32_inputs=False, segment=13)
    assert np.array_equal(a.grad, b.grad)


def test_zero_residual_gives_zero_gradient():
    g, vel, rho, wav, src, rec, _ = _fd_case(True)
    d = oracle.forward(g, vel, rho, wav, src, rec, fp32_inputs=False).seis
    r = oracle.gradient(g, vel, rho, wav, src, rec, d, fp32_inputs=False)
    assert r.misfit == 0.0
    assert np.all(r.grad == 0.0)


def test_zero_top_planes_and_illumination():
    g, vel, rho, wav, src, rec, dobs = _fd_case(False)
    r = oracle.gradient(g, vel, rho, wav, src, rec, dobs, fp32_inputs=False,
                        zero_top_planes=3, illumination=True)
    assert np.all(r.grad[:3] == 0.0) and np.any(r.grad[3] != 0.0)
    f = oracle.forward(g, vel, rho, wav, src, rec, fp32_inputs=False, illumination=True)
    assert np.allclose(r.illum, f.illum, rtol=1e-12, atol=0)


# ---------------------------------------------------------------------------
# 10. invariants: reciprocity and axis permutation
# ---------------------------------------------------------------------------
def test_reciprocity_heterogeneous_vd():
    n, h = 16, 10.0
    vel = seisgen.layered_model(31, n, 0.05).astype(np.float64)
    rho = seisgen.gardner_density(vel).astype(np.float64) * (1.0 + 0.2 * np.linspace(0, 1, n))[:, None, None]
    dt = 0.4 * h / vel.max()
    g = oracle.Grid(n, n, n, h, h, h, border=5, dt=dt, nt=140)
    wav = seisgen.ricker(140, dt, 20.0).astype(np.float64)
    a, b = (3, 5, 4), (12, 9, 11)          # (ix, iy, iz)
    xa = [a[0] * h, a[1] * h, a[2] * h]
    xb = [b[0] * h, b[1] * h, b[2] * h]
    tab = oracle.forward(g, vel, rho, wav, xa, [xb], fp32_inputs=False).seis[0]
    tba = oracle.forward(g, vel, rho, wav, xb, [xa], fp32_inputs=False).seis[0]
    wa = rho[a[2], a[1], a[0]] * vel[a[2], a[1], a[0]] ** 2
    wb = rho[b[2], b[1], b[0]] * vel[b[2], b[1], b[0]] ** 2
    assert np.max(np.abs(tab * wa - tba * wb)) <= 1e-12 * np.max(np.abs(tab * wa))


def test_axis_permutation_symmetry():
    n, h = 14, 10.0
    vel = seisgen.layered_model(8, n, 0.05).astype(np.float64)
    rho = seisgen.gardner_density(vel).astype(np.float64)
    g = oracle.Grid(n, n, n, h, h, h, border=4, dt=0.4 * h / vel.max(), nt=60)
    wav = seisgen.ricker(60, g.dt, 25.0).astype(np.float64)
    src = [30.0, 70.0, 110.0]
    rec = [[10.0, 20.0, 120.0], [100.0, 40.0, 60.0]]
    a = oracle.forward(g, vel, rho, wav, src, rec, fp32_inputs=False)
    # swap x and z: v'[z][y][x] = v[x][y][z], positions (x,y,z) -> (z,y,x)
    vt, rt = vel.transpose(2, 1, 0).copy(), rho.transpose(2, 1, 0).copy()
    b = oracle.forward(g, vt, rt, wav, src[::-1], [r[::-1] for r in rec], fp32_inputs=False)
    assert np.max(np.abs(a.seis - b.seis)) <= 1e-12 * np.max(np.abs(a.seis))
    assert np.max(np.abs(a.last - b.last.transpose(2, 1, 0))) <= 1e-12 * np.max(np.abs(a.last))


# ---------------------------------------------------------------------------
# 11. padding / sponge / geometry / misfit pieces
# ---------------------------------------------------------------------------
def test_fold_is_transpose_of_edge_padding():
    rng = np.random.default_rng(0)
    for shape, N in [((5, 6, 7), 3), ((1, 4, 2), 2), ((3, 3, 3), 0)]:
        a = rng.standard_normal(shape)
        b = rng.standard_normal(tuple(s + 2 * N for s in shape))
        lhs = np.sum(oracle.pad_edge(a, N) * b)
        rhs = np.sum(a * oracle.fold_padding(b, N))
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(b))


def test_sponge_profile_values():
    g = oracle.sponge_profile(10, 4)
    assert g.shape == (18,)
    assert np.all(g[4:14] == 1.0)
    assert abs(g[0] - math.exp(-0.16)) < 1e-15 and abs(g[-1] - math.exp(-0.16)) < 1e-15
    assert abs(g[2] - math.exp(-(0.4 * 2 / 4) ** 2)) < 1e-15
    assert np.all(np.diff(g[:5]) > 0) and np.array_equal(g, g[::-1])
    assert np.all(oracle.sponge_profile(7, 0) == 1.0)


def test_node_index_round_half_up_and_range():
    g = oracle.Grid(10, 8, 6, 10.0, 5.0, 2.0, ox=100.0, oy=-20.0, oz=0.0, border=3)
    assert oracle.node_index(g, [100.0, -20.0, 0.0]) == (3, 3, 3)
    assert oracle.node_index(g, [104.999, -17.5, 0.999]) == (3, 4, 3)   # 2.5 rounds up
    assert oracle.node_index(g, [105.0, -17.6, 1.0]) == (4, 3, 4)
    assert oracle.node_index(g, [190.0, 15.0, 10.0]) == (8, 10, 12)
    for bad in ([94.9, 0.0, 0.0], [195.0, 0.0, 0.0], [100.0, 17.5, 0.0], [100.0, 0.0, 11.0]):
        with pytest.raises(ValueError):
            oracle.node_index(g, bad)


def test_misfit_half_sum_of_squares():
    d = np.array([[1.0, 2.0], [3.0, -1.0]])
    o = np.array([[0.5, 2.0], [1.0, 0.0]])
    J, res = oracle.misfit(d, o, fp32_inputs=False)
    assert J == 0.5 * (0.25 + 0 + 4.0 + 1.0)
    assert np.array_equal(res, d - o)


# ---------------------------------------------------------------------------
# 12. optimal checkpointing counts (closed form vs dynamic programme)
# ---------------------------------------------------------------------------
def test_revolve_closed_form_matches_dynamic_programme():
    cost = oracle.optimal_cost_table(60, 6)
    for l in range(1, 61):
        for c in range(0, 7):
            assert cost[l, c] == oracle.forward_steps_closed_form(l, c + 1), (l, c)


def test_revolve_known_values():
    assert oracle.forward_steps_closed_form(1200, 20) == 3347
    assert oracle.forward_steps_closed_form(10, 1) == 45
    assert oracle.forward_steps_closed_form(2, 1) == 1


# ---------------------------------------------------------------------------
# 13. input generators used by both sides
# ---------------------------------------------------------------------------
def test_ricker_closed_form():
    dt, f = 1e-4, 12.0
    w = seisgen.ricker(4000, dt, f, t0=0.1).astype(np.float64)
    assert w[1000] == 1.0 and np.argmax(w) == 1000
    assert w[999] == w[1001] < 1.0
    assert abs(np.sum(w) * dt) < 1e-6
    assert seisgen.ricker(201, 1e-3, 10.0, amplitude=1e5).max() == 1e5


def test_layered_generator_ranges():
    v = seisgen.layered_model(2502, (40, 36, 128), 0.05)
    assert v.dtype == np.float32 and v.shape == (128, 36, 40)
    assert v.min() >= 1500.0 and v.max() <= 4500.0
    prof = v.mean(axis=(1, 2))
    assert prof[-1] > prof[0] + 2000
    rho = seisgen.gardner_density(v)
    assert 1929.0 <= rho.min() and rho.max() <= 2540.0


def test_paper_example_config_fixture():
    """The 'example' workload uses the parameter values printed in the paper."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_example_config.txt")
    cfg = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = (s.strip() for s in line.split("="))
            cfg[k] = float(v)
    w = seisgen.workload("example")
    assert (w.nx, w.ny, w.nz) == (cfg["nx"], cfg["ny"], cfg["nz"])
    assert (w.dx, w.dy, w.dz) == (cfg["dx"], cfg["dy"], cfg["dz"])
    assert w.border == cfg["border"] and w.nt == cfg["ns"] and w.dt == cfg["dt"]
    assert (w.ox, w.oy, w.oz) == (cfg["ox"], cfg["oy"], cfg["oz"])
    assert len(w.sources) == cfg["n_src"]
    assert abs(float(np.max(w.wavelet)) - cfg["amplitude"]) <= 1e-3 * cfg["amplitude"]
    assert int(cfg["stencil"]) == wave.RADIUS      # 'stencil = 4': radius-4, eighth order


# ---------------------------------------------------------------------------
# 11. free surface (R23): the discrete image principle, and the adjoint
# ---------------------------------------------------------------------------
def _mirror_case(nh=9, n=10, border=4, nt=60, seed=31):
    """A half-space model with a free surface and the full-space model made by
    mirroring it evenly about its top plane (full plane c = nh - 1)."""
    h = 10.0
    vh = seisgen.layered_model(seed, (n, n, nh), 0.05).astype(np.float64)
    rh = seisgen.gardner_density(vh).astype(np.float64)
    c = nh - 1
    idx = np.abs(np.arange(2 * nh - 1) - c)           # full plane -> half plane
    vf, rf = vh[idx], rh[idx]
    dt = 0.4 * h / vh.max()
    gh = oracle.Grid(n, n, nh, h, h, h, border=border, dt=dt, nt=nt, free_surface=True)
    gf = oracle.Grid(n, n, 2 * nh - 1, h, h, h, oz=-c * h, border=border, dt=dt, nt=nt)
    return gh, gf, vh, rh, vf, rf


def test_free_surface_equals_antisymmetric_image_source():
    """With a free surface the half-space solution equals, on every receiver,
    the full-space solution of the mirrored model driven by the source minus
    its mirror image (the field is odd about the surface)."""
    gh, gf, vh, rh, vf, rf = _mirror_case()
    rng = np.random.default_rng(5)
    f = rng.standard_normal(gh.nt)
    src = [45.0, 55.0, 30.0]
    img = [45.0, 55.0, -30.0]
    rec = [[15.0, 25.0, 10.0], [75.0, 35.0, 50.0], [45.0, 55.0, 80.0], [25.0, 85.0, 0.0]]
    half = oracle.forward(gh, vh, rh, f, src, rec, fp32_inputs=False).seis
    full = (oracle.forward(gf, vf, rf, f, src, rec, fp32_inputs=False).seis
            - oracle.forward(gf, vf, rf, f, img, rec, fp32_inputs=False).seis)
    assert np.max(np.abs(half[:3])) > 0
    assert np.max(np.abs(half - full)) <= 1e-12 * np.max(np.abs(full))
    assert np.all(half[3] == 0.0)                     # a receiver on the surface
    # without the surface the half-space result differs (the pin is not vacuous)
    gn = oracle.Grid(**{**gh.__dict__, "free_surface": False})
    none = oracle.forward(gn, vh, rh, f, src, rec, fp32_inputs=False).seis
    assert np.max(np.abs(none[:3] - full[:3])) > 1e-2 * np.max(np.abs(full))


def test_free_surface_adjoint_dot_product():
    g, vel, rho, src, rec = _small_vd_case()
    g = oracle.Grid(**{**g.__dict__, "free_surface": True})
    rng = np.random.default_rng(12)
    f = rng.standard_normal(g.nt)
    dp = rng.standard_normal((len(rec), g.nt))
    Ff = oracle.forward(g, vel, rho, f, src, rec, fp32_inputs=False).seis
    Ftd = oracle.adjoint_source_transpose(g, vel, rho, src, rec, dp, fp32_inputs=False)
    lhs = float(np.sum(Ff * dp))
    rhs = float(np.dot(f, Ftd))
    assert np.max(np.abs(Ff)) > 0
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), np.linalg.norm(Ff) * np.linalg.norm(dp))
