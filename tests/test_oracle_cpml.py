"""Pins of the CPML oracle (oracle/cpml.py, reading R26): the first-difference
weights in closed form, exactness on polynomials, the zero-strength layer
reducing to the undamped scheme on a larger model, the adjoint as the exact
transpose (dot test), the gradient against central differences, and the
layer absorbing far better than the sponge of the same thickness."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import cpml, wave


def test_first_difference_weights_closed_form():
    # D1 f = sum_j c_j (f(x + j h) - f(x - j h)) / h: consistency 2 sum j c_j = 1,
    # odd moments 3, 5, 7 vanish (eighth order), moment 9 does not
    c = [Fraction(4, 5), Fraction(-1, 5), Fraction(4, 105), Fraction(-1, 280)]
    assert [float(x) for x in c] == list(cpml.FD1)
    assert 2 * sum(j * c[j - 1] for j in range(1, 5)) == 1
    for p in (3, 5, 7):
        assert sum(j ** p * c[j - 1] for j in range(1, 5)) == 0
    assert sum(j ** 9 * c[j - 1] for j in range(1, 5)) != 0


def test_first_difference_exact_on_polynomials():
    h = 0.37
    x = h * np.arange(-12, 13)
    for p in range(9):
        u = x ** p
        du = cpml.first_derivative(u[None, None, :], 2, h)[0, 0]
        ref = p * x ** (p - 1) if p else np.zeros_like(x)
        inner = slice(4, -4)
        assert np.allclose(du[inner], ref[inner], rtol=0, atol=1e-9 * max(1.0, np.abs(ref).max()))
    # degree 9 misses by the ninth-moment term
    du = cpml.first_derivative((x ** 9)[None, None, :], 2, h)[0, 0]
    assert np.max(np.abs(du[4:-4] - 9 * x[4:-4] ** 8)) > 1e-6


def test_profiles():
    a, b = cpml.profile(10, 5, 10.0, 1e-3, 3000.0, 12.0)
    delta = cpml.layer_depth(10, 5)
    assert np.all(a[delta == 0] == 0.0) and np.all(a[delta > 0] < 0.0)
    assert np.all((b > 0) & (b <= 1))
    # innermost layer cell: d = d0 / 25, alpha = pi f (1 - 1/5)
    d0 = -3 * 3000.0 * np.log(1e-3) / (2 * 5 * 10.0)
    d, al = d0 / 25, np.pi * 12.0 * 0.8
    bb = np.exp(-(d + al) * 1e-3)
    assert b[4] == pytest.approx(bb, rel=1e-15)
    assert a[4] == pytest.approx(d * (bb - 1) / (d + al), rel=1e-15)
    # free top: no layer before the model
    a2, _ = cpml.profile(10, 5, 10.0, 1e-3, 3000.0, 12.0, free_top=True)
    assert np.all(a2[:5] == 0.0) and np.all(a2[-5:] < 0.0)


def _case(rng, fs=False, vd=True, n=6, N=4, nt=14):
    g = wave.Grid(n, n + 1, n, 10.0, 11.0, 9.0, border=N, dt=1.2e-3, nt=nt, free_surface=fs)
    vel = 2000 + 300 * rng.random((n, n + 1, n))
    rho = (1500 + 500 * rng.random((n, n + 1, n))) if vd else None
    src = [20.0, 30.0, 25.0]
    rec = np.array([[10.0, 20.0, 30.0], [40.0, 50.0, 10.0], [0.0, 0.0, 0.0], [50.0, 60.0, 45.0]])
    return g, vel, rho, src, rec


def test_zero_strength_layer_is_the_undamped_scheme_on_a_larger_model():
    # R0 = 1 gives d = 0, so a = 0 and psi = zeta = 0: the step is the plain
    # leapfrog with no sponge, i.e. border 0 on the edge-padded model
    rng = np.random.default_rng(1)
    g, vel, rho, src, rec = _case(rng)
    f = rng.standard_normal(g.nt)
    out = cpml.forward(g, vel, rho, f, src, rec, vmax=2300.0, fpeak=15.0, r0=1.0,
                       fp32_inputs=False)
    N = g.border
    big = wave.Grid(g.nx + 2 * N, g.ny + 2 * N, g.nz + 2 * N, g.dx, g.dy, g.dz,
                    ox=-N * g.dx, oy=-N * g.dy, oz=-N * g.dz, border=0, dt=g.dt, nt=g.nt)
    ref = wave.forward(big, wave.pad_edge(vel, N), wave.pad_edge(rho, N), f, src, rec,
                       fp32_inputs=False)
    assert np.max(np.abs(out.seis - ref.seis)) <= 1e-13 * np.max(np.abs(ref.seis))
    # and the real layer changes the result
    act = cpml.forward(g, vel, rho, f, src, rec, vmax=2300.0, fpeak=15.0, fp32_inputs=False)
    assert np.max(np.abs(act.seis - ref.seis)) > 1e-5 * np.max(np.abs(ref.seis))


@pytest.mark.parametrize("fs,vd", [(False, False), (False, True), (True, True)])
def test_dot_test_adjoint_is_the_transpose(fs, vd):
    rng = np.random.default_rng(2 + fs + 2 * vd)
    g, vel, rho, src, rec = _case(rng, fs, vd)
    for _ in range(2):
        f = rng.standard_normal(g.nt)
        dp = rng.standard_normal((len(rec), g.nt))
        Ff = cpml.forward(g, vel, rho, f, src, rec, vmax=2300.0, fpeak=15.0,
                          fp32_inputs=False).seis
        Ftd = cpml.adjoint_source_transpose(g, vel, rho, src, rec, dp, vmax=2300.0, fpeak=15.0,
                                            fp32_inputs=False)
        lhs, rhs = float(np.sum(Ff * dp)), float(np.sum(f * Ftd))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("fs", [False, True])
def test_gradient_matches_central_differences(fs):
    rng = np.random.default_rng(7 + fs)
    g, vel, rho, src, rec = _case(rng, fs, True, nt=20)
    f = np.sin(np.arange(g.nt) * 0.7) * np.exp(-0.02 * np.arange(g.nt))
    true = vel * (1 + 0.02 * rng.standard_normal(vel.shape))
    kw = dict(vmax=2400.0, fpeak=15.0, fp32_inputs=False)
    dobs = cpml.forward(g, true, rho, f, src, rec, **kw).seis
    res = cpml.gradient(g, vel, rho, f, src, rec, dobs, **kw)
    dv = rng.standard_normal(vel.shape)
    eps = 1e-2

    def J(v):
        return wave.misfit(cpml.forward(g, v, rho, f, src, rec, **kw).seis, dobs, False)[0]

    fd = (J(vel + eps * dv) - J(vel - eps * dv)) / (2 * eps)
    an = float(np.sum(res.grad * dv))
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_layer_absorbs_better_than_the_sponge():
    # homogeneous 3-D box, source at its centre; once the direct wave has left
    # the model, the energy still inside it is what the boundary sent back
    n, N, h = 24, 10, 10.0
    c = 2000.0
    dt = 0.35 * h / c
    nt = 130
    vel = np.full((n, n, n), c)
    t = np.arange(nt) * dt
    fp = 25.0
    arg = (np.pi * fp * (t - 1.2 / fp)) ** 2
    f = (1 - 2 * arg) * np.exp(-arg)
    src = [12 * h, 12 * h, 12 * h]
    g = wave.Grid(n, n, n, h, h, h, border=N, dt=dt, nt=nt)
    core = (slice(N, N + n),) * 3

    def late_energy(states):
        w1, w0 = states[-1][core], states[-2][core]
        return float(np.sum((w1 - w0) ** 2))

    def peak_energy(states):
        return max(float(np.sum((states[i][core] - states[i - 1][core]) ** 2))
                   for i in range(1, len(states)))

    st_c = cpml.forward(g, vel, None, f, src, [src], vmax=c, fpeak=fp, keep_states=True).states
    st_s = wave.forward(g, vel, None, f, src, [src], keep_states=True).states
    rc = late_energy(st_c) / peak_energy(st_c)
    rs = late_energy(st_s) / peak_energy(st_s)
    # measured: 5.5e-8 against 7.7e-5 for the sponge
    assert rc < 0.01 * rs
    assert rc < 1e-6
