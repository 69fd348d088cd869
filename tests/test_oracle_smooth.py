"""Pins of the gradient-smoothing oracle (oracle/smooth.py): closed forms of
the exponential kernel, constants kept, symmetry, and the reduction of the
3-D Bessel solve to a 1-D banded solve."""

import numpy as np
import scipy.linalg

from oracle import smooth


def test_laplace_interior_impulse_is_the_exponential_kernel():
    # far from the ends the 1-D response to a unit impulse is
    # (1 - a)/(1 + a) a^|n| with a = exp(-h / l)
    n, h, l = 201, 10.0, 25.0
    g = np.zeros((1, 1, n))
    g[0, 0, 100] = 1.0
    u = smooth.laplace_filter(g, (l, 0.0, 0.0), (h, h, h))[0, 0]
    a = np.exp(-h / l)
    k = (1 - a) / (1 + a) * a ** np.abs(np.arange(n) - 100)
    assert np.max(np.abs(u[60:141] - k[60:141])) <= 1e-12
    assert abs(u.sum() - 1.0) <= 1e-12          # zero-flux ends keep the mass


def test_filters_keep_constants_and_are_symmetric():
    rng = np.random.default_rng(3)
    shape, lens, hs = (6, 7, 9), (20.0, 15.0, 30.0), (10.0, 10.0, 12.0)
    c = np.full(shape, 3.5)
    for f in (smooth.laplace_filter, smooth.bessel_filter):
        assert np.allclose(f(c, lens, hs), c, rtol=0, atol=1e-12)
        x, y = rng.standard_normal(shape), rng.standard_normal(shape)
        lhs, rhs = np.sum(f(x, lens, hs) * y), np.sum(x * f(y, lens, hs))
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(x * y))
        # smoothing: the output varies less than the input
        assert np.std(f(x, lens, hs)) < np.std(x)


def test_bessel_reduces_to_a_one_dimensional_solve():
    # an input that varies along z only: the 3-D solve equals the 1-D banded
    # solve of (1 - l_z^2 D_zz) with zero-flux ends
    rng = np.random.default_rng(4)
    nz, lz, hz = 11, 25.0, 10.0
    col = rng.standard_normal(nz)
    g = np.broadcast_to(col[:, None, None], (nz, 5, 6)).copy()
    u = smooth.bessel_filter(g, (20.0, 20.0, lz), (10.0, 10.0, hz))
    r = (lz / hz) ** 2
    ab = np.zeros((3, nz))
    ab[0, 1:] = -r
    ab[2, :-1] = -r
    ab[1, :] = 1 + 2 * r
    ab[1, 0] = ab[1, -1] = 1 + r
    ref = scipy.linalg.solve_banded((1, 1), ab, col)
    assert np.max(np.abs(u - ref[:, None, None])) <= 1e-12


def test_laplace_is_separable_product_of_axis_filters():
    # filtering a separable input f(x) g(y) h(z) gives the product of the
    # three 1-D filtered factors
    rng = np.random.default_rng(5)
    fx, fy, fz = rng.standard_normal(8), rng.standard_normal(6), rng.standard_normal(5)
    g = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    lens, hs = (15.0, 25.0, 35.0), (10.0, 10.0, 10.0)
    u = smooth.laplace_filter(g, lens, hs)
    ux = smooth.laplace_filter(fx[None, None, :], (lens[0], 0, 0), hs)[0, 0]
    uy = smooth.laplace_filter(fy[None, :, None], (0, lens[1], 0), hs)[0, :, 0]
    uz = smooth.laplace_filter(fz[:, None, None], (0, 0, lens[2]), hs)[:, 0, 0]
    assert np.allclose(u, uz[:, None, None] * uy[None, :, None] * ux[None, None, :],
                       rtol=1e-12, atol=1e-14)
