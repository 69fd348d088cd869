"""The FWI loop's L-BFGS-B (host logic, CPU): on bound-constrained problems
it must reach a first-order (KKT) point with the right active set, agree with
SciPy's L-BFGS-B, reduce to plain L-BFGS without bounds, and handle the four
bound types of the paper (none, lower, both, upper)."""

import numpy as np
import pytest
import torch
from scipy.optimize import minimize as sp_minimize

from paper_2502_12350_amd.lbfgsb import LBFGSB, minimize, projected_gradient


def _quadratic(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.geomspace(1.0, cond, n)) @ Q.T
    c = rng.standard_normal(n) * 3.0
    return A, c


def _fun(A, c):
    At = torch.from_numpy(A)
    ct = torch.from_numpy(c)

    def f(x):
        g = At @ x - ct
        return float(0.5 * x @ (At @ x) - ct @ x), g
    return f


def _kkt(x, g, lo, hi, tol):
    """First-order conditions of min f on [lo, hi]: the gradient vanishes on
    free coordinates, points inward (g >= 0) at a lower bound, outward
    (g <= 0) at an upper bound."""
    at_lo = np.isclose(x, lo, atol=1e-12, rtol=0) if lo is not None else np.zeros(len(x), bool)
    at_hi = np.isclose(x, hi, atol=1e-12, rtol=0) if hi is not None else np.zeros(len(x), bool)
    free = ~(at_lo | at_hi)
    assert np.all(np.abs(g[free]) <= tol)
    assert np.all(g[at_lo] >= -tol)
    assert np.all(g[at_hi] <= tol)
    return at_lo, at_hi


@pytest.mark.parametrize("kind", ["both", "lower", "upper", "none"])
def test_bound_constrained_quadratic_matches_scipy(kind):
    n = 60
    A, c = _quadratic(n, seed=3)
    lo = np.full(n, -0.4) if kind in ("both", "lower") else None
    hi = np.full(n, 0.5) if kind in ("both", "upper") else None
    f = _fun(A, c)
    x0 = np.zeros(n)
    x, fx, g, it = minimize(f, torch.from_numpy(x0),
                            None if lo is None else torch.from_numpy(lo),
                            None if hi is None else torch.from_numpy(hi),
                            memory=7, max_iter=500, pgtol=1e-7, ftol=0.0)
    x, g = x.numpy(), g.numpy()
    at_lo, at_hi = _kkt(x, g, lo, hi, 1e-6)
    if kind != "none":
        assert at_lo.sum() + at_hi.sum() >= 5     # the bounds matter here
    bnds = [(None if lo is None else lo[i], None if hi is None else hi[i]) for i in range(n)]
    ref = sp_minimize(lambda v: (0.5 * v @ A @ v - c @ v, A @ v - c), x0, jac=True,
                      method="L-BFGS-B", bounds=bnds,
                      options=dict(maxiter=5000, ftol=1e-15, gtol=1e-12, maxcor=7))
    assert np.max(np.abs(x - ref.x)) <= 1e-6
    assert fx <= ref.fun + 1e-10 * abs(ref.fun)
    if kind != "none":
        ref_lo = np.isclose(ref.x, lo, atol=1e-9, rtol=0) if lo is not None else np.zeros(n, bool)
        ref_hi = np.isclose(ref.x, hi, atol=1e-9, rtol=0) if hi is not None else np.zeros(n, bool)
        assert np.array_equal(at_lo, ref_lo) and np.array_equal(at_hi, ref_hi)


def test_unbounded_step_is_the_lbfgs_two_loop_step():
    """Without bounds the direction equals the classic two-loop recursion
    with H0 = (s'y / y'p y) p."""
    rng = np.random.default_rng(1)
    n, m = 40, 4
    opt = LBFGSB(None, None, memory=m)
    A, _ = _quadratic(n, seed=2)
    for _ in range(m):
        s = rng.standard_normal(n)
        opt.update(torch.from_numpy(s), torch.from_numpy(A @ s))
    x = torch.from_numpy(rng.standard_normal(n))
    g = torch.from_numpy(rng.standard_normal(n))
    p = torch.from_numpy(rng.uniform(0.5, 2.0, n))
    d = (opt.direction(x, g, p) - x).numpy()
    # two-loop recursion
    S = [s.numpy() for s in opt.S]
    Y = [y.numpy() for y in opt.Y]
    q = g.numpy().copy()
    al = []
    for s, y in reversed(list(zip(S, Y))):
        a = (s @ q) / (y @ s)
        al.append(a)
        q -= a * y
    pn = p.numpy()
    r = (S[-1] @ Y[-1]) / (Y[-1] @ (pn * Y[-1])) * pn * q
    for (s, y), a in zip(zip(S, Y), reversed(al)):
        bta = (y @ r) / (y @ s)
        r += (a - bta) * s
    assert np.allclose(d, -r, rtol=1e-9, atol=1e-12)


def test_cauchy_point_on_a_diagonal_problem():
    """With no pairs and B0 = I, the generalized Cauchy point of
    g'dx + |dx|^2 / 2 on a box is the projection of x - g; the subspace step
    is then zero on every free coordinate."""
    x = torch.tensor([0.0, 0.0, 0.0, 0.5])
    g = torch.tensor([1.0, -3.0, 0.25, -1.0])
    lo = torch.tensor([-0.5, -1.0, -1.0, -1.0])
    hi = torch.tensor([1.0, 1.0, 1.0, 1.0])
    opt = LBFGSB(lo, hi)
    xbar = opt.direction(x, g)
    assert torch.allclose(xbar, torch.tensor([-0.5, 1.0, -0.25, 1.0]))


def test_kkt_of_the_result_with_a_diagonal_preconditioner():
    """A badly scaled quadratic with a diagonal preconditioner (the role the
    illumination plays in FWI): same minimizer, reached in fewer iterations."""
    n = 50
    rng = np.random.default_rng(8)
    scale = np.geomspace(1.0, 1e4, n)
    A0, c = _quadratic(n, seed=5, cond=5.0)
    A = A0 * np.sqrt(scale)[:, None] * np.sqrt(scale)[None, :]
    lo, hi = np.full(n, -0.01), np.full(n, 0.02)
    f = _fun(A, c)
    pre = torch.from_numpy(1.0 / np.diag(A))
    x1, _, g1, it1 = minimize(f, torch.zeros(n, dtype=torch.float64), torch.from_numpy(lo),
                              torch.from_numpy(hi), max_iter=2000, pgtol=1e-7, ftol=0.0,
                              precond=lambda x, g: pre)
    x2, _, _, it2 = minimize(f, torch.zeros(n, dtype=torch.float64), torch.from_numpy(lo),
                             torch.from_numpy(hi), max_iter=2000, pgtol=1e-7, ftol=0.0)
    _kkt(x1.numpy(), g1.numpy(), lo, hi, 1e-6)
    assert np.max(np.abs(x1.numpy() - x2.numpy())) <= 1e-6
    assert it1 < it2
    assert float(projected_gradient(x1, g1, torch.from_numpy(lo),
                                    torch.from_numpy(hi)).abs().max()) <= 1e-6
