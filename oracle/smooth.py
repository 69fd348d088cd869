"""FP64 oracle of the gradient-smoothing filters (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product library.
It shares no code with the GPU path.

The paper smooths every FWI gradient with a filter chosen by
`gradient_preconditioning_mode`: none, a Bessel filter or a Laplace filter,
with lengths l_x, l_y, l_z that default to twice the grid spacing (§2.2, FWI
parameters; the method is that of Trinh et al. 2017).  The paper gives no
formula; the readings (R24) are:

* Laplace filter: a separable exponential kernel, along each axis
  k(n) = (1 - a)/(1 + a) a^|n| with a = exp(-h / l).  Discretely this is the
  inverse of the tridiagonal operator T = [(1 + a^2) I - a (S + S^-1)] / (1 - a)^2
  (S the unit shift), whose end rows use a zero-flux (mirror) condition so that
  constants are kept; the filter applies T^-1 along x, then y, then z.
* Bessel filter: the inverse of the 3-D elliptic operator
  B = I - l_x^2 D_xx - l_y^2 D_yy - l_z^2 D_zz, D the 3-point second
  difference with zero-flux ends; its Green's function decays like
  exp(-r) / r in the scaled distance (the K_1/2 Bessel kernel), hence the
  name.  B is symmetric positive definite and keeps constants.

Volumes are [z][y][x]; lengths and spacings are (x, y, z) in metres.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


def _tri_laplace(n: int, a: float):
    """Banded form (solve_banded) of (1 - a)^2 T for a line of n points."""
    ab = np.zeros((3, n))
    ab[0, 1:] = -a
    ab[1, :] = 1.0 + a * a
    ab[2, :-1] = -a
    if n == 1:
        ab[1, 0] = (1.0 - a) ** 2
    else:
        ab[1, 0] = ab[1, -1] = 1.0 + a * a - a   # zero-flux ends
    return ab


def laplace_filter(g, lengths: Sequence[float], spacing: Sequence[float]) -> np.ndarray:
    """Separable exponential smoothing (R24), x then y then z."""
    u = np.asarray(g, dtype=np.float64).copy()
    for axis, l, h in ((2, lengths[0], spacing[0]), (1, lengths[1], spacing[1]),
                       (0, lengths[2], spacing[2])):
        if l <= 0:
            continue
        a = float(np.exp(-h / l))
        n = u.shape[axis]
        ab = _tri_laplace(n, a)
        moved = np.moveaxis(u, axis, 0).reshape(n, -1)
        sol = scipy.linalg.solve_banded((1, 1), ab, (1.0 - a) ** 2 * moved)
        u = np.moveaxis(sol.reshape(np.moveaxis(u, axis, 0).shape), 0, axis)
    return np.ascontiguousarray(u)


def _second_difference(n: int, h: float):
    """Sparse 3-point D with zero-flux ends (a mirror ghost)."""
    if n == 1:
        return scipy.sparse.csr_matrix((1, 1))
    main = -2.0 * np.ones(n)
    main[0] = main[-1] = -1.0
    off = np.ones(n - 1)
    return scipy.sparse.diags([off, main, off], [-1, 0, 1], format="csr") / (h * h)


def bessel_operator(shape, lengths: Sequence[float], spacing: Sequence[float]):
    """B = I - sum_d l_d^2 D_dd as a sparse matrix on [z][y][x] (C order)."""
    nz, ny, nx = shape
    I = [scipy.sparse.identity(m, format="csr") for m in (nz, ny, nx)]
    Dx = _second_difference(nx, spacing[0])
    Dy = _second_difference(ny, spacing[1])
    Dz = _second_difference(nz, spacing[2])
    kron = scipy.sparse.kron
    L = (lengths[0] ** 2 * kron(kron(I[0], I[1]), Dx)
         + lengths[1] ** 2 * kron(kron(I[0], Dy), I[2])
         + lengths[2] ** 2 * kron(kron(Dz, I[1]), I[2]))
    return (scipy.sparse.identity(nz * ny * nx, format="csr") - L).tocsc()


def bessel_filter(g, lengths: Sequence[float], spacing: Sequence[float]) -> np.ndarray:
    """u = B^-1 g (R24), solved directly (small volumes only)."""
    g = np.asarray(g, dtype=np.float64)
    B = bessel_operator(g.shape, lengths, spacing)
    return scipy.sparse.linalg.spsolve(B, g.ravel()).reshape(g.shape)
