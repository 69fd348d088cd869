"""Limited-memory BFGS with bounds (L-BFGS-B) for the FWI loop.

The paper's FWI optimizer is L-BFGS-b with four bound types (none, lower,
both, upper; §2.1 and the FWI parameter table of §2.2.1), citing Byrd, Lu,
Nocedal and Zhu (1995).  This module follows that method:

1. the generalized Cauchy point: the first local minimizer of the quadratic
   model m(x + dx) = g'dx + 1/2 dx'B dx along the projected path
   P(x + t d0), d0 = -B0^-1 g, found by walking the breakpoints where
   coordinates reach their bounds, in increasing t;
2. subspace minimization: with the variables at a bound in the Cauchy point
   held fixed, the unconstrained minimizer of the model over the free ones
   (the direct primal method, B restricted to them inverted by the
   Sherman-Morrison-Woodbury formula), truncated to stay in the box;
3. a backtracking line search on the segment from x to that point, which is
   feasible, so the sufficient-decrease test uses the exact slope g'd.

B is the compact limited-memory BFGS matrix B = B0 - W M W' with
W = [Y, B0 S] and M = [[-D, L'], [L, S'B0 S]]^-1 (D = diag(s_i'y_i), L the
strictly lower part of S'Y).  B0 is diagonal: theta / p with p a positive
diagonal preconditioner (for FWI the illumination compensation, an
approximate inverse Hessian) and theta = y'p y / s'y from the latest pair,
so that with no bounds and p = 1 the step is the textbook L-BFGS step.

Vectors are flat torch tensors (any device); small matrices are FP64 numpy.
Inner products are taken in FP64.
"""

from __future__ import annotations

from typing import Callable, List, Optional, Tuple

import numpy as np


def _t():
    import torch
    return torch


def project(x, lower, upper):
    """Clamp to the box; lower / upper are tensors of x's shape or None."""
    torch = _t()
    if lower is not None:
        x = torch.maximum(x, lower)
    if upper is not None:
        x = torch.minimum(x, upper)
    return x


def projected_gradient(x, g, lower, upper):
    """P(x - g) - x: zero exactly at a first-order (KKT) point of the box."""
    return project(x - g, lower, upper) - x


class LBFGSB:
    """Direction computation and curvature-pair memory of L-BFGS-B."""

    def __init__(self, lower=None, upper=None, memory: int = 5):
        self.lower, self.upper = lower, upper
        self.m = int(memory)
        self.S: List = []
        self.Y: List = []

    # -- memory ---------------------------------------------------------------
    def update(self, s, y) -> bool:
        """Add the pair (s, y) if it has positive curvature; returns whether."""
        torch = _t()
        sy = float(torch.sum(s.double() * y.double()))
        ns = float(torch.linalg.vector_norm(s.double()))
        ny = float(torch.linalg.vector_norm(y.double()))
        if not (sy > 1e-10 * ns * ny):
            return False
        self.S.append(s.clone())
        self.Y.append(y.clone())
        if len(self.S) > self.m:
            self.S.pop(0)
            self.Y.pop(0)
        return True

    def reset(self):
        self.S, self.Y = [], []

    # -- the compact matrix ---------------------------------------------------
    def _compact(self, b):
        """(Sd, Yd, M) with Sd, Yd the stacked pairs [k][n] in FP64 and M the
        2k x 2k middle matrix for B0 = diag(b)."""
        torch = _t()
        Sd = torch.stack([s.reshape(-1).double() for s in self.S])
        Yd = torch.stack([y.reshape(-1).double() for y in self.Y])
        SY = (Sd @ Yd.T).cpu().numpy()
        SBS = ((Sd * b) @ Sd.T).cpu().numpy()
        k = len(self.S)
        D = np.diag(np.diag(SY))
        L = np.tril(SY, -1)
        mid = np.block([[-D, L.T], [L, SBS]])
        return Sd, Yd, np.linalg.inv(mid)

    # -- one direction ----------------------------------------------------------
    def direction(self, x, g, p=None, theta: Optional[float] = None):
        """Point xbar in the box such that xbar - x is the L-BFGS-B search
        direction at x (gradient g).  p: positive diagonal preconditioner (the
        inverse of B0 up to theta; None = 1); theta: B0 = theta / p (None =
        from the latest pair, 1 without pairs)."""
        torch = _t()
        shape = x.shape
        xv, gv = x.reshape(-1).double(), g.reshape(-1).double()
        pv = torch.ones_like(xv) if p is None else p.reshape(-1).double()
        lo = None if self.lower is None else self.lower.reshape(-1).double()
        hi = None if self.upper is None else self.upper.reshape(-1).double()
        k = len(self.S)
        if theta is None:
            if k:
                y = self.Y[-1].reshape(-1).double()
                s = self.S[-1].reshape(-1).double()
                theta = float(torch.sum(y * pv * y)) / float(torch.sum(s * y))
            else:
                theta = 1.0
        b = theta / pv                                   # B0 = diag(b)
        if k:
            Sd, Yd, M = self._compact(b)
        d0 = -gv / b                                     # Cauchy path direction

        # breakpoints t_i where coordinate i reaches its bound along x + t d0
        inf = torch.full_like(xv, float("inf"))
        tb = inf.clone()
        if lo is not None:
            neg = d0 < 0
            tb = torch.where(neg, (lo - xv) / torch.where(neg, d0, -1.0), tb)
        if hi is not None:
            pos = d0 > 0
            tb = torch.where(pos, (hi - xv) / torch.where(pos, d0, 1.0), tb)
        tb = torch.clamp(tb, min=0.0)
        d = torch.where(tb > 0, d0, torch.zeros_like(d0))

        def wT(v):   # W' v = [Y v ; (b S) v]
            return np.concatenate([(Yd @ v).cpu().numpy(), (Sd @ (b * v)).cpu().numpy()])

        fp = float(torch.sum(gv * d))
        fpp = float(torch.sum(b * d * d))
        if k:
            pvec = wT(d)
            fpp -= float(pvec @ M @ pvec)
            c = np.zeros(2 * k)
        t_old = 0.0
        # walk the finite breakpoints in increasing order, a batch at a time
        order = torch.argsort(tb)
        finite = int(torch.isfinite(tb).sum())
        pos_ = int((tb == 0).sum())   # already at a bound along d0: not part of the path
        done = False
        while pos_ < finite and not done:
            idx = order[pos_:min(finite, pos_ + 256)]
            t_h = tb[idx].cpu().numpy()
            g_h = gv[idx].cpu().numpy()
            d_h = d[idx].cpu().numpy()
            b_h = b[idx].cpu().numpy()
            x_h = xv[idx].cpu().numpy()
            if k:
                w_h = np.concatenate([Yd[:, idx].T.cpu().numpy(),
                                      (Sd[:, idx] * b[idx]).T.cpu().numpy()], axis=1)
            for j in range(len(idx)):
                dt = t_h[j] - t_old
                dt_min = -fp / fpp if fpp > 0 else float("inf")
                if dt_min < dt:
                    done = True
                    break
                # coordinate hits its bound at t_h[j]
                gb, db, bb = g_h[j], d_h[j], b_h[j]
                zb = t_h[j] * db           # x^cp_b - x_b
                fp = fp + dt * fpp
                fpp_next = fpp - bb * db * db
                if k:
                    c = c + dt * pvec
                    wb = w_h[j]
                    Mc, Mp, Mw = M @ c, M @ pvec, M @ wb
                    fp += -gb * db - db * (bb * zb - wb @ Mc)
                    fpp_next += 2.0 * db * (wb @ Mp) - db * db * (wb @ Mw)
                    pvec = pvec - db * wb
                else:
                    fp += -gb * db - db * bb * zb
                fpp = fpp_next
                t_old = t_h[j]
            else:
                pos_ += len(idx)
                continue
        dt_min = max(-fp / fpp, 0.0) if fpp > 0 else 0.0
        t_cp = t_old + dt_min
        xcp = project(xv + t_cp * d0, lo, hi)

        # subspace minimization over the variables not at a bound in xcp
        free = torch.ones_like(xv, dtype=torch.bool)
        if lo is not None:
            free &= xcp > lo
        if hi is not None:
            free &= xcp < hi
        dx = xcp - xv
        r = gv + b * dx
        if k:
            cc = wT(dx)
            Wc = M @ cc
            r = r - (Yd.T @ torch.from_numpy(Wc[:k]).to(Yd) +
                     b * (Sd.T @ torch.from_numpy(Wc[k:]).to(Sd)))
        r = torch.where(free, r, torch.zeros_like(r))
        if k:
            fm = free.double()
            Yf, Sf = Yd * fm, Sd * fm * b           # rows of W on the free set
            K = np.block([[(Yf @ (Yd / b).T).cpu().numpy(), (Yf @ Sd.T).cpu().numpy()],
                          [(Sf @ (Yd / b).T).cpu().numpy(), (Sf @ Sd.T).cpu().numpy()]])
            v = np.concatenate([((Yd * fm) @ (r / b)).cpu().numpy(),
                                ((Sd * fm) @ r).cpu().numpy()])
            u = np.linalg.solve(np.eye(2 * k) - M @ K, M @ v)
            Wu = Yd.T @ torch.from_numpy(u[:k]).to(Yd) + b * (Sd.T @ torch.from_numpy(u[k:]).to(Sd))
            du = -(r + Wu) / b
        else:
            du = -r / b
        du = torch.where(free, du, torch.zeros_like(du))
        # largest alpha <= 1 keeping xcp + alpha du in the box
        alpha = 1.0
        if lo is not None:
            m_ = du < 0
            if bool(m_.any()):
                alpha = min(alpha, float(torch.min((lo - xcp)[m_] / du[m_])))
        if hi is not None:
            m_ = du > 0
            if bool(m_.any()):
                alpha = min(alpha, float(torch.min((hi - xcp)[m_] / du[m_])))
        alpha = max(alpha, 0.0)
        xbar = xcp + alpha * du
        return xbar.to(x.dtype).reshape(shape)


def minimize(fun: Callable, x0, lower=None, upper=None, *, memory: int = 5,
             max_iter: int = 200, pgtol: float = 1e-8, ftol: float = 1e-15,
             precond: Optional[Callable] = None) -> Tuple[object, float, object, int]:
    """Minimize fun(x) -> (f, g) over lower <= x <= upper from x0.

    precond(x, g) -> p (positive diagonal, approximate inverse Hessian) or
    None.  Stops when max|P(x - g) - x| <= pgtol, when a step lowers f by
    less than ftol * max(1, |f|), or after max_iter iterations.  Returns
    (x, f, g, iterations)."""
    torch = _t()
    opt = LBFGSB(lower, upper, memory)
    x = project(x0.clone(), lower, upper)
    f, g = fun(x)
    for it in range(max_iter):
        if float(projected_gradient(x, g, lower, upper).abs().max()) <= pgtol:
            return x, f, g, it
        p = precond(x, g) if precond is not None else None
        xbar = opt.direction(x, g, p)
        d = xbar - x
        gd = float(torch.sum(g.double() * d.double()))
        if not (gd < 0):
            if not opt.S:
                return x, f, g, it
            opt.reset()
            continue
        lam, ok = 1.0, False
        for _ in range(30):
            xt = x + lam * d
            ft, gt = fun(xt)
            if ft <= f + 1e-4 * lam * gd:
                ok = True
                break
            lam *= 0.5
        if not ok:
            if not opt.S:
                return x, f, g, it
            opt.reset()
            continue
        opt.update(xt - x, gt - g)
        done = f - ft <= ftol * max(1.0, abs(f))
        x, f, g = xt, ft, gt
        if done:
            return x, f, g, it + 1
    return x, f, g, max_iter
