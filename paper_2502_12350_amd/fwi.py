"""Full waveform inversion on top of the library (paper Alg. 2, FWI::run).

* ``WaveFn`` — a ``torch.autograd.Function`` from a velocity volume to the
  total misfit of a set of shots.  Its forward pass runs the library's
  one-shot gradient for every shot (forward sweep, misfit, adjoint sweep and
  imaging, Alg. 3) and keeps the accumulated dJ/dv for the backward pass, so
  ``loss.backward()`` costs nothing more.
* ``fwi`` — the outer loop of Alg. 2 with two model-update rules:
  steepest descent on the illumination-compensated gradient
  g / (I + eps max I) with a quadratic line search (exact slope plus one
  trial misfit), projected onto the velocity bounds, and L-BFGS-B (the
  paper's L-BFGS-b, §2.1: generalized Cauchy point and subspace
  minimization, ``lbfgsb.py``) with velocity bounds as in the paper's
  example (2000 to 3500 m/s) and the same preconditioner in its initial
  matrix, with an Armijo backtracking line search on the feasible segment.
  Trial misfits use the library's forward-only misfit; every accepted point
  gets one gradient.

All wave-equation arithmetic runs in the HIP library; this module only
composes calls and does the O(model size) optimizer algebra in torch.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .api import GridSpec, Propagator
from .lbfgsb import LBFGSB


@dataclass
class Shots:
    """Acquisition: one wavelet, per-shot source positions, receivers and data."""
    wavelet: "object"                  # torch float32 [nt] on the device
    sources: np.ndarray                # [nshot][3] metres
    receivers: Sequence[np.ndarray]    # per shot [nrec][3] metres
    dobs: Sequence["object"]           # per shot torch float32 [nrec][nt] on the device

    def __len__(self):
        return len(self.sources)


def auto_checkpoint(prop: Propagator, nrec: int, fraction: float = 0.8):
    """Full storage when it fits in `fraction` of the free device memory,
    else binomial checkpointing sized to that memory (the paper's check_mem;
    on a CPML grid each checkpoint also holds the layer's memory variables,
    which the library counts)."""
    import torch
    free, _ = torch.cuda.mem_get_info(prop.device)
    if prop.workspace_bytes(nrec, "full") <= fraction * free:
        return "full"
    return ("revolve", 0, fraction)


class WaveFn:
    """Velocity -> total misfit over shots, differentiable through the library."""

    @staticmethod
    def apply(vel, prop: Propagator, grid: GridSpec, rho, shots: Shots, ckpt="auto",
              illum=None):
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, v):
                J, g = evaluate(prop, grid, v.detach(), rho, shots, ckpt=ckpt, illum=illum)
                ctx.save_for_backward(g)
                return J

            @staticmethod
            def backward(ctx, gout):
                (g,) = ctx.saved_tensors
                return gout.to(g.dtype) * g

        return _Fn.apply(vel)


def _save_shot_state(path, key, done, grad, misfit, illum):
    """Partial sums of one gradient evaluation after `done` shots."""
    import os
    tmp = path + ".tmp.npz"
    np.savez(tmp, key=np.array(key), done=np.int64(done), grad=grad.cpu().numpy(),
             misfit=np.float64(misfit.item()),
             illum=illum.cpu().numpy() if illum is not None else np.zeros(0, np.float32))
    os.replace(tmp, path)


def evaluate(prop: Propagator, grid: GridSpec, vel, rho, shots: Shots, ckpt="auto",
             illum=None, zero_top_planes: int = 0, smoothing=None, shot_state=None,
             shot_key: str = "", shot_hook=None):
    """(misfit, dJ/dv) summed over shots; illum (if given) accumulates sum (w^n)^2.
    smoothing = (mode, lengths) applies the paper's gradient smoothing ("laplace"
    or "bessel", lengths (x, y, z) in metres) before the top planes are zeroed
    (GradientPreconditioning, then ZeroesNearSurface, as in Alg. 3).

    shot_state: a file that receives the partial sums (gradient, misfit,
    illumination) after every shot, tagged with shot_key; an evaluation with
    the same key that finds it continues after the shots it holds, and ends
    with bitwise the sums of an uninterrupted one (shots are added in the same
    order).  shot_hook(shot_key, s), if given, is called after shot s."""
    import os
    import torch
    prop.set_model(grid, vel.contiguous(), rho)
    misfit = torch.zeros((), dtype=torch.float64, device=prop.device)
    grad = torch.zeros_like(vel)
    first = 0
    if shot_state is not None and os.path.exists(shot_state):
        with np.load(shot_state, allow_pickle=False) as z:
            if str(z["key"]) == shot_key:
                first = int(z["done"])
                grad.copy_(torch.from_numpy(z["grad"]))
                misfit.fill_(float(z["misfit"]))
                if illum is not None:
                    illum.copy_(torch.from_numpy(z["illum"]))
    for s in range(first, len(shots)):
        rec = shots.receivers[s]
        ck = auto_checkpoint(prop, len(rec)) if ckpt == "auto" else ckpt
        prop.gradient(shots.wavelet, shots.sources[s], rec, shots.dobs[s], ckpt=ck, grad=grad,
                      misfit=misfit, illum=illum)
        if shot_state is not None:
            _save_shot_state(shot_state, shot_key, s + 1, grad, misfit, illum)
        if shot_hook is not None:
            shot_hook(shot_key, s)
    if smoothing is not None:
        from .api import smooth
        mode, lengths = smoothing
        grad, _ = smooth(grad, mode, lengths, (grid.dx, grid.dy, grid.dz))
    if zero_top_planes:
        prop.gradient_finish(grad, zero_top_planes)
    return misfit, grad


def misfit_only(prop: Propagator, grid: GridSpec, vel, rho, shots: Shots):
    """Total misfit from forward sweeps only."""
    import torch
    prop.set_model(grid, vel.contiguous(), rho)
    misfit = torch.zeros((), dtype=torch.float64, device=prop.device)
    for s in range(len(shots)):
        prop.forward_misfit(shots.wavelet, shots.sources[s], shots.receivers[s], shots.dobs[s],
                            misfit=misfit)
    return misfit


def illumination_compensate(grad, illum, eps: float = 1.0e-3):
    """g / (I + eps * max I): the plain illumination-compensated gradient."""
    return grad / (illum + eps * illum.max())


@dataclass
class FwiTrace:
    method: str
    gpu_seconds: List[float] = field(default_factory=list)
    misfit: List[float] = field(default_factory=list)
    n_gradients: int = 0
    n_misfits: int = 0
    n_network: int = 0   # accepted steps along the learned direction

    def record(self, t: float, J: float):
        self.gpu_seconds.append(t)
        self.misfit.append(J)

    def misfit_cut_per_gpu_s(self) -> float:
        """Relative misfit reduction per GPU-second over the whole run."""
        if len(self.misfit) < 2 or self.gpu_seconds[-1] <= 0:
            return 0.0
        return (1.0 - self.misfit[-1] / self.misfit[0]) / self.gpu_seconds[-1]

    def time_to_reach(self, rel_misfit: float) -> Optional[float]:
        """GPU-seconds until misfit <= rel_misfit * initial misfit."""
        for t, J in zip(self.gpu_seconds, self.misfit):
            if J <= rel_misfit * self.misfit[0]:
                return t
        return None


def _dot(a, b) -> float:
    """Inner product in FP64 (gradients of the misfit are ~1e-20 and smaller)."""
    import torch
    return float(torch.sum(a.double() * b.double()))


def _quadratic_step(J_at, v, d, J0, gd, a1, bounds):
    """Step length along d from the quadratic J(a) ~ J0 + gd a + c a^2 fixed by
    the exact slope gd = <g, d> and one trial J(a1) (backtracking first if the
    trial does not lower J); returns the better of the evaluated steps, or None."""
    J1 = J_at(_project(v + a1 * d, bounds))
    for _ in range(6):
        if J1 < J0:
            break
        a1 *= 0.25
        J1 = J_at(_project(v + a1 * d, bounds))
    best = (J1, a1)
    c = (J1 - J0 - gd * a1) / (a1 * a1)
    if c > 0:
        a_star = min(-gd / (2.0 * c), 50.0 * a1)
        if abs(a_star - a1) > 0.05 * a1:
            best = min(best, (J_at(_project(v + a_star * d, bounds)), a_star))
    elif J1 < J0:  # no positive curvature seen: try a longer step
        best = min(best, (J_at(_project(v + 4.0 * a1 * d, bounds)), 4.0 * a1))
    return best[1] if best[0] < J0 else None


def _span_step(J_at, v, d1, d2, J0, s1, s2, a1, b1, bounds):
    """Step in the plane spanned by d1 (the plain direction) and d2 (the
    network's): the quadratic J(a, b) ~ J0 + s1 a + s2 b + 1/2 [a b] H [a b]'
    fixed by the exact slopes and three trials (a1, 0), (0, b1), (a1, b1),
    minimized (within 4 trial lengths per axis) and evaluated; returns the
    best evaluated step vector, or None if no trial lowers J."""
    tried = []

    def trial(x, y):
        step = x * a1 * d1 + y * b1 * d2
        tried.append((J_at(_project(v + step, bounds)), x, y))
        return tried[-1][0]

    J10, J01, J11 = trial(1.0, 0.0), trial(0.0, 1.0), trial(1.0, 1.0)
    S1, S2 = s1 * a1, s2 * b1                  # slopes per trial length
    A = 2.0 * (J10 - J0 - S1)
    C = 2.0 * (J01 - J0 - S2)
    B = J11 - J10 - J01 + J0
    det = A * C - B * B
    if A > 0 and C > 0 and det > 0:
        x = (-C * S1 + B * S2) / det
        y = (B * S1 - A * S2) / det
        x, y = min(max(x, -1.0), 4.0), min(max(y, -1.0), 4.0)
        if min(abs(x - px) + abs(y - py) for _, px, py in tried) > 0.05:
            trial(x, y)
    Jb, x, y = min(tried)
    return (x * a1 * d1 + y * b1 * d2) if Jb < J0 else None


def _project(v, bounds):
    """Clamp to the velocity bounds: None, or (lower, upper) where either side
    may be None (the paper's L-BFGS-b bound types: unbounded, lower only,
    both, upper only)."""
    if bounds is None or (bounds[0] is None and bounds[1] is None):
        return v
    return v.clamp(bounds[0], bounds[1])


def _save_state(path, it, v, g, illum, J, S, Y, dv_prev, trace):
    """Everything the loop needs to continue after iteration it - 1."""
    import os
    tmp = path + ".tmp.npz"
    np.savez(tmp, it=np.int64(it), v=v.cpu().numpy(), g=g.cpu().numpy(),
             illum=illum.cpu().numpy(), J=np.float64(J),
             S=np.stack([s.cpu().numpy() for s in S]) if S else np.zeros((0,) + tuple(v.shape)),
             Y=np.stack([y.cpu().numpy() for y in Y]) if Y else np.zeros((0,) + tuple(v.shape)),
             dv_prev=np.float64(np.nan if dv_prev is None else dv_prev),
             misfit=np.asarray(trace.misfit, dtype=np.float64),
             gpu_seconds=np.asarray(trace.gpu_seconds, dtype=np.float64),
             counts=np.asarray([trace.n_gradients, trace.n_misfits, trace.n_network]))
    os.replace(tmp, path)  # a crash while writing leaves the previous state


def _load_state(path, device):
    import torch
    with np.load(path, allow_pickle=False) as z:
        st = {k: z[k] for k in z.files}
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    dv = float(st["dv_prev"])
    return (int(st["it"]), t(st["v"]), t(st["g"]), t(st["illum"]), float(st["J"]),
            [t(a) for a in st["S"]], [t(a) for a in st["Y"]], None if np.isnan(dv) else dv,
            st["misfit"].tolist(), st["gpu_seconds"].tolist(), st["counts"].tolist())


def fwi(prop: Propagator, grid: GridSpec, v0, rho, shots: Shots, *, n_iter: int = 10,
        method: str = "sd", bounds: Optional[Tuple[float, float]] = None,
        max_rel_step: float = 0.02, eps_illum: float = 1.0e-3, memory: int = 5,
        ckpt="auto", zero_top_planes: int = 0, precond=None, progress=None, smoothing=None,
        state_file: Optional[str] = None, shot_hook=None):
    """Alg. 2: repeat {gradient, model update} for n_iter iterations.

    method "sd": steepest descent on the illumination-compensated gradient;
    "lbfgs": L-BFGS-B with that preconditioner in B0 = theta / P; "cnn": steepest
    descent along the learned preconditioner's direction (`precond`, a
    precond.Preconditioner), falling back to the illumination-compensated
    gradient when the network's direction does not descend; "cnn_span": a
    step in the plane of both directions, from a two-dimensional quadratic
    fit of three trial misfits and the exact slopes.

    Returns (final velocity, FwiTrace).  GPU-seconds are wall time of the
    synchronised GPU work (the device runs nothing else meanwhile), including
    the network's inference.  progress(iteration, misfit, gpu_seconds, model),
    if given, is called after every iteration.  smoothing = (mode, lengths)
    smooths every gradient as the paper's GradientPreconditioning does.

    state_file: fault tolerance in the manner of the paper's DeLIA restart.
    The loop state (model, gradient, illumination, L-BFGS pairs, step memory,
    history) is written there after every iteration, atomically; if the file
    exists when fwi starts, the run continues from it and ends exactly as an
    uninterrupted run would.  Within a gradient evaluation the partial sums
    are also kept after every shot (state_file + ".shot.npz", keyed by the
    iteration), so a failure in the middle of one costs only the shot that
    was running.  shot_hook(key, s) is called after each shot (monitoring;
    the tests use it to fail on purpose).
    """
    import torch
    trace = FwiTrace(method)
    clock = [0.0]

    def timed(fn, *a, **k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn(*a, **k)
        torch.cuda.synchronize()
        clock[0] += time.perf_counter() - t0
        return out

    import os
    resume = state_file is not None and os.path.exists(state_file)
    v = _project(v0.clone(), bounds)
    illum = torch.zeros_like(v)

    shot_state = None if state_file is None else state_file + ".shot.npz"

    def grad_at(vv, key):
        illum.zero_()
        J, g = timed(evaluate, prop, grid, vv, rho, shots, ckpt=ckpt, illum=illum,
                     zero_top_planes=zero_top_planes, smoothing=smoothing,
                     shot_state=shot_state, shot_key=key, shot_hook=shot_hook)
        trace.n_gradients += 1
        return float(J.item()), g

    def J_at(vv):
        trace.n_misfits += 1
        return float(timed(misfit_only, prop, grid, vv, rho, shots).item())

    S, Y = [], []
    lo_b = None if bounds is None or bounds[0] is None else torch.full_like(v, float(bounds[0]))
    hi_b = None if bounds is None or bounds[1] is None else torch.full_like(v, float(bounds[1]))
    opt = LBFGSB(lo_b, hi_b, memory)
    dv_prev = None  # largest model change of the last accepted steepest-descent step
    start = 0
    if resume:
        (start, v, g, il, J, S, Y, dv_prev, trace.misfit, trace.gpu_seconds,
         (trace.n_gradients, trace.n_misfits, trace.n_network)) = _load_state(state_file, v.device)
        illum.copy_(il)
        clock[0] = trace.gpu_seconds[-1]
    else:
        J, g = grad_at(v, "0")
        trace.record(clock[0], J)
        if state_file is not None:
            _save_state(state_file, 0, v, g, illum, J, S, Y, dv_prev, trace)

    def first_step(d, warm: bool = True):
        """Initial trial step: a largest model change of max_rel_step * max|v|
        (the default), or with `warm` twice the last accepted change but at
        least 5 % of the default."""
        dmax = float(d.abs().max())
        default = max_rel_step * float(v.abs().max())
        if dv_prev is None or not warm:
            return default / dmax
        return max(2.0 * dv_prev, 0.05 * default) / dmax

    for it in range(start, n_iter):
        if progress and it > start:
            progress(it - 1, J, clock[0], v)
        P = 1.0 / (illum + eps_illum * illum.max())      # preconditioner (diagonal)
        used = False                                       # step along the network's direction
        if method == "lbfgs":
            # L-BFGS-B: the generalized Cauchy point and subspace minimization
            # with B0 = theta / P; without pairs theta makes the full Cauchy
            # step change the model by at most max_rel_step * max|v|
            opt.S, opt.Y = S, Y
            theta = None
            if not S:
                theta = float((P * g).abs().max()) / (max_rel_step * float(v.abs().max()))
            d = opt.direction(v, g, P, theta) - v
            alpha0 = 1.0
        elif method == "cnn":
            d, used = timed(precond.direction, g, illum, eps_illum)
            alpha0 = first_step(d)
        elif method == "cnn_span":
            d2, used = timed(precond.direction, g, illum, eps_illum)
            d = -P * g
            alpha0 = first_step(d)
        else:
            d = -P * g
            alpha0 = first_step(d)
        gd = _dot(g, d)
        if gd >= 0 and method == "lbfgs" and S:  # not a descent direction: drop the pairs
            S, Y = [], []
            opt.S, opt.Y = S, Y
            theta = float((P * g).abs().max()) / (max_rel_step * float(v.abs().max()))
            d = opt.direction(v, g, P, theta) - v
            gd = _dot(g, d)
        if gd >= 0 and method != "lbfgs":  # restart from the preconditioned gradient
            S, Y = [], []
            d = -P * g
            alpha0 = first_step(d)
            gd = _dot(g, d)
            used = False
        if gd >= 0:  # a first-order point of the box: nothing left to do
            trace.record(clock[0], J)
            if state_file is not None:
                _save_state(state_file, it + 1, v, g, illum, J, S, Y, dv_prev, trace)
            continue
        if method == "lbfgs":
            # Armijo backtracking on the segment from v to the L-BFGS-B point,
            # which lies in the box: the slope <g, d> is exact for every trial
            alpha, ok = alpha0, False
            for _ in range(10):
                Jt = J_at(v + alpha * d)
                if Jt <= J + 1e-4 * alpha * gd:
                    ok = True
                    break
                alpha *= 0.5
            if not ok:
                S, Y = [], []
                trace.record(clock[0], J)
                if state_file is not None:
                    _save_state(state_file, it + 1, v, g, illum, J, S, Y, dv_prev, trace)
                continue
        elif method == "cnn_span" and used:
            step = _span_step(J_at, v, d, d2, J, gd, _dot(g, d2), alpha0, first_step(d2),
                              bounds)
            if step is None:  # no decrease in the plane: the plain direction alone
                alpha = _quadratic_step(J_at, v, d, J, gd, first_step(d, warm=False), bounds)
                used = False
            else:
                d, alpha = step, 1.0
            if alpha is None:
                trace.record(clock[0], J)
                if state_file is not None:
                    _save_state(state_file, it + 1, v, g, illum, J, S, Y, dv_prev, trace)
                continue
            trace.n_network += int(used)
            dv_prev = alpha * float(d.abs().max())
        else:
            alpha = _quadratic_step(J_at, v, d, J, gd, alpha0, bounds)
            if alpha is None and dv_prev is not None:  # warm start failed: default step
                alpha = _quadratic_step(J_at, v, d, J, gd, first_step(d, warm=False), bounds)
            if alpha is None and used:  # the network's direction failed: plain one
                d = -P * g
                gd = _dot(g, d)
                used = False
                alpha = _quadratic_step(J_at, v, d, J, gd, first_step(d, warm=False), bounds)
            if alpha is None:  # no decrease found: stop updating
                trace.record(clock[0], J)
                if state_file is not None:
                    _save_state(state_file, it + 1, v, g, illum, J, S, Y, dv_prev, trace)
                continue
            trace.n_network += int(used)
            dv_prev = alpha * float(d.abs().max())
        v_new = v + alpha * d if method == "lbfgs" else _project(v + alpha * d, bounds)
        J_new, g_new = grad_at(v_new, str(it + 1))
        if method == "lbfgs":
            opt.S, opt.Y = S, Y
            opt.update(v_new - v, g_new - g)
            S, Y = opt.S, opt.Y
        v, J, g = v_new, J_new, g_new
        trace.record(clock[0], J)
        if state_file is not None:
            _save_state(state_file, it + 1, v, g, illum, J, S, Y, dv_prev, trace)
    if progress:
        progress(n_iter - 1, J, clock[0], v)
    return v, trace
