"""Checks at the full bench size (576^3 padded, variable density, 2000 steps,
65,536 receivers), in the launch configuration bench.py times.  The FP64
oracle cannot run 2000 steps at this size, so these are (a) properties that
hold at any size: determinism, reciprocity, zero misfit at the true model, the
trace at a receiver staying finite and bounded, and the gradient's directional
derivative against central differences of the misfit under binomial
checkpointing; and (b) the oracle's own step applied to the GPU's states:
the last of the 2000 steps recomputed in FP64 from the GPU's two previous
states, over three 96-plane slabs of the model (top, with the sponge, source
and receivers; middle; bottom, with the other sponge face, which the wave
has barely reached), every x and y tile."""

import numpy as np
import pytest

import oracle
import seisgen
from gpu_util import gpu_or_skip, rel_l2, say

pytestmark = pytest.mark.gpu

_C2 = {}


def _c2():
    if "w" not in _C2:
        _C2["w"] = seisgen.workload("c2")
    return _C2["w"]


def test_c2_forward_deterministic_and_zero_self_misfit():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, Propagator
    w = _c2()
    say(f"[c2 full size] padded {w.padded_shape} nt {w.nt} nrec {len(w.receivers)}")
    P = Propagator(0)
    P.set_model(GridSpec(**w.grid_kwargs()), torch.from_numpy(w.vel).cuda(),
                torch.from_numpy(w.rho).cuda())
    wav = torch.from_numpy(w.wavelet).cuda()
    a = P.forward(wav, w.sources[0], w.receivers).clone()
    b = P.forward(wav, w.sources[0], w.receivers)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert bool(torch.isfinite(a).all())
    assert float(a.abs().max()) > 0
    J = P.forward_misfit(wav, w.sources[0], w.receivers, a)
    assert float(J.item()) == 0.0
    # the trace at the receiver above the source carries the direct wave
    i = int(np.argmin(np.linalg.norm(w.receivers[:, :2] - w.sources[0][:2], axis=1)))
    assert float(a[i].abs().max()) == pytest.approx(float(a.abs().max()), rel=0.5)


def test_c2_reciprocity_full_size():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, Propagator
    w = _c2()
    say("[c2 reciprocity]")
    P = Propagator(0)
    P.set_model(GridSpec(**w.grid_kwargs()), torch.from_numpy(w.vel).cuda(),
                torch.from_numpy(w.rho).cuda())
    wav = torch.from_numpy(w.wavelet).cuda()
    na, nb = (150, 200, 60), (330, 290, 140)   # (ix, iy, iz), far from each other
    xa = w.nodes_to_metres([na])
    xb = w.nodes_to_metres([nb])
    tab = P.forward(wav, xa[0], xb)[0].double().cpu().numpy()
    tba = P.forward(wav, xb[0], xa)[0].double().cpu().numpy()
    wa = float(w.rho[na[2], na[1], na[0]]) * float(w.vel[na[2], na[1], na[0]]) ** 2
    wb = float(w.rho[nb[2], nb[1], nb[0]]) * float(w.vel[nb[2], nb[1], nb[0]]) ** 2
    lhs, rhs = tab * wa, tba * wb
    err = np.linalg.norm(lhs - rhs) / np.linalg.norm(lhs)
    say(f"  reciprocity rel-L2 {err:.2e}")
    assert np.linalg.norm(lhs) > 0
    assert err <= 1e-4


def _states(w, nt):
    """GPU states (w^nt, w^(nt-1)) after nt steps of the workload."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, Propagator
    P = Propagator(0)
    kw = w.grid_kwargs()
    kw["nt"] = nt
    P.set_model(GridSpec(**kw), torch.from_numpy(w.vel).cuda(), torch.from_numpy(w.rho).cuda())
    _, fin = P.forward(torch.from_numpy(w.wavelet[:nt].copy()).cuda(), w.sources[0],
                       w.receivers, final=True)
    torch.cuda.synchronize()
    out = fin.cpu().numpy()
    del P, fin
    torch.cuda.empty_cache()
    return out[0], out[1]


def test_c2_last_step_matches_the_oracle_step_full_size():
    gpu_or_skip()
    w = _c2()
    nt, N = w.nt, w.border
    a_last, a_prev = _states(w, nt)            # w^2000, w^1999
    b_last, b_prev = _states(w, nt - 1)        # w^1999, w^1998
    assert np.array_equal(a_prev, b_last)      # the same 1999 steps, bit for bit
    scale = float(np.max(np.abs(b_last)))
    assert scale > 0
    src_iz = int(round((w.sources[0][2] - w.oz) / w.dz))
    for lo, hi in ((0, 96), (208, 304), (w.nz - 96, w.nz)):
        # sub-model of planes [lo, hi) with the grid's own border: its padded
        # planes are planes [lo, hi + 2N) of the full padded grid, and its
        # steps are exact wherever the stencil stays inside them
        sub = oracle.Grid(w.nx, w.ny, hi - lo, w.dx, w.dy, w.dz, w.ox, w.oy, w.oz + lo * w.dz,
                          border=N, dt=w.dt, nt=1)
        zs = slice(lo, hi + 2 * N)
        if lo <= src_iz < hi:
            src, f = w.sources[0], w.wavelet[nt - 1:nt]
        else:  # no source in the slab: a silent one at its centre
            src, f = w.nodes_to_metres([[w.nx // 2, w.ny // 2, (lo + hi) // 2]])[0], np.zeros(1)
        ref = oracle.forward(sub, w.vel[lo:hi], w.rho[lo:hi], f, src, np.zeros((0, 3)),
                             w0=b_last[zs], w_m1=b_prev[zs]).last
        # exact planes: the full grid's own planes [lo, hi + 2N), minus 4 next
        # to an edge of the slab that is not an edge of the full grid
        k0 = 0 if lo == 0 else N + 4
        k1 = 2 * N + (hi - lo) - (0 if hi == w.nz else N + 4)
        got = a_last[zs][k0:k1]
        exp = ref[k0:k1]
        err_max = float(np.max(np.abs(got - exp))) / scale
        err_l2 = rel_l2(got, exp)
        say(f"[c2 last step] model planes [{lo}, {hi}): {k1 - k0} padded planes, "
            f"max |gpu - oracle| / max|w| {err_max:.2e}, rel-L2 {err_l2:.2e}")
        # one FP32 step: about 30 roundings of terms up to ~5 max|w|
        assert err_max <= 2e-5 and err_l2 <= 1e-5


def test_c2_gradient_directional_derivative_full_size():
    # bench configuration: binomial checkpointing with 96 stored pairs; a
    # perturbation of the whole model (smooth noise, 8-cell Gaussian, 1 % of v
    # at most), so that the residual is a sizeable part of the traces and
    # FP32 rounding in them stays far below the misfit differences; observed
    # data from v + 5 dv
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, Propagator
    w = _c2()
    dv = (w.vel * seisgen.smooth_noise((w.nx, w.ny, w.nz), 77, 8.0, 0.01)).astype(np.float32)
    wav = torch.from_numpy(w.wavelet).cuda()
    P = Propagator(0)
    gs = GridSpec(**w.grid_kwargs())
    rho = torch.from_numpy(w.rho).cuda()

    def setv(v):
        P.set_model(gs, torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).cuda(), rho)

    setv(w.vel + 5.0 * dv)
    dobs = P.forward(wav, w.sources[0], w.receivers).clone()
    setv(w.vel)
    J, g = P.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=("revolve", 96))
    torch.cuda.synchronize()
    an = float(np.sum(g.cpu().numpy().astype(np.float64) * dv))
    J0 = float(J.item())
    P.release_workspace()

    def Jv(v):
        setv(v)
        return float(P.forward_misfit(wav, w.sources[0], w.receivers, dobs).item())

    # central differences at eps and 2 eps; their Richardson combination
    # removes the O(eps^2) term (about 1 % at eps = 1 for an anomaly that
    # shifts travel times by a tenth of a radian at 10 Hz)
    eps = 0.25
    fd1 = (Jv(w.vel + eps * dv) - Jv(w.vel - eps * dv)) / (2.0 * eps)
    fd2 = (Jv(w.vel + 2 * eps * dv) - Jv(w.vel - 2 * eps * dv)) / (4.0 * eps)
    fd = (4.0 * fd1 - fd2) / 3.0
    say(f"[c2 gradient FD] J {J0:.6e} analytic {an:.6e} central differences "
        f"{fd1:.6e} (eps {eps}) {fd2:.6e} (eps {2 * eps}) extrapolated {fd:.6e}")
    assert J0 > 0 and an < 0
    assert abs(fd - an) <= 1e-3 * abs(an)
    P.release_workspace()
    del P, dobs, g
    torch.cuda.empty_cache()
