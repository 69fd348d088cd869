"""FWI layer on the GPU: autograd wrapper, forward-only misfit, outer loop,
and checkpointing at the full gradient-workload size."""

import time

import numpy as np
import pytest

import oracle
import seisgen
from gpu_util import gpu_or_skip, oracle_grid, rel_l2, say

pytestmark = pytest.mark.gpu


def _shots_for(w, true_vel, torch, nshots=None):
    """Shots of workload w with observed data from the library on true_vel."""
    from paper_2502_12350_amd import GridSpec, Propagator
    from paper_2502_12350_amd.fwi import Shots
    g = GridSpec(**w.grid_kwargs())
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(true_vel).cuda(),
                None if w.rho is None else torch.from_numpy(w.rho).cuda())
    wav = torch.from_numpy(w.wavelet).cuda()
    srcs = w.sources if nshots is None else w.sources[:nshots]
    dobs = [P.forward(wav, s, w.receivers).clone() for s in srcs]
    torch.cuda.synchronize()
    return g, Shots(wav, np.asarray(srcs), [w.receivers] * len(srcs), dobs)


def _small_case(torch):
    w = seisgen.workload("c4_fd")
    n = w.nx
    true = seisgen.blob_anomalies(w.vel, seed=7, n_blobs=2, amp=0.08, sigma_cells=(3, 5),
                                  centre_lo=(10, 10, 12), centre_hi=(22, 22, 22))
    w.sources = w.nodes_to_metres([[8, 8, 4], [24, 8, 4], [8, 24, 4], [24, 24, 4]])
    w.receivers = w.nodes_to_metres([[1 + 2 * i, 1 + 2 * j, 2] for i in range(16)
                                     for j in range(16)])
    g, shots = _shots_for(w, true, torch)
    return w, g, shots, true


def test_forward_misfit_equals_gradient_misfit_and_oracle():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import Propagator
    w = seisgen.workload("c4_fd_vd")
    true = (w.vel + 5.0 * w.extra["dv"]).astype(np.float32)
    say("[forward misfit]")
    g, shots = _shots_for(w, true, torch, nshots=1)
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(w.vel).cuda(), torch.from_numpy(w.rho).cuda())
    J1 = P.forward_misfit(shots.wavelet, shots.sources[0], w.receivers, shots.dobs[0])
    J2, _ = P.gradient(shots.wavelet, shots.sources[0], w.receivers, shots.dobs[0])
    assert float(J1.item()) == float(J2.item())
    Jo, _ = oracle.misfit(oracle.forward(oracle_grid(w), w.vel, w.rho, w.wavelet, w.sources[0],
                                         w.receivers).seis, shots.dobs[0].cpu().numpy())
    assert abs(float(J1.item()) - Jo) <= 1e-4 * Jo


def test_wavefn_backward_is_the_library_gradient():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import Propagator
    from paper_2502_12350_amd.fwi import WaveFn, evaluate
    w, g, shots, _ = _small_case(torch)
    say("[WaveFn backward]")
    P = Propagator(0)
    v = torch.from_numpy(w.vel).cuda().requires_grad_(True)
    loss = WaveFn.apply(v, P, g, None, shots, "full")
    loss.backward()
    J, grad = evaluate(P, g, v.detach(), None, shots, ckpt="full")
    assert float(loss.item()) == float(J.item())
    assert torch.equal(v.grad, grad)
    # chain rule through a scaled loss
    v.grad = None
    (3.0 * WaveFn.apply(v, P, g, None, shots, "full")).backward()
    assert torch.allclose(v.grad, 3.0 * grad, rtol=1e-6, atol=0)


def test_wavefn_gradient_matches_finite_differences():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import Propagator
    from paper_2502_12350_amd.fwi import WaveFn, misfit_only
    w, g, shots, _ = _small_case(torch)
    say("[WaveFn finite differences]")
    P = Propagator(0)
    v = torch.from_numpy(w.vel).cuda().requires_grad_(True)
    WaveFn.apply(v, P, g, None, shots, "full").backward()
    dv = torch.from_numpy(w.extra["dv"]).cuda()

    def central(h):
        Jp = float(misfit_only(P, g, v.detach() + h * dv, None, shots).item())
        Jm = float(misfit_only(P, g, v.detach() - h * dv, None, shots).item())
        return (Jp - Jm) / (2.0 * h)

    # Richardson extrapolation of central differences at 1 % and 0.5 %
    # perturbations removes the O(h^2) truncation of the blob model's curvature
    f1, f2 = central(1.0), central(0.5)
    fd = (4.0 * f2 - f1) / 3.0
    an = float(torch.sum(v.grad.double() * dv.double()).item())
    say(f"  fd(1%) {f1:.6e} fd(0.5%) {f2:.6e} extrapolated {fd:.6e} adjoint {an:.6e}")
    assert abs(fd - an) <= 1e-3 * abs(an)


@pytest.mark.parametrize("method", ["sd", "lbfgs"])
def test_fwi_loop_reduces_misfit(method):
    torch = gpu_or_skip()
    from paper_2502_12350_amd import Propagator
    from paper_2502_12350_amd.fwi import fwi
    w, g, shots, true = _small_case(torch)
    say(f"[fwi {method}]")
    P = Propagator(0)
    v0 = torch.from_numpy(w.vel).cuda()
    # the top 6 planes hold the sources (depth 4) and receivers (depth 2):
    # their footprint is zeroed, as the paper's ZeroesNearSurface option does
    v, tr = fwi(P, g, v0, None, shots, n_iter=5, method=method, bounds=(1500.0, 4500.0),
                zero_top_planes=6)
    say(f"  misfit {tr.misfit[0]:.3e} -> {tr.misfit[-1]:.3e} in {tr.gpu_seconds[-1]:.2f} GPU-s, "
        f"{tr.n_gradients} gradients, {tr.n_misfits} misfits")
    assert tr.misfit[-1] < (0.6 if method == "lbfgs" else 0.8) * tr.misfit[0]
    assert all(b <= a * (1 + 1e-9) for a, b in zip(tr.misfit, tr.misfit[1:]))
    assert float(v.min()) >= 1500.0 and float(v.max()) <= 4500.0
    # the model moved towards the truth where the anomalies are
    err0 = np.linalg.norm(w.vel - true)
    err1 = np.linalg.norm(v.cpu().numpy() - true)
    assert err1 < err0


def test_gradient_workload_revolve_20_pairs_equals_full_storage():
    """200x200x160 model + 20-cell sponge, 1200 steps, 2500 receivers: binomial
    checkpointing with 20 stored pairs gives bitwise the full-storage gradient."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, Propagator, checkpoint_plan
    w = seisgen.workload("c4_start")
    say(f"[c4 revolve vs full] padded {w.padded_shape} nt {w.nt}")
    g = GridSpec(**w.grid_kwargs())
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(w.extra["v_true"]).cuda())
    wav = torch.from_numpy(w.wavelet).cuda()
    dobs = P.forward(wav, w.sources[0], w.receivers).clone()
    P.set_model(g, torch.from_numpy(w.vel).cuda())
    out = {}
    for ck in ["full", ("revolve", 20)]:
        P._workspace(P.workspace_bytes(len(w.receivers), ck))   # allocate outside the timing
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, grad = P.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=ck)
        torch.cuda.synchronize()
        out[str(ck)] = (float(J.item()), grad.clone(), time.perf_counter() - t0,
                        P.workspace_bytes(len(w.receivers), ck))
        P.release_workspace()
    (Jf, gf, tf, bf), (Jr, gr, tr_, br) = out["full"], out[str(("revolve", 20))]
    _, steps = checkpoint_plan(w.nt, 20)
    say(f"  full: {tf:.3f} s, {bf / 2**30:.1f} GiB; revolve(20): {tr_:.3f} s, "
        f"{br / 2**30:.2f} GiB, {steps} forward steps")
    assert steps == oracle.forward_steps_closed_form(w.nt + 1, 21)
    assert Jf == Jr and Jf > 0
    assert torch.equal(gf, gr)


@pytest.mark.parametrize("method", ["sd", "lbfgs"])
def test_fwi_restart_from_state_file_matches_uninterrupted_run(method, tmp_path):
    """Fault tolerance: a run stopped after 2 of 4 iterations and restarted
    from its state file ends bitwise where an uninterrupted run ends."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd import Propagator
    from paper_2502_12350_amd.fwi import fwi
    w, g, shots, _ = _small_case(torch)
    say(f"[fwi restart] {method}")
    P = Propagator(0)
    v0 = torch.from_numpy(w.vel).cuda()
    kw = dict(method=method, bounds=(1500.0, None), zero_top_planes=6)
    v_ref, tr_ref = fwi(P, g, v0, None, shots, n_iter=4, state_file=str(tmp_path / "a.npz"), **kw)
    state = str(tmp_path / "b.npz")
    fwi(P, g, v0, None, shots, n_iter=2, state_file=state, **kw)       # "interrupted"
    v, tr = fwi(P, g, v0, None, shots, n_iter=4, state_file=state, **kw)
    torch.cuda.synchronize()
    assert torch.equal(v, v_ref)
    assert tr.misfit == tr_ref.misfit
    assert tr.n_gradients == tr_ref.n_gradients and tr.n_misfits == tr_ref.n_misfits
    assert float(v.min()) >= 1500.0                                   # lower bound only


def test_fwi_restart_after_a_failure_in_the_middle_of_a_gradient(tmp_path):
    """Fault tolerance at shot granularity: a run that fails after shot 1 of
    the gradient evaluation of iteration 2 (four shots) and is restarted from
    its state files continues with shot 2 of that evaluation, and ends bitwise
    where an uninterrupted run ends."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd import Propagator
    from paper_2502_12350_amd.fwi import fwi
    w, g, shots, _ = _small_case(torch)
    assert len(shots) == 4
    P = Propagator(0)
    v0 = torch.from_numpy(w.vel).cuda()
    kw = dict(method="sd", bounds=(1500.0, 4500.0), zero_top_planes=6, n_iter=3)
    v_ref, tr_ref = fwi(P, g, v0, None, shots, state_file=str(tmp_path / "a.npz"), **kw)

    class Failure(Exception):
        pass

    def fail(key, s):
        if key == "2" and s == 1:
            raise Failure()

    state = str(tmp_path / "b.npz")
    with pytest.raises(Failure):
        fwi(P, g, v0, None, shots, state_file=state, shot_hook=fail, **kw)
    seen = []
    v, tr = fwi(P, g, v0, None, shots, state_file=state,
                shot_hook=lambda key, s: seen.append((key, s)), **kw)
    torch.cuda.synchronize()
    say(f"[fwi shot restart] shots run after the restart: {seen}")
    assert seen[0] == ("2", 2)                      # shots 0 and 1 came from the state file
    assert torch.equal(v, v_ref)
    assert tr.misfit == tr_ref.misfit


def test_gradient_workload_eight_shots_against_central_differences():
    """The gradient workload's sizes (200x200x160, 8 shots, 1200 steps, 2500
    receivers each, binomial checkpointing with 20 stored pairs): the
    directional derivative of the summed misfit along a smooth whole-model
    perturbation dv (1 % of v at most), with observed data from v + 5 dv,
    against central differences at eps = 0.25 and 0.5, combined by Richardson
    extrapolation (the O(eps^2) term cancels).  Along a direction unrelated
    to the residual the derivative would be about 1e-3 of the misfit, below
    what FP32 traces resolve in a difference of misfits."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, Propagator
    w = seisgen.workload("c4_start")
    g = GridSpec(**w.grid_kwargs())
    dv = (w.vel * seisgen.smooth_noise((w.nx, w.ny, w.nz), 78, 8.0, 0.01)).astype(np.float32)
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(w.vel + 5.0 * dv).cuda())
    wav = torch.from_numpy(w.wavelet).cuda()
    dobs = [P.forward(wav, s, w.receivers).clone() for s in w.sources]
    P.set_model(g, torch.from_numpy(w.vel).cuda())
    grad = torch.zeros((w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda")
    J = torch.zeros((), dtype=torch.float64, device="cuda")
    for s, d in zip(w.sources, dobs):
        P.gradient(wav, s, w.receivers, d, ckpt=("revolve", 20), grad=grad, misfit=J)
    torch.cuda.synchronize()
    an = float(np.sum(grad.cpu().numpy().astype(np.float64) * dv))
    P.release_workspace()

    def Jv(v):
        P.set_model(g, torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).cuda())
        m = torch.zeros((), dtype=torch.float64, device="cuda")
        for s, d in zip(w.sources, dobs):
            P.forward_misfit(wav, s, w.receivers, d, misfit=m)
        return float(m.item())

    eps = 0.25
    fd1 = (Jv(w.vel + eps * dv) - Jv(w.vel - eps * dv)) / (2 * eps)
    fd2 = (Jv(w.vel + 2 * eps * dv) - Jv(w.vel - 2 * eps * dv)) / (4 * eps)
    fd = (4 * fd1 - fd2) / 3
    say(f"[c4 gradient FD] J {float(J.item()):.6e} analytic {an:.6e} central differences "
        f"{fd1:.6e} {fd2:.6e} extrapolated {fd:.6e}")
    assert float(J.item()) > 0 and an < 0
    assert abs(fd - an) <= 1e-3 * abs(an)
