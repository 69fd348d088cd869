"""Batched multi-shot forward (one launch per step over every shot's window,
optionally one HIP graph) and launch-shape tuning, on the GPU.

The batch must give bitwise the traces of the per-shot forward of each
window, which in turn matches the FP64 oracle (seismogram rel-L2 <= 1e-4);
every tile shape must give bitwise the same result as the default one.
"""

import numpy as np
import pytest

import oracle
import seisgen
from gpu_util import gpu_or_skip, oracle_grid, propagator, rel_l2, say

pytestmark = pytest.mark.gpu

SEIS_TOL = 1e-4


def _windows(name):
    w = seisgen.workload(name)
    return w, [seisgen.shot_window(w, i) for i in range(len(w.sources))]


def _batch(torch, shots, stream=None, rec_override=None):
    from paper_2502_12350_amd import ShotBatch
    props = [propagator(s) for s in shots]
    wav = torch.from_numpy(shots[0].wavelet).cuda()
    recs = [s.receivers for s in shots] if rec_override is None else rec_override
    if stream is not None:
        with torch.cuda.stream(stream):
            b = ShotBatch(props, wav, [s.sources[0] for s in shots], recs, stream=stream)
    else:
        b = ShotBatch(props, wav, [s.sources[0] for s in shots], recs)
    return b, props, wav


def test_batch_equals_per_shot_and_oracle():
    torch = gpu_or_skip()
    w, shots = _windows("c3_small")
    say(f"[batch] c3_small {len(shots)} windows "
        f"{[s.padded_shape for s in shots]} nt {w.nt}")
    recs = [s.receivers for s in shots]
    recs[1] = np.zeros((0, 3))          # a shot without receivers in the middle
    b, props, wav = _batch(torch, shots, rec_override=recs)
    seis = [t.clone() for t in b.run()]
    torch.cuda.synchronize()
    for i, (s, P) in enumerate(zip(shots, props)):
        ref = P.forward(wav, s.sources[0], recs[i])
        torch.cuda.synchronize()
        assert seis[i].shape == ref.shape
        assert torch.equal(seis[i], ref), f"shot {i}"
    for i in (0, 2):
        s = shots[i]
        o = oracle.forward(oracle_grid(s), s.vel, s.rho, s.wavelet, s.sources[0], s.receivers)
        e = rel_l2(seis[i].cpu().numpy(), o.seis)
        say(f"  shot {i} vs oracle rel-L2 {e:.3e}")
        assert e <= SEIS_TOL
    # a second run repeats the acquisition exactly
    again = b.run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for a, c in zip(seis, again))
    b.close()


def test_batch_graph_replays_match_eager():
    torch = gpu_or_skip()
    w, shots = _windows("c3_small")
    say("[batch graph] c3_small")
    stream = torch.cuda.Stream()
    b, props, wav = _batch(torch, shots, stream=stream)
    with torch.cuda.stream(stream):
        eager = [t.clone() for t in b.run(use_graph=False)]
    torch.cuda.synchronize()
    side = torch.zeros(1 << 20, device="cuda")
    for rep in range(3):
        with torch.cuda.stream(stream):
            for t in b.seis:
                t.fill_(float("nan"))
            b.run(use_graph=True)
        torch.cuda.synchronize()
        for i, (a, e) in enumerate(zip(b.seis, eager)):
            assert torch.equal(a, e), f"replay {rep} shot {i}"
        # the program's own eager work between replays
        side.add_(1.0)
        x = props[0].forward(wav, shots[0].sources[0], shots[0].receivers)
        torch.cuda.synchronize()
        assert torch.equal(x, eager[0])
        assert float(side.sum()) == float((rep + 1) * side.numel())
    b.close()


def test_batch_rejects_bad_arguments():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import ShotBatch, WfdError
    w, shots = _windows("c3_small")
    say("[batch errors]")
    props = [propagator(s) for s in shots[:2]]
    wav = torch.from_numpy(shots[0].wavelet).cuda()
    src = [s.sources[0] for s in shots[:2]]
    rec = [s.receivers for s in shots[:2]]
    with pytest.raises(WfdError) as e:          # the same context twice
        ShotBatch([props[0], props[0]], wav, src, rec)
    assert e.value.name == "WFD_E_ARG"
    other = seisgen.shot_window(w, 1)
    other.nt = w.nt - 10
    other.wavelet = other.wavelet[:other.nt]
    q = propagator(other)
    with pytest.raises(WfdError) as e:          # different nt
        ShotBatch([props[0], q], wav, src, rec)
    assert e.value.name == "WFD_E_ARG"
    cd = seisgen.shot_window(w, 1)
    cd.rho = None
    with pytest.raises(WfdError) as e:          # mixed density modes
        ShotBatch([props[0], propagator(cd)], wav, src, rec)
    assert e.value.name == "WFD_E_ARG"
    with pytest.raises(WfdError) as e:          # source outside shot 1's window
        ShotBatch(props, wav, [src[0], src[0]], rec)
    assert e.value.name == "WFD_E_RANGE"
    b = ShotBatch(props, wav, src, rec)          # legacy NULL stream: no graph
    if torch.cuda.current_stream().cuda_stream == 0:
        with pytest.raises(WfdError) as e:
            b.run(use_graph=True)
        assert e.value.name == "WFD_E_ARG"
    b.close()


def test_batch_refuses_to_run_after_a_member_model_changed():
    """A batch's step descriptors hold the coefficient pointers of each
    context's model at creation: setting a model again on a member context
    makes the batch refuse to run (WFD_E_STATE) rather than read a freed or
    reused buffer; the old buffers stay referenced by the batch meanwhile."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, ShotBatch, WfdError
    w, shots = _windows("c3_small")
    say("[batch after set_model]")
    b, props, wav = _batch(torch, shots[:2])
    first = [t.clone() for t in b.run()]
    torch.cuda.synchronize()
    old = props[1]._model
    s = shots[1]
    props[1].set_model(GridSpec(**s.grid_kwargs()), torch.from_numpy(s.vel).cuda(),
                       torch.from_numpy(s.rho).cuda())
    assert b._models[1] is old            # still alive while the batch exists
    with pytest.raises(WfdError) as e:
        b.run()
    assert e.value.name == "WFD_E_STATE" and "model changed" in str(e.value)
    b.close()
    b2 = ShotBatch(props, wav, [x.sources[0] for x in shots[:2]], [x.receivers for x in shots[:2]])
    again = b2.run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for a, c in zip(first, again))
    b2.close()


@pytest.mark.parametrize("variant,rounds", [(0, 0), (0, 2), (1, 0), (1, 8), (2, 0), (2, 4),
                                            (3, 0), (3, 6), (4, 0), (4, 3)])
def test_forward_tile_shapes_are_bitwise_identical(variant, rounds):
    torch = gpu_or_skip()
    w = seisgen.workload("c2_small")
    say(f"[tuning] forward c2_small variant {variant} rounds {rounds}")
    P = propagator(w)
    wav = torch.from_numpy(w.wavelet).cuda()
    base, fb = P.forward(wav, w.sources[0], w.receivers, final=True)
    base, fb = base.clone(), fb.clone()
    P.set_tuning(variant, rounds)
    assert P.tuning() == (variant, rounds, 0, 0)
    s, f = P.forward(wav, w.sources[0], w.receivers, final=True)
    torch.cuda.synchronize()
    assert torch.equal(s, base)
    assert torch.equal(f, fb)


@pytest.mark.parametrize("adj_variant,adj_rounds", [(0, 2), (1, 0), (1, 8), (2, 0), (2, 3), (3, 0),
                                                    (3, 4)])
def test_adjoint_tile_shapes_are_bitwise_identical(adj_variant, adj_rounds):
    torch = gpu_or_skip()
    w = seisgen.workload("c4_fd_vd")
    say(f"[tuning] adjoint c4_fd_vd variant {adj_variant} rounds {adj_rounds}")
    P = propagator(w)
    wav = torch.from_numpy(w.wavelet).cuda()
    dobs = torch.zeros((len(w.receivers), w.nt), dtype=torch.float32, device="cuda")
    illum0 = torch.zeros((w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda")
    J0, g0 = P.gradient(wav, w.sources[0], w.receivers, dobs, illum=illum0)
    J0, g0 = float(J0.item()), g0.clone()
    P.set_tuning(1, 3, adj_variant, adj_rounds)
    illum1 = torch.zeros_like(illum0)
    J1, g1 = P.gradient(wav, w.sources[0], w.receivers, dobs, illum=illum1)
    torch.cuda.synchronize()
    assert float(J1.item()) == J0 and J0 > 0
    assert torch.equal(g1, g0)
    assert torch.equal(illum1, illum0)


def test_autotune_picks_shapes_and_keeps_results():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import WfdError
    w = seisgen.workload("c2_small")
    say("[autotune] c2_small")
    P = propagator(w)
    wav = torch.from_numpy(w.wavelet).cuda()
    base = P.forward(wav, w.sources[0], w.receivers).clone()
    dobs = torch.zeros_like(base)
    _, gbase = P.gradient(wav, w.sources[0], w.receivers, dobs)
    gbase = gbase.clone()
    t, fus, aus = P.autotune(steps=5)
    say(f"  picked {t}: forward {fus:.1f} us/step, adjoint {aus:.1f} us/step")
    assert t[0] in range(5) and t[2] in range(4)
    assert t[1] in (0, 2, 3, 4, 6, 8) and t[3] in (0, 2, 3, 4, 6, 8)
    assert fus > 0 and aus > 0
    assert P.tuning() == t
    s = P.forward(wav, w.sources[0], w.receivers)
    _, g = P.gradient(wav, w.sources[0], w.receivers, dobs)
    torch.cuda.synchronize()
    assert torch.equal(s, base)
    assert torch.equal(g, gbase)
    with pytest.raises(WfdError):
        P.set_tuning(5, 0)
    with pytest.raises(WfdError):
        P.set_tuning(0, 0, 4, 0)
    with pytest.raises(WfdError):
        P.set_tuning(0, 65)
    with pytest.raises(WfdError):
        P.autotune(steps=0)


@pytest.mark.slow
def test_c3_full_size_batch_graph_equals_per_shot():
    """All 24 windows of the 400 x 400 x 256 model, 1500 steps, in the launch
    configuration the benchmark times (graph replay on a side stream)."""
    torch = gpu_or_skip()
    w, shots = _windows("c3")
    say(f"[c3 full size] {len(shots)} windows, nt {w.nt}")
    stream = torch.cuda.Stream()
    b, props, wav = _batch(torch, shots, stream=stream)
    with torch.cuda.stream(stream):
        b.run(use_graph=True)
    torch.cuda.synchronize()
    for i, (s, P) in enumerate(zip(shots, props)):
        ref = P.forward(wav, s.sources[0], s.receivers)
        torch.cuda.synchronize()
        assert torch.equal(b.seis[i], ref), f"shot {i}"
        assert bool(torch.isfinite(ref).all()) and float(ref.abs().max()) > 0
    b.close()


def test_batch_with_free_surface_windows_equals_per_shot():
    # windows 0 and 2 have a free surface: the batch runs the kernels with
    # image loads for every window, and each window must still equal its own
    # forward (which uses the kernels without them when it has no surface)
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, Propagator, ShotBatch
    w, shots = _windows("c3_small")
    say(f"[batch] c3_small with free surfaces on windows 0 and 2")
    props = []
    for i, s in enumerate(shots):
        P = Propagator(0)
        P.set_model(GridSpec(**s.grid_kwargs(), free_surface=i in (0, 2)),
                    torch.from_numpy(s.vel).cuda(), torch.from_numpy(s.rho).cuda())
        props.append(P)
    wav = torch.from_numpy(shots[0].wavelet).cuda()
    recs = [s.receivers for s in shots]
    b = ShotBatch(props, wav, [s.sources[0] for s in shots], recs)
    seis = [t.clone() for t in b.run()]
    torch.cuda.synchronize()
    for i, (s, P) in enumerate(zip(shots, props)):
        ref = P.forward(wav, s.sources[0], recs[i])
        torch.cuda.synchronize()
        assert torch.equal(seis[i], ref), f"shot {i}"
    # the surface changes the traces of its windows
    Q = Propagator(0)
    Q.set_model(GridSpec(**shots[0].grid_kwargs()), torch.from_numpy(shots[0].vel).cuda(),
                torch.from_numpy(shots[0].rho).cuda())
    plain = Q.forward(wav, shots[0].sources[0], recs[0])
    torch.cuda.synchronize()
    assert not torch.equal(plain, seis[0])
    b.close()


@pytest.mark.parametrize("variant,adj_variant", [(1, 1), (2, 2), (3, 1), (4, 3)])
def test_tile_shapes_bitwise_identical_with_free_surface(variant, adj_variant):
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GridSpec, Propagator
    w = seisgen.workload("c4_fd_vd")
    say(f"[tuning] free surface, forward variant {variant}, adjoint variant {adj_variant}")
    P = Propagator(0)
    P.set_model(GridSpec(**w.grid_kwargs(), free_surface=True), torch.from_numpy(w.vel).cuda(),
                torch.from_numpy(w.rho).cuda())
    wav = torch.from_numpy(w.wavelet).cuda()
    dobs = torch.zeros((len(w.receivers), w.nt), dtype=torch.float32, device="cuda")
    J0, g0, s0 = P.gradient(wav, w.sources[0], w.receivers, dobs, seis=True)
    J0, g0, s0 = float(J0.item()), g0.clone(), s0.clone()
    P.set_tuning(variant, 0, adj_variant, 0)
    J1, g1, s1 = P.gradient(wav, w.sources[0], w.receivers, dobs, seis=True)
    torch.cuda.synchronize()
    assert float(J1.item()) == J0 and J0 > 0
    assert torch.equal(s1, s0)
    assert torch.equal(g1, g0)


# ---------------------------------------------------------------------------
# batched gradients
# ---------------------------------------------------------------------------
def _gradient_windows(torch):
    """c3_small's 4 windows with observed data from a true model (three
    +/-8 % blobs on a 3 % faster background), each window's data from its own
    forward run on the true window."""
    import copy
    w, shots = _windows("c3_small")
    wt = copy.copy(w)
    wt.vel = (seisgen.blob_anomalies(w.vel, seed=31, n_blobs=3, amp=0.08, sigma_cells=(3.0, 6.0),
                                     centre_lo=(15, 15, 12), centre_hi=(80, 65, 40))
              * np.float32(1.03)).astype(np.float32)
    true = [seisgen.shot_window(wt, i) for i in range(len(shots))]
    wav = torch.from_numpy(shots[0].wavelet).cuda()
    dobs = []
    for s, t in zip(shots, true):
        P = propagator(t)
        dobs.append(P.forward(wav, s.sources[0], s.receivers).clone())
    torch.cuda.synchronize()
    return w, shots, true, wav, dobs


def test_gradient_batch_equals_per_shot_and_oracle():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GradientBatch
    w, shots, true, wav, dobs = _gradient_windows(torch)
    say(f"[gradient batch] c3_small {len(shots)} windows {[s.padded_shape for s in shots]} "
        f"nt {w.nt}, 3 stored pairs")
    recs = [s.receivers for s in shots]
    recs[1] = np.zeros((0, 3))          # a shot without receivers
    dob = list(dobs)
    dob[1] = None
    props = [propagator(s) for s in shots]
    b = GradientBatch(props, wav, [s.sources[0] for s in shots], recs, dob, 3, illum=True)
    J, grads = b.run()
    torch.cuda.synchronize()
    J = J.cpu().numpy()
    grads = [g.cpu().numpy() for g in grads]
    ills = [i.cpu().numpy() for i in b.illum]
    for i, (s, P) in enumerate(zip(shots, props)):
        il = torch.zeros((s.nz, s.ny, s.nx), dtype=torch.float32, device="cuda")
        if i == 1:
            assert J[1] == 0.0 and not grads[1].any()
            continue
        Ji, gi = P.gradient(wav, s.sources[0], recs[i], dobs[i], ckpt=("revolve", 3), illum=il)
        torch.cuda.synchronize()
        assert float(Ji.item()) == J[i], f"shot {i}"
        assert np.array_equal(gi.cpu().numpy(), grads[i]), f"shot {i}"
        assert np.array_equal(il.cpu().numpy(), ills[i]), f"shot {i}"
    s = shots[0]
    ref = oracle.gradient(oracle_grid(s), s.vel, s.rho, s.wavelet, s.sources[0], s.receivers,
                          dobs[0].cpu().numpy(), illumination=True)
    eJ = abs(J[0] - ref.misfit) / ref.misfit
    eg = rel_l2(grads[0], ref.grad)
    say(f"  shot 0 vs oracle: misfit {eJ:.2e}, gradient rel-L2 {eg:.2e}")
    assert eJ <= SEIS_TOL and eg <= 1e-3 and rel_l2(ills[0], ref.illum) <= SEIS_TOL
    b.close()


def test_gradient_batch_graph_replays_match_eager():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import GradientBatch
    w, shots, true, wav, dobs = _gradient_windows(torch)
    say("[gradient batch graph] c3_small")
    stream = torch.cuda.Stream()
    props = [propagator(s) for s in shots]
    with torch.cuda.stream(stream):
        b = GradientBatch(props, wav, [s.sources[0] for s in shots], [s.receivers for s in shots],
                          dobs, 2, stream=stream)
        J0, g0 = b.run(use_graph=False)
        J0, g0 = J0.clone(), [g.clone() for g in g0]
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.cuda.stream(stream):
            b.misfit.zero_()
            for g in b.grad:
                g.fill_(0.0)
            J, g = b.run(use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(J, J0), f"replay {rep}"
        assert all(torch.equal(a, c) for a, c in zip(g, g0)), f"replay {rep}"
        # the program's own eager work between replays
        x = props[0].forward(wav, shots[0].sources[0], shots[0].receivers)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(x).all())
    b.close()
