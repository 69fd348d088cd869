"""Forward wavefield kept in host memory (the paper's second wavefield option,
§2.1: the whole forward wavefield in secondary storage, read back during the
adjoint sweep).  The states travel over PCIe on a copy stream; the gradient
must be bitwise that of full device storage, and the host slots must hold
exactly the forward states w^1 .. w^nt."""

import numpy as np
import pytest

import seisgen
from gpu_util import gpu_or_skip, propagator, say

pytestmark = pytest.mark.gpu


def _case(nt=None):
    """c4_fd_vd (32^3 model, 48^3 padded), observed data from a perturbed model."""
    torch = gpu_or_skip()
    w = seisgen.workload("c4_fd_vd")
    if nt is not None:
        w.nt = nt
        w.wavelet = w.wavelet[:nt].copy()
    true = (w.vel + 5.0 * w.extra["dv"]).astype(np.float32)
    P = propagator(w, vel=true)
    dobs = P.forward(torch.from_numpy(w.wavelet).cuda(), w.sources[0], w.receivers).clone()
    torch.cuda.synchronize()
    return w, dobs


def _grad(w, dobs, ckpt):
    torch = gpu_or_skip()
    P = propagator(w)
    il = torch.zeros((w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda")
    J, g, seis = P.gradient(torch.from_numpy(w.wavelet).cuda(), w.sources[0], w.receivers, dobs,
                            ckpt=ckpt, illum=il, seis=True)
    torch.cuda.synchronize()
    return P, float(J.item()), g.cpu().numpy(), seis.cpu().numpy(), il.cpu().numpy()


@pytest.mark.parametrize("nt", [None, 1, 3, 4, 5, 9])
def test_host_store_equals_full_storage_bitwise(nt):
    # nt around the 4-volume staging ring: fewer steps than the ring, exactly
    # the ring, one past it, and the full 300-step case
    w, dobs = _case(nt)
    say(f"[host store] nt {w.nt}")
    _, Jf, gf, sf, ilf = _grad(w, dobs, "full")
    _, Jh, gh, sh, ilh = _grad(w, dobs, "host")
    assert Jf == Jh
    assert np.array_equal(sf, sh)
    assert np.array_equal(gf, gh)
    assert np.array_equal(ilf, ilh)


def test_host_slots_hold_the_forward_states():
    # slot m-1 of a caller-provided store is 2^e w^m: compare slots with the final
    # state of forward runs that stop after m steps (same kernels, same bits)
    torch = gpu_or_skip()
    w, dobs = _case(40)
    P = propagator(w)
    nbytes = P.host_store_bytes()
    store = torch.empty(nbytes // 4, dtype=torch.float32, pin_memory=True)
    store.fill_(np.nan)
    e = torch.zeros((), dtype=torch.int32, device="cuda")
    P.gradient(torch.from_numpy(w.wavelet).cuda(), w.sources[0], w.receivers, dobs,
               ckpt=("host", store), field_exp2=e)
    torch.cuda.synchronize()
    e = int(e.item())   # the slots hold 2^e w^m (exact power-of-two field scaling)
    say(f"  field exponent {e}")
    Nz, Ny, Nx = w.padded_shape
    pitch = (Nx + 63) // 64 * 64          # rows of the pitched device volumes
    assert nbytes == w.nt * Nz * Ny * pitch * 4
    slots = store.view(w.nt, Nz, Ny, pitch)[..., :Nx]
    assert not torch.isnan(slots).any()
    for m in (1, 2, 17, 39, 40):
        wm = seisgen.workload("c4_fd_vd")
        wm.nt = m
        wm.wavelet = w.wavelet[:m].copy()
        Q = propagator(wm)
        _, fin = Q.forward(torch.from_numpy(wm.wavelet).cuda(), w.sources[0], w.receivers,
                           final=True)
        torch.cuda.synchronize()
        say(f"  slot {m - 1} vs forward to step {m}")
        assert torch.equal(slots[m - 1] * (2.0 ** -e), fin[0].cpu())


def test_host_store_reused_across_calls_and_accumulates():
    # two calls on one context share the copy stream and its events; gradients
    # accumulate exactly as with full storage
    torch = gpu_or_skip()
    w, dobs = _case(60)
    res = {}
    for mode in ("full", "host"):
        P = propagator(w)
        wav = torch.from_numpy(w.wavelet).cuda()
        g = torch.zeros((w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda")
        J = torch.zeros((), dtype=torch.float64, device="cuda")
        for s in (w.sources[0], w.nodes_to_metres([[10, 20, 6]])[0]):
            P.gradient(wav, s, w.receivers, dobs, ckpt=mode, grad=g, misfit=J)
        torch.cuda.synchronize()
        res[mode] = (float(J.item()), g.cpu().numpy())
    assert res["full"][0] == res["host"][0]
    assert np.array_equal(res["full"][1], res["host"][1])


def test_host_store_errors():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import WfdError
    w, dobs = _case(12)
    P = propagator(w)
    wav = torch.from_numpy(w.wavelet).cuda()
    need = P.host_store_bytes()
    Nz, Ny, Nx = w.padded_shape
    assert need == w.nt * Nz * Ny * ((Nx + 63) // 64 * 64) * 4
    small = torch.empty(need // 4 - 1, dtype=torch.float32, pin_memory=True)
    with pytest.raises(WfdError, match="host store has"):
        P.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=("host", small))
    pageable = torch.empty(need // 4, dtype=torch.float32)
    with pytest.raises(WfdError, match="page-locked"):
        P.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=("host", pageable))
    with pytest.raises(ValueError):
        P.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=("host", dobs))
