"""wfd_forward_noalloc (the forward entry point that takes its workspace from
the library's static device scratch) against wfd_forward, through the C ABI.

Two calls in a row on one context's GPU, the second on a smaller grid than
the first (the scratch keeps the first call's contents), each bitwise equal
to wfd_forward with a caller workspace; a shot too large for the scratch is
refused before anything is launched.
"""

import ctypes as C

import numpy as np
import pytest

import seisgen
from gpu_util import gpu_or_skip, propagator, say

pytestmark = pytest.mark.gpu


def _noalloc(P, w, torch):
    from paper_2502_12350_amd import _lib
    from paper_2502_12350_amd.api import _dptr, _xyz
    nrec = len(w.receivers)
    seis = torch.full((nrec, w.nt), float("nan"), dtype=torch.float32, device="cuda")
    fin = torch.full((2,) + w.padded_shape, float("nan"), dtype=torch.float32, device="cuda")
    wav = torch.from_numpy(w.wavelet).cuda()
    src, rec = _xyz(w.sources[0]), _xyz(w.receivers)
    P._sync_stream()
    _lib.check(_lib.lib().wfd_forward_noalloc(P._ctx, wav.data_ptr(), _dptr(src), nrec,
                                              _dptr(rec), seis.data_ptr(), fin.data_ptr()))
    torch.cuda.synchronize()
    return seis.cpu().numpy(), fin.cpu().numpy()


def test_noalloc_forward_equals_forward_twice_shrinking():
    torch = gpu_or_skip()
    for name in ("c2_small", "c4_fd_vd"):   # 125 x 109 x 93 padded, then 48^3
        w = seisgen.workload(name)
        say(f"[noalloc] {name} padded {w.padded_shape} nt {w.nt} nrec {len(w.receivers)}")
        P = propagator(w)
        s_na, f_na = _noalloc(P, w, torch)
        s_ref, f_ref = P.forward(torch.from_numpy(w.wavelet).cuda(), w.sources[0], w.receivers,
                                 final=True)
        torch.cuda.synchronize()
        assert np.array_equal(s_na, s_ref.cpu().numpy())
        assert np.array_equal(f_na, f_ref.cpu().numpy())


def test_noalloc_refuses_a_shot_larger_than_the_scratch():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import _lib
    from paper_2502_12350_amd.api import _dptr, _xyz
    w = seisgen.workload("c4_fd")
    w.nx = w.ny = 200
    w.nz = 160
    w.border = 20     # 240 x 240 x 200 padded: two 49 MB volumes
    w.vel = np.full((w.nz, w.ny, w.nx), 2000.0, dtype=np.float32)
    say("[noalloc] 240 x 240 x 200 padded: refused")
    P = propagator(w, rho=None)
    assert P.workspace_bytes(len(w.receivers)) > _lib.NOALLOC_SCRATCH_BYTES
    seis = torch.zeros((len(w.receivers), w.nt), dtype=torch.float32, device="cuda")
    wav = torch.from_numpy(w.wavelet).cuda()
    st = _lib.lib().wfd_forward_noalloc(P._ctx, wav.data_ptr(), _dptr(_xyz(w.sources[0])),
                                        len(w.receivers), _dptr(_xyz(w.receivers)),
                                        seis.data_ptr(), None)
    assert st == -4   # WFD_E_NOMEM
    assert b"static scratch" in _lib.lib().wfd_last_error()
