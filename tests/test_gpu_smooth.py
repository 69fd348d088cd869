"""Gradient smoothing (Laplace and Bessel filters) on the GPU against the
FP64 oracle (oracle/smooth.py) on a ragged volume, plus its use in the FWI
gradient."""

import numpy as np
import pytest

from oracle import smooth as osm
from gpu_util import gpu_or_skip, rel_l2, say

pytestmark = pytest.mark.gpu

SHAPE = (11, 17, 23)   # [z][y][x]
H = (10.0, 12.0, 8.0)  # (x, y, z)


@pytest.mark.parametrize("mode", ["laplace", "bessel"])
def test_smoothing_matches_oracle(mode):
    torch = gpu_or_skip()
    from paper_2502_12350_amd import smooth
    rng = np.random.default_rng(7)
    g = rng.standard_normal(SHAPE).astype(np.float32)
    lens = (2 * H[0], 3 * H[1], 1.5 * H[2])
    ref = (osm.laplace_filter if mode == "laplace" else osm.bessel_filter)(g, lens, H)
    out, it = smooth(torch.from_numpy(g).cuda(), mode, lens, H, tol=1e-7)
    torch.cuda.synchronize()
    e = rel_l2(out.cpu().numpy(), ref)
    say(f"[smooth {mode}] rel-L2 {e:.2e}, {it} iterations")
    assert e <= 1e-5
    # constants are kept
    c, _ = smooth(torch.full(SHAPE, 2.5, device="cuda"), mode, lens, H, tol=1e-7)
    assert float((c - 2.5).abs().max()) <= 1e-5
    if mode == "laplace":  # in place gives the same bits
        x = torch.from_numpy(g).cuda()
        smooth(x, mode, lens, H, out=x)
        assert torch.equal(x, out)


def test_smoothing_errors():
    torch = gpu_or_skip()
    from paper_2502_12350_amd import smooth, WfdError
    x = torch.zeros(SHAPE, device="cuda")
    with pytest.raises(WfdError):
        smooth(x, "bessel", (10.0, 10.0, 10.0), H, out=x)       # needs out != in
    with pytest.raises(WfdError):
        smooth(x, "laplace", (-1.0, 10.0, 10.0), H)
    with pytest.raises(WfdError) as e:                          # too few iterations
        smooth(torch.randn(SHAPE, device="cuda"), "bessel", (40.0, 40.0, 40.0), H,
               tol=1e-9, max_iter=2)
    assert e.value.name == "WFD_E_RANGE"


def test_fwi_gradient_smoothing_is_applied_before_zeroing():
    torch = gpu_or_skip()
    import seisgen
    from paper_2502_12350_amd import GridSpec, Propagator, smooth
    from paper_2502_12350_amd.fwi import Shots, evaluate
    w = seisgen.workload("c4_fd")
    g = GridSpec(**w.grid_kwargs())
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(w.vel + 5.0 * w.extra["dv"]).cuda())
    wav = torch.from_numpy(w.wavelet).cuda()
    d = P.forward(wav, w.sources[0], w.receivers).clone()
    shots = Shots(wav, np.asarray(w.sources), [w.receivers], [d])
    v = torch.from_numpy(w.vel).cuda()
    _, raw = evaluate(P, g, v, None, shots, ckpt="full")
    raw = raw.clone()
    lens = (20.0, 20.0, 20.0)
    _, sm = evaluate(P, g, v, None, shots, ckpt="full", zero_top_planes=3,
                     smoothing=("bessel", lens))
    ref, _ = smooth(raw, "bessel", lens, (w.dx, w.dy, w.dz))
    ref[:3] = 0.0
    torch.cuda.synchronize()
    assert float((sm - ref).abs().max()) <= 1e-6 * float(ref.abs().max())


@pytest.mark.parametrize("mode", ["nearest", "sinc"])
def test_resampling_matches_oracle(mode):
    torch = gpu_or_skip()
    from oracle import resample as ors
    from paper_2502_12350_amd import resample
    rng = np.random.default_rng(9)
    d = rng.standard_normal((37, 300)).astype(np.float32)
    for dt_in, nt_out, dt_out in ((2e-3, 600, 1e-3), (1e-3, 130, 2.3e-3), (1.5e-3, 300, 1.5e-3)):
        ref = ors.resample(d, dt_in, nt_out, dt_out, mode)
        got = resample(torch.from_numpy(d).cuda(), dt_in, nt_out, dt_out, mode)
        torch.cuda.synchronize()
        g = got.cpu().numpy().astype(np.float64)
        if mode == "nearest":
            assert np.array_equal(g, ref)
        else:
            e = rel_l2(g, ref)
            say(f"[resample sinc] dt {dt_in} -> {dt_out}: rel-L2 {e:.2e}")
            assert e <= 1e-6
