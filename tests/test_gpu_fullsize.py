"""Properties checked at the full bench size (576^3 padded, variable density,
2000 steps, 65,536 receivers), in the launch configuration bench.py times.
The FP64 oracle cannot run at this size, so these are properties that hold at
any size: determinism, reciprocity, zero misfit at the true model, and the
trace at a receiver staying finite and bounded."""

import numpy as np
import pytest

import seisgen
from gpu_util import gpu_or_skip, say

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
