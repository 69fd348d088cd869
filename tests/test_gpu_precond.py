"""What the trained preconditioner gains over the method without it, on
models outside its training set (the training recipe with seeds 9000+):
direction quality, model error, and the headline comparison, GPU-seconds to
equal final misfit."""

import numpy as np
import pytest

import seisgen
from gpu_util import gpu_or_skip, say

pytestmark = pytest.mark.gpu


def _case(torch):
    from paper_2502_12350_amd import GridSpec, Propagator
    from paper_2502_12350_amd.fwi import Shots
    w = seisgen.c5_model(9000)
    g = GridSpec(**w.grid_kwargs())
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(w.extra["v_true"]).cuda())
    wav = torch.from_numpy(w.wavelet).cuda()
    dobs = [P.forward(wav, s, w.receivers).clone() for s in w.sources]
    shots = Shots(wav, np.asarray(w.sources), [w.receivers] * len(w.sources), dobs)
    return w, g, P, shots


def test_network_direction_is_closer_to_the_true_perturbation():
    """Mean over four unseen 128^3 models of the cosine between a direction
    and the true perturbation: the network's must beat the plain one's."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd.precond import (Preconditioner, TRAINED, cosine,
                                              fallback_direction, solver_pair)
    from paper_2502_12350_amd import Propagator
    say("[precond] direction quality on unseen 128^3 models")
    net = Preconditioner.load(TRAINED)
    prop = Propagator(0)
    c_net, c_fb = [], []
    for seed in range(9000, 9004):
        grad, illum, dv = solver_pair(prop, seisgen.c5_model(seed))
        d_net, _ = net.direction(grad, illum)
        c_net.append(cosine(d_net, dv))
        c_fb.append(cosine(fallback_direction(grad, illum), dv))
        say(f"  seed {seed}: network {c_net[-1]:.3f}, fallback {c_fb[-1]:.3f}")
    assert np.mean(c_net) > 1.2 * np.mean(c_fb) > 0


def test_fwi_with_the_network_moves_the_model_closer_to_the_truth():
    """Three FWI iterations on an unseen model: stepping along the network's
    direction ends closer to the true model than stepping along the plain
    illumination-compensated gradient (the data misfit, dominated by shallow
    well-lit cells, falls about as fast either way and is only reported)."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd.fwi import fwi
    from paper_2502_12350_amd.precond import Preconditioner, TRAINED
    w, g, P, shots = _case(torch)
    say("[precond] 3 FWI iterations, network vs plain")
    err0 = float(np.linalg.norm(w.vel - w.extra["v_true"]))
    net = Preconditioner.load(TRAINED)
    v0 = torch.from_numpy(w.vel).cuda()
    res = {}
    for method in ("sd", "cnn"):
        v, tr = fwi(P, g, v0, None, shots, n_iter=3, method=method, bounds=(1500.0, 4500.0),
                    zero_top_planes=10, precond=net)
        res[method] = (tr.misfit, float(np.linalg.norm(v.cpu().numpy() - w.extra["v_true"])))
        say(f"  {method}: misfit {tr.misfit[0]:.4e} -> {tr.misfit[-1]:.4e}, "
            f"model error {res[method][1] / err0:.6f} of the start, network steps {tr.n_network}")
    assert res["cnn"][1] < res["sd"][1] < err0
    assert res["cnn"][0][-1] < res["cnn"][0][0]


def test_span_step_reaches_the_plain_final_misfit_in_fewer_gpu_seconds():
    """The headline comparison on an unseen model: FWI misfit cut per GPU-s at
    equal final misfit.  The step in the plane of the plain and the network
    directions must reach the misfit the plain method ends with after four
    iterations in fewer GPU-seconds, and end at a lower misfit."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd.fwi import fwi
    from paper_2502_12350_amd.precond import Preconditioner, TRAINED
    w, g, P, shots = _case(torch)
    say("[precond] 4 FWI iterations, plane step vs plain, GPU-s to equal misfit")
    net = Preconditioner.load(TRAINED)
    v0 = torch.from_numpy(w.vel).cuda()
    tr = {}
    for method in ("sd", "cnn_span"):
        _, tr[method] = fwi(P, g, v0, None, shots, n_iter=4, method=method,
                            bounds=(1500.0, 4500.0), zero_top_planes=10, precond=net)
        say(f"  {method}: misfit {tr[method].misfit[0]:.4e} -> {tr[method].misfit[-1]:.4e} in "
            f"{tr[method].gpu_seconds[-1]:.2f} GPU-s ({tr[method].n_misfits} forward misfits, "
            f"{tr[method].n_network} plane steps)")
    sd, span = tr["sd"], tr["cnn_span"]
    target = sd.misfit[-1] / sd.misfit[0]
    t_sd, t_span = sd.time_to_reach(target), span.time_to_reach(target)
    say(f"  GPU-s to the plain method's final misfit: plain {t_sd:.2f}, plane step {t_span}")
    assert t_span is not None and t_span < t_sd
    assert span.misfit[-1] < sd.misfit[-1]
    assert span.n_network > 0
