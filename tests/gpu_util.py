"""Shared helpers of the GPU tests (run the library and the oracle on one input)."""

import sys

import numpy as np
import pytest

import oracle
import seisgen


def gpu_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def propagator(w, vel=None, rho="same"):
    """Library context with the workload's model loaded."""
    torch = gpu_or_skip()
    from paper_2502_12350_amd import Propagator, GridSpec
    P = Propagator(0)
    g = GridSpec(**w.grid_kwargs())
    v = w.vel if vel is None else vel
    r = w.rho if isinstance(rho, str) else rho
    P.set_model(g, torch.from_numpy(np.ascontiguousarray(v)).cuda(),
                None if r is None else torch.from_numpy(np.ascontiguousarray(r)).cuda())
    return P


def gpu_forward(w, src=None, rec=None, vel=None, rho="same", final=False):
    torch = gpu_or_skip()
    P = propagator(w, vel, rho)
    wav = torch.from_numpy(w.wavelet).cuda()
    out = P.forward(wav, w.sources[0] if src is None else src,
                    w.receivers if rec is None else rec, final=final)
    torch.cuda.synchronize()
    if final:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


def oracle_grid(w):
    return oracle.Grid(**w.grid_kwargs())
