"""Oracle references computed in background threads while the GPU tests run.

The FP64 oracle is plain numpy, whose large array operations release the
interpreter lock, so a few references computed in threads overlap each other
and the GPU tests that run meanwhile.  Threads (not processes) are used so that
nothing is forked or executed once the GPU is in use.  ``start`` is called from
the collection hook in ``conftest.py`` when a test that needs a reference is
selected; ``result`` waits for one (starting it first if needed).
"""

from __future__ import annotations

import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import seisgen

_pool = None
_jobs = {}
_lock = threading.Lock()


def c2_small_case(variant: str):
    """c2_small (93 x 77 x 61 + 16, 300 steps, 1748 receivers) with the
    density ("vd"), without it ("cd") or with a free surface ("fs")."""
    w = seisgen.workload("c2_small")
    if variant == "cd":
        w.rho = None
    return w, variant == "fs"


def _gradient_c2_small(variant: str):
    w, fs = c2_small_case(variant)
    kw = w.grid_kwargs()
    g = oracle.Grid(**kw, free_surface=fs)
    true = w.extra["v_true"]
    dobs = oracle.forward(g, true, w.rho, w.wavelet, w.sources[0], w.receivers).seis
    dobs = dobs.astype(np.float32)
    ref = oracle.gradient(g, w.vel, w.rho, w.wavelet, w.sources[0], w.receivers, dobs,
                          illumination=True)
    return dobs, ref


_wl = {}


def cached_workload(name: str):
    """seisgen.workload(name), built once per session (c2_crop cuts the 512^3
    c2 model, about 20 s)."""
    with _lock:
        if name not in _wl:
            _wl[name] = seisgen.workload(name)
        return _wl[name]


def _forward_c2_crop():
    w = cached_workload("c2_crop")
    return oracle.forward(oracle.Grid(**w.grid_kwargs()), w.vel, w.rho, w.wavelet, w.sources[0],
                          w.receivers)


CASES = {
    "c2_small_vd": lambda: _gradient_c2_small("vd"),
    "c2_small_cd": lambda: _gradient_c2_small("cd"),
    "c2_small_fs": lambda: _gradient_c2_small("fs"),
    "c2_crop": _forward_c2_crop,
}


def start(names):
    global _pool
    with _lock:
        if _pool is None:
            _pool = ThreadPoolExecutor(max_workers=4, thread_name_prefix="oracle")
        for n in names:
            if n not in _jobs:
                _jobs[n] = _pool.submit(CASES[n])


def result(name):
    start([name])
    return _jobs[name].result()
