#!/usr/bin/env python3
"""Throughput of the acoustic FD hot path on one MI355X.

One bench step = one full pass of the hot path for one shot on the
variable-density 512^3 model with a 32-cell sponge (576^3 = 191,102,976
padded points), 2000 time steps, 65,536 receivers:
  model prep is done once (untimed); each step runs the forward sweep with
  source injection and receiver recording, the misfit, the reverse sweep
  (adjoint step fused with the imaging condition) with binomial
  checkpointing of the forward states, and the gradient fold.

value = padded points x (nt forward + nt adjoint updates) / step time, in
Gpt/s (recomputation of checkpointed states is overhead, not counted).
Per-kernel averages come from HIP events recorded around every launch on
the library's stream during the timed region.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2502_12350_amd", "csrc", "wfd_step.hip")


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def committed_traffic(kernel: str, density: str):
    """HBM bytes per launch of `kernel` ("variable" or "constant" density) from
    the committed counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    pat = re.compile(r"^TRAFFIC kernel=(\S+) density=(\S+) source=(\S+) bytes_per_launch=(\d+)")
    for line in open(path):
        m = pat.match(line.strip())
        if m and m.group(1) == kernel and m.group(2) == density and m.group(3) == kernel_hash():
            return int(m.group(4))
    return None


def cpu_baseline(w, n_steps: int = 2):
    """The FP64 oracle on a bounded sample of the same workload: forward and
    adjoint(+imaging) steps on a 32-plane model crop with the same 32-cell
    sponge (576 x 576 x 96 padded points), one process."""
    import numpy as np
    import oracle

    z0 = w.nz // 2 - 16
    crop = dict(w.grid_kwargs())
    crop["nz"] = 32
    g = oracle.Grid(**crop)
    vel = w.vel[z0:z0 + 32].astype(np.float64)
    rho = None if w.rho is None else w.rho[z0:z0 + 32].astype(np.float64)
    c = oracle.coefficients(g, vel, rho)
    rng = np.random.default_rng(0)
    shape = g.padded_shape
    f = [rng.standard_normal(shape) * 1e-6 for _ in range(4)]
    gacc = np.zeros(shape)
    t_f = t_a = 0.0
    for _ in range(n_steps):
        t0 = time.perf_counter()
        f[1] = oracle.step(c, g, f[0], f[1])
        t1 = time.perf_counter()
        f[3] = oracle.step(c, g, f[2], f[3])
        gacc += f[2] * (oracle.laplacian(f[0], g.h) - c.m2 * f[0])
        t2 = time.perf_counter()
        t_f += t1 - t0
        t_a += t2 - t1
        f = [f[1], f[0], f[3], f[2]]
    pts = shape[0] * shape[1] * shape[2]
    gpts = 2 * n_steps * pts / (t_f + t_a) / 1e9
    return {"value": gpts, "unit": "Gpt/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_steps} forward + {n_steps} adjoint/imaging FP64 numpy steps on a "
                      f"{shape[2]}x{shape[1]}x{shape[0]} padded slab (32-plane model crop, same "
                      f"32-cell sponge), single process",
            "host_cpus": os.cpu_count(),
            "seconds": round(t_f + t_a, 2),
            "legs": cpu_legs()}


def cpu_legs(n_steps: int = 2):
    """The other workloads' oracle figures, one process: the whole 64^3 plain
    forward run (200 steps on 80^3 padded points), and one shot of the
    gradient workload (240 x 240 x 200 padded, 1200 steps) estimated from
    timed steps: the oracle's gradient takes nt forward steps, about nt more
    to recompute its segments, and nt adjoint steps with the imaging term."""
    import numpy as np
    import oracle
    import seisgen

    c1 = seisgen.workload("c1")
    t0 = time.perf_counter()
    oracle.forward(oracle.Grid(**c1.grid_kwargs()), c1.vel, c1.rho, c1.wavelet, c1.sources[0],
                   c1.receivers)
    t_c1 = time.perf_counter() - t0
    c4 = seisgen.workload("c4_start")
    g = oracle.Grid(**c4.grid_kwargs())
    c = oracle.coefficients(g, c4.vel.astype(np.float64), None)
    shape = g.padded_shape
    rng = np.random.default_rng(1)
    f = [rng.standard_normal(shape) * 1e-6 for _ in range(4)]
    gacc = np.zeros(shape)
    t_f = t_a = 0.0
    for _ in range(n_steps):
        t0 = time.perf_counter()
        f[1] = oracle.step(c, g, f[0], f[1])
        t1 = time.perf_counter()
        f[3] = oracle.step(c, g, f[2], f[3])
        gacc += f[2] * (oracle.laplacian(f[0], g.h) - c.m2 * f[0])
        t2 = time.perf_counter()
        t_f += t1 - t0
        t_a += t2 - t1
        f = [f[1], f[0], f[3], f[2]]
    per_f, per_a = t_f / n_steps, t_a / n_steps
    shot = c4.nt * (2 * per_f + per_a)
    pts4 = shape[0] * shape[1] * shape[2]
    return {"c1_full_run": {"seconds": round(t_c1, 2),
                            "gpts": round(c1.padded_points * c1.nt / t_c1 / 1e9, 5),
                            "what": "oracle.forward, 64^3 + 8-cell sponge, 200 steps, 64 receivers"},
            "c4_shot_estimate": {"seconds": round(shot, 1),
                                 "gpts": round(2 * c4.nt * pts4 / shot / 1e9, 5),
                                 "what": f"{c4.nt} x (2 forward + 1 adjoint/imaging) steps at "
                                         f"{shape[2]}x{shape[1]}x{shape[0]}, from "
                                         f"{n_steps} timed steps of each",
                                 "forward_step_s": round(per_f, 3),
                                 "adjoint_step_s": round(per_a, 3)}}


def copy_probe(gib: float = 4.0, reps: int = 10):
    """Streaming references of known size: a plain device copy (also the
    counter calibration) and a 3-read / 1-write elementwise kernel."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    c = torch.ones_like(a)
    d = torch.ones_like(a)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_copy = timed(lambda: b.copy_(a))
    t_r3w1 = timed(lambda: torch.addcmul(a, c, d, out=b))
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "copy_GBps": round(8 * n / t_copy / 1e9, 1),
                      "addcmul_r3w1_GBps": round(16 * n / t_r3w1 / 1e9, 1)}), flush=True)


def _probe_lib():
    """bench_probe.so: the streaming probe kernels (bench_probe.hip, built by
    __graft_entry__.build()); measurement code, not part of the library."""
    import ctypes as C
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_probe.so")
    if not os.path.exists(path):
        raise SystemExit(f"{path} is missing: run __graft_entry__.build() first")
    L = C.CDLL(path)
    L.bench_stream_probe.restype = C.c_int
    L.bench_stream_probe.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_int,
                                     C.c_void_p]
    L.bench_march_probe.restype = C.c_int
    L.bench_march_probe.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                    C.c_int, C.c_void_p]
    return L


def stream_probe(reps: int = 10):
    """Achievable streaming bandwidth: plain float4 probe kernels (no reuse)
    reading R and writing W arrays of 576^3 floats, over several grid sizes,
    plain and nontemporal; the best rate per mix."""
    import ctypes as C
    import torch
    L = _probe_lib()
    n = 576 ** 3
    buf = torch.ones(8 * n, dtype=torch.float32, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rows = {}
    for r, w in ((1, 1), (3, 1), (4, 1), (6, 2)):
        best = None
        for nt in (0, 1):
            for blocks in (2048, 8192, 32768):
                def run():
                    rc = L.bench_stream_probe(r, w, nt, buf.data_ptr(), n, blocks, st)
                    if rc != 0:
                        raise RuntimeError(f"bench_stream_probe failed with HIP error {rc}")
                for _ in range(2):
                    run()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    run()
                e1.record()
                torch.cuda.synchronize()
                gbs = (r + w) * 4.0 * n / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
                print(f"[stream-probe] R{r}W{w} nontemporal {nt} blocks {blocks}: {gbs:.0f} GB/s",
                      file=sys.stderr, flush=True)
                if best is None or gbs > best[0]:
                    best = (gbs, nt, blocks)
        rows[f"r{r}w{w}"] = {"GBps": round(best[0], 0), "nontemporal": best[1], "blocks": best[2]}
    # the step kernels' own pattern: 64-wide column tiles marching z chunks of
    # 192 planes (3 chunks at 576^3, as the cost model picks for both kernels)
    march = {}
    for r, w, tile in ((4, 1, "64x16"), (6, 2, "64x32")):
        def run_m():
            rc = L.bench_march_probe(r, w, buf.data_ptr(), 576, 576, 576, 192, st)
            if rc != 0:
                raise RuntimeError(f"bench_march_probe failed with HIP error {rc}")
        for _ in range(2):
            run_m()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            run_m()
        e1.record()
        torch.cuda.synchronize()
        gbs = (r + w) * 4.0 * n / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
        print(f"[stream-probe] tile march R{r}W{w} {tile} tiles, 192-plane chunks: {gbs:.0f} GB/s",
              file=sys.stderr, flush=True)
        march[f"r{r}w{w}"] = {"GBps": round(gbs, 0), "tile": tile, "z_chunk": 192}
    print(json.dumps({"metric": "streaming probe bandwidth", "unit": "GB/s", "n_floats_per_array": n,
                      "best": rows, "tile_march": march}), flush=True)


def fwi_bench(n_iter: int):
    """FWI on the gradient workload: 200x200x160 model + 20-cell sponge, 1200
    steps, 8 shots x 2500 receivers, true model = smooth background + six
    +/-10 % blobs, start = background, constant density.  Observed data come
    from the library's forward modeling on the true model.  Reports misfit
    versus GPU-seconds for steepest descent on the illumination-compensated
    gradient and for projected L-BFGS, and one shot's gradient with full
    storage versus 20 stored pairs."""
    import numpy as np
    import torch
    import seisgen
    from paper_2502_12350_amd import GridSpec, Propagator, checkpoint_plan
    from paper_2502_12350_amd.fwi import Shots, fwi

    w = seisgen.workload("c4_start")
    g = GridSpec(**w.grid_kwargs())
    dev = torch.device("cuda", 0)
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(w.extra["v_true"]).to(dev))
    wav = torch.from_numpy(w.wavelet).to(dev)
    dobs = [P.forward(wav, s, w.receivers).clone() for s in w.sources]
    torch.cuda.synchronize()
    P.release_workspace()
    shots = Shots(wav, np.asarray(w.sources), [w.receivers] * len(w.sources), dobs)
    v0 = torch.from_numpy(w.vel).to(dev)
    vt = w.extra["v_true"]
    out = {"metric": "FWI misfit cut per GPU-s", "unit": "1/GPU-s", "higher_is_better": True,
           "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "FWI, 200x200x160 model + 20-cell sponge, 1200 steps, 8 shots, "
                                  "2500 receivers, smooth background + six +/-10 % blobs",
                      "iterations": n_iter, "bounds_m_s": [1500.0, 4500.0],
                      "zero_top_planes": 24,
                      "preconditioner": "g / (I + 1e-3 max I), I = source illumination"},
           "methods": {}}
    for method in ("sd", "lbfgs"):
        print(f"[bench-fwi] {method}", file=sys.stderr, flush=True)
        # sources and receivers sit at depth index 4 and the anomalies start at 40:
        # the acquisition footprint in the top 24 gradient planes is zeroed
        # (ZeroesNearSurface of Alg. 3)
        v, tr = fwi(P, g, v0, None, shots, n_iter=n_iter, method=method, bounds=(1500.0, 4500.0),
                    zero_top_planes=24)
        out["methods"][method] = {
            "misfit": [float(x) for x in tr.misfit],
            "gpu_seconds": [round(t, 3) for t in tr.gpu_seconds],
            "misfit_cut_per_gpu_s": tr.misfit_cut_per_gpu_s(),
            "gpu_s_to_half_misfit": tr.time_to_reach(0.5),
            "gradients": tr.n_gradients, "forward_misfits": tr.n_misfits,
            "model_error_rel": float(np.linalg.norm(v.cpu().numpy() - vt) / np.linalg.norm(w.vel - vt)),
        }
    out["value"] = out["methods"]["lbfgs"]["misfit_cut_per_gpu_s"]
    # one shot: full storage vs binomial checkpointing with 20 stored pairs
    P.set_model(g, v0)
    ck_out = {}
    for ck in ("full", ("revolve", 20)):
        P._workspace(P.workspace_bytes(len(w.receivers), ck))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, grad = P.gradient(wav, w.sources[0], w.receivers, dobs[0], ckpt=ck)
        torch.cuda.synchronize()
        ck_out[str(ck[0] if isinstance(ck, tuple) else ck)] = {
            "seconds": round(time.perf_counter() - t0, 4),
            "workspace_GiB": round(P.workspace_bytes(len(w.receivers), ck) / 2**30, 2),
            "grad": grad.clone()}
        P.release_workspace()
    _, steps = checkpoint_plan(w.nt, 20)
    out["checkpointing_one_shot"] = {
        "full": {k: v for k, v in ck_out["full"].items() if k != "grad"},
        "revolve_20_pairs": {**{k: v for k, v in ck_out["revolve"].items() if k != "grad"},
                             "forward_steps": steps},
        "bitwise_equal": bool(torch.equal(ck_out["full"]["grad"], ck_out["revolve"]["grad"]))}
    print(json.dumps(out), flush=True)


def cpml_forward_bench(steps: int):
    """The 576^3 variable-density forward with the CPML layer for a few steps
    (the workload the layer kernels' trace and counters in profiles/ come
    from): ms per step and the layer kernels' share."""
    import time
    import torch
    import seisgen
    from paper_2502_12350_amd import GridSpec, Propagator, K_FORWARD, K_OTHER
    dev = torch.device("cuda", 0)
    c2 = seisgen.workload("c2")
    gs = GridSpec(**{**c2.grid_kwargs(), "nt": steps}, cpml=True, fpeak=10.0)
    R = Propagator(0)
    R.set_model(gs, torch.from_numpy(c2.vel).to(dev), torch.from_numpy(c2.rho).to(dev))
    wv = torch.from_numpy(c2.wavelet[:steps]).to(dev)
    R.forward(wv, c2.sources[0], c2.receivers)  # warm-up
    torch.cuda.synchronize()
    R.set_profiling(True)
    t0 = time.perf_counter()
    R.forward(wv, c2.sources[0], c2.receivers)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    nf, msf = R.kernel_stats(K_FORWARD)
    no, mso = R.kernel_stats(K_OTHER)
    R.set_profiling(False)
    print(json.dumps({"metric": "CPML forward step", "unit": "ms", "higher_is_better": False,
                      "n_gpus": 1, "dtype": "f32", "data": "synthetic", "steps": steps,
                      "config": {"workload": "576^3 padded VD (c2 model), 32-cell CPML layer"},
                      "ms_per_step": round(wall, 3), "step_kernel_us": round(1e3 * msf / nf, 1),
                      "layer_kernels_us_per_step": round(1e3 * mso / steps, 1)}), flush=True)


def options_bench():
    """Cost of the paper's boundary and storage options.  (1) One gradient shot
    of the 200x200x160 + 20 workload (1200 steps, 2500 receivers) with the
    forward wavefield in device memory, in 20 binomial checkpoints and in
    pinned host memory over PCIe, and with the CPML layer instead of the
    sponge (full storage).  (2) The 576^3 variable-density forward (c2 model,
    100 steps) with the sponge and with the CPML layer."""
    import numpy as np
    import torch
    import seisgen
    from paper_2502_12350_amd import GridSpec, Propagator, K_FORWARD, K_OTHER

    dev = torch.device("cuda", 0)
    out = {"metric": "seconds per gradient shot / ms per forward step by option", "unit": "s",
           "n_gpus": 1, "dtype": "f32", "data": "synthetic", "config": {}}

    w = seisgen.workload("c4_start")
    g = GridSpec(**w.grid_kwargs())
    wav = torch.from_numpy(w.wavelet).to(dev)
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(w.extra["v_true"]).to(dev))
    dobs = P.forward(wav, w.sources[0], w.receivers).clone()
    P.set_model(g, torch.from_numpy(w.vel).to(dev))
    rows, grads = {}, {}

    def timed_gradient(Q, ck, name):
        Q.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=ck)  # warm (allocations)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, gr = Q.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=ck)
        torch.cuda.synchronize()
        rows[name] = {"seconds": round(time.perf_counter() - t0, 4),
                      "device_workspace_GiB": round(Q.workspace_bytes(len(w.receivers), ck) / 2**30, 2)}
        grads[name] = gr.clone()
        print(f"[bench-options] gradient {name}: {rows[name]}", file=sys.stderr, flush=True)

    timed_gradient(P, "full", "full_device")
    P.release_workspace()
    timed_gradient(P, ("revolve", 20), "revolve_20_pairs")
    P.release_workspace()
    timed_gradient(P, "host", "host_memory")
    rows["host_memory"]["host_GiB"] = round(P.host_store_bytes() / 2**30, 2)
    P.release_workspace()
    del P
    torch.cuda.empty_cache()
    Q = Propagator(0)
    gc = GridSpec(**w.grid_kwargs(), cpml=True, fpeak=10.0)
    Q.set_model(gc, torch.from_numpy(w.vel).to(dev))
    timed_gradient(Q, "full", "cpml_full_device")
    del Q
    torch.cuda.empty_cache()
    out["gradient_one_shot_200x200x160"] = {
        **rows,
        "bitwise_equal_full_revolve_host": bool(torch.equal(grads["full_device"], grads["revolve_20_pairs"])
                                               and torch.equal(grads["full_device"], grads["host_memory"]))}

    c2 = seisgen.workload("c2")
    fw = {}
    for cp in (False, True):
        nt = 100
        gs = GridSpec(**{**c2.grid_kwargs(), "nt": nt}, cpml=cp, fpeak=10.0)
        R = Propagator(0)
        R.set_model(gs, torch.from_numpy(c2.vel).to(dev), torch.from_numpy(c2.rho).to(dev))
        wv = torch.from_numpy(c2.wavelet[:nt]).to(dev)
        R.forward(wv, c2.sources[0], c2.receivers)
        torch.cuda.synchronize()
        R.set_profiling(True)
        t0 = time.perf_counter()
        R.forward(wv, c2.sources[0], c2.receivers)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / nt
        nf, msf = R.kernel_stats(K_FORWARD)
        no, mso = R.kernel_stats(K_OTHER)
        R.set_profiling(False)
        fw["cpml" if cp else "sponge"] = {"ms_per_step": round(wall, 3),
                                          "step_kernel_us": round(1e3 * msf / nf, 1),
                                          "other_kernels_us_per_step": round(1e3 * mso / nt, 1)}
        print(f"[bench-options] forward 576^3 {'cpml' if cp else 'sponge'}: {fw['cpml' if cp else 'sponge']}",
              file=sys.stderr, flush=True)
        R.release_workspace()
        del R
        torch.cuda.empty_cache()
    out["forward_576_vd"] = fw
    out["config"] = {"workload": "gradient: 200x200x160 + 20 sponge/layer, 1200 steps, 2500 receivers, "
                                 "one shot; forward: 512^3 VD + 32, 100 steps, 65536 receivers"}
    print(json.dumps(out), flush=True)


def batch_bench(steps: int, warmup: int, autotune: bool):
    """Batched multi-shot forward: 24 shots on the 400x400x256 variable-density
    model, each on its own aperture window (sides 160-320 cells, clipped),
    32-cell sponge, 1500 steps.  Compares one wfd_forward per shot with one
    launch per step over all windows, eager and replayed as a HIP graph."""
    import torch
    import seisgen
    from paper_2502_12350_amd import GridSpec, Propagator, ShotBatch

    w = seisgen.workload("c3")
    shots = [seisgen.shot_window(w, i) for i in range(len(w.sources))]
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream()
    props = []
    for s in shots:
        P = Propagator(0)
        P.set_model(GridSpec(**s.grid_kwargs()), torch.from_numpy(s.vel).to(dev),
                    torch.from_numpy(s.rho).to(dev))
        props.append(P)
    wav = torch.from_numpy(w.wavelet).to(dev)
    pts = sum(s.padded_points for s in shots)
    print(f"[bench-batch] {len(shots)} windows, {pts / 1e6:.1f} M padded points, nt {w.nt}",
          file=sys.stderr, flush=True)
    tuned = None
    if autotune:
        tuned = [P.autotune(steps=10)[0] for P in props]
        print(f"[bench-batch] autotuned {tuned}", file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        batch = ShotBatch(props, wav, [s.sources[0] for s in shots], [s.receivers for s in shots],
                          stream=stream)

        def per_shot():
            for s, P in zip(shots, props):
                P.forward(wav, s.sources[0], s.receivers)

        modes = {"per_shot": per_shot, "batched_eager": lambda: batch.run(use_graph=False),
                 "batched_graph": lambda: batch.run(use_graph=True)}
        res = {}
        for name, fn in modes.items():
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                fn()
                torch.cuda.synchronize()
                print(f"[bench-batch] {name} step {i + 1}/{steps} done", file=sys.stderr,
                      flush=True)
            dt = (time.perf_counter() - t0) / steps
            res[name] = {"ms_per_pass": round(dt * 1e3, 2), "gpts": round(pts * w.nt / dt / 1e9, 2)}
    out = {"metric": "batched multi-shot forward throughput", "unit": "Gpt/s",
           "value": res["batched_graph"]["gpts"], "higher_is_better": True, "n_gpus": 1,
           "steps": steps, "warmup": warmup, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "24 shots, 400x400x256 variable-density model, per-shot "
                                  "aperture windows of side 160-320 cells (clipped), 32-cell "
                                  "sponge, 1500 steps",
                      "padded_points_all_windows": pts,
                      "tile_variant": props[0].tuning()[0],
                      "autotuned": tuned},
           "modes": res,
           "speedup_graph_vs_per_shot": round(res["batched_graph"]["gpts"] /
                                              res["per_shot"]["gpts"], 3)}
    batch.close()
    print(json.dumps(out), flush=True)


def batch_fwi_bench(n_iter: int = 3):
    """Windowed FWI on the batched-shot workload: 24 shots on the 400x400x256
    variable-density model, each on its own aperture window (160-320 cells,
    clipped, full depth), 1500 steps; true model = the layered model with eight
    +/-8 % blobs, start = the layered model, density fixed.  Each iteration adds
    every window's gradient (binomial checkpointing, 24 pairs) into the model
    gradient and takes a steepest-descent step on g / (I + 1e-3 max I) with a
    quadratic line search.  The two runs differ only in how the shots are
    launched: one wfd_gradient / wfd_forward per window, or all windows
    advanced together (one launch per forward or adjoint step, the gradients
    replayed as one HIP graph).  Both produce bitwise the same gradients,
    traces and misfits, so they follow the same misfit sequence and only the
    GPU time differs."""
    import numpy as np
    import torch
    import seisgen
    from paper_2502_12350_amd import GradientBatch, GridSpec, Propagator, ShotBatch

    dev = torch.device("cuda", 0)
    w = seisgen.workload("c3")
    vtrue = seisgen.blob_anomalies(w.vel, seed=41, n_blobs=8, amp=0.08, sigma_cells=(8.0, 16.0),
                                   centre_lo=(60, 60, 60), centre_hi=(340, 340, 200))
    rho = torch.from_numpy(w.rho).to(dev)
    wins = [tuple(int(v) for v in win) for win in w.extra["windows"]]
    shots = [seisgen.shot_window(w, i) for i in range(len(w.sources))]
    wav = torch.from_numpy(w.wavelet).to(dev)
    props = [Propagator(0) for _ in shots]

    def load(v):
        for (x0, x1, y0, y1), s, P in zip(wins, shots, props):
            P.set_model(GridSpec(**s.grid_kwargs()), v[:, y0:y1, x0:x1].contiguous(),
                        rho[:, y0:y1, x0:x1].contiguous())

    load(torch.from_numpy(vtrue).to(dev))
    dobs = [P.forward(wav, s.sources[0], s.receivers).clone() for s, P in zip(shots, props)]
    torch.cuda.synchronize()

    def misfit(v, batched):
        load(v)
        if batched:  # set_model gives new coefficient buffers: a new batch each time
            b = ShotBatch(props, wav, [s.sources[0] for s in shots], [s.receivers for s in shots])
            seis = b.run()
            J = sum(0.5 * float(torch.sum((a.double() - d.double()) ** 2))
                    for a, d in zip(seis, dobs))
            b.close()
        else:
            J = sum(0.5 * float(torch.sum((P.forward(wav, s.sources[0], s.receivers).double()
                                           - d.double()) ** 2))
                    for s, P, d in zip(shots, props, dobs))
        return J

    def gradient(v, batched):
        load(v)
        g = torch.zeros_like(v)
        il = torch.zeros_like(v)
        if batched:  # every window's gradient together: one launch per step
            side = torch.cuda.Stream()
            torch.cuda.synchronize()
            with torch.cuda.stream(side):
                b = GradientBatch(props, wav, [s.sources[0] for s in shots],
                                  [s.receivers for s in shots], dobs, 24, illum=True,
                                  stream=side)
                b.run(use_graph=True)
            torch.cuda.synchronize()
            for (x0, x1, y0, y1), gi, ii in zip(wins, b.grad, b.illum):
                g[:, y0:y1, x0:x1] += gi
                il[:, y0:y1, x0:x1] += ii
            b.close()
            del b
        else:
            for (x0, x1, y0, y1), s, P, d in zip(wins, shots, props, dobs):
                gi = torch.zeros((s.nz, s.ny, s.nx), dtype=torch.float32, device=dev)
                ii = torch.zeros_like(gi)
                P.gradient(wav, s.sources[0], s.receivers, d, ckpt=("revolve", 24), grad=gi,
                           illum=ii)
                P.release_workspace()
                g[:, y0:y1, x0:x1] += gi
                il[:, y0:y1, x0:x1] += ii
        g[:16] = 0.0  # ZeroesNearSurface: sources and receivers sit in the top planes
        return g, il

    out = {"metric": "FWI misfit cut per GPU-s, batched vs per-shot trial misfits",
           "unit": "1/GPU-s", "higher_is_better": True, "n_gpus": 1, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "windowed FWI, 24 shots on a 400x400x256 VD model, windows "
                                  "160-320 cells, 32-cell sponge, 1500 steps, eight +/-8 % blobs",
                      "iterations": n_iter, "checkpoint": "binomial, 24 pairs per window"},
           "modes": {}}
    v0 = torch.from_numpy(w.vel).to(dev)
    for batched in (False, True):
        name = "batched" if batched else "per_shot"
        v = v0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_mis = t_grad = 0.0
        J0 = misfit(v, batched)
        hist, secs = [J0], [time.perf_counter() - t0]
        for it in range(n_iter):
            tg = time.perf_counter()
            g, il = gradient(v, batched)
            torch.cuda.synchronize()
            t_grad += time.perf_counter() - tg
            d = -g / (il + 1e-3 * il.max())
            slope = float(torch.sum(g.double() * d.double()))
            a1 = 30.0 / float(d.abs().max())   # first trial moves the model by 30 m/s at most
            tm = time.perf_counter()
            J1 = misfit(torch.clamp(v + a1 * d, 1500.0, 4500.0), batched)
            curv = 2.0 * (J1 - hist[-1] - slope * a1) / (a1 * a1)
            a = min(max(-slope / curv, 0.1 * a1), 4.0 * a1) if curv > 0 else 2.0 * a1
            Ja = misfit(torch.clamp(v + a * d, 1500.0, 4500.0), batched)
            t_mis += time.perf_counter() - tm
            if Ja <= J1:
                v = torch.clamp(v + a * d, 1500.0, 4500.0)
                hist.append(Ja)
            else:
                v = torch.clamp(v + a1 * d, 1500.0, 4500.0)
                hist.append(J1)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            print(f"[bench-batch-fwi] {name} iteration {it + 1}: misfit {hist[-1]:.6e} "
                  f"({secs[-1]:.1f} s)", file=sys.stderr, flush=True)
        out["modes"][name] = {"misfit": hist, "gpu_seconds": [round(x, 3) for x in secs],
                              "line_search_seconds": round(t_mis, 3),
                              "gradient_seconds": round(t_grad, 3),
                              "misfit_cut_per_gpu_s": (hist[0] - hist[-1]) / hist[0] / secs[-1]}
    ps, bt = out["modes"]["per_shot"], out["modes"]["batched"]
    out["equal_misfit_sequences"] = ps["misfit"] == bt["misfit"]
    out["value"] = bt["misfit_cut_per_gpu_s"]
    out["ratio_batched_vs_per_shot"] = round(bt["misfit_cut_per_gpu_s"] / ps["misfit_cut_per_gpu_s"], 4)
    print(json.dumps(out), flush=True)


def batch_gradient_bench(name: str = "c3_narrow", n_snapshots: int = 8):
    """Per-window gradients of a windowed workload, one wfd_gradient per window
    against all windows together (wfd_gbatch: one launch per forward and
    adjoint step over every window, replayed as a HIP graph), with the same
    binomial checkpointing; Gpt/s over all windows' padded points x (nt
    forward + nt adjoint updates).  The results are bitwise equal (GPU
    tests); only the time differs."""
    import numpy as np
    import torch
    import seisgen
    from paper_2502_12350_amd import GradientBatch, GridSpec, Propagator

    dev = torch.device("cuda", 0)
    w = seisgen.workload(name)
    shots = [seisgen.shot_window(w, i) for i in range(len(w.sources))]
    wav = torch.from_numpy(w.wavelet).to(dev)
    props = []
    for s in shots:
        P = Propagator(0)
        P.set_model(GridSpec(**s.grid_kwargs()), torch.from_numpy(s.vel).to(dev),
                    torch.from_numpy(s.rho).to(dev))
        props.append(P)
    rng = np.random.default_rng(7)
    dobs = [torch.from_numpy((rng.standard_normal((len(s.receivers), w.nt)) * 1e-12)
                             .astype(np.float32)).to(dev) for s in shots]
    pts = sum(s.padded_points for s in shots)

    def per_shot():
        for s, P, d in zip(shots, props, dobs):
            P.gradient(wav, s.sources[0], s.receivers, d, ckpt=("revolve", n_snapshots))

    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        b = GradientBatch(props, wav, [s.sources[0] for s in shots], [s.receivers for s in shots],
                          dobs, n_snapshots, stream=side)
    rows = {}
    for mode in ("per_shot", "batched_eager", "batched_graph"):
        def run():
            if mode == "per_shot":
                per_shot()
            else:
                with torch.cuda.stream(side):
                    b.run(use_graph=(mode == "batched_graph"))
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 3
        rows[mode] = {"seconds": round(dt, 4), "gpts": round(pts * 2 * w.nt / dt / 1e9, 2)}
        print(f"[bench-batch-gradient] {mode}: {rows[mode]}", file=sys.stderr, flush=True)
    b.close()
    out = {"metric": "batched per-window gradients: Gpt/s over all windows", "unit": "Gpt/s",
           "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{name}: {len(shots)} windows, padded sizes "
                                  f"{min(s.padded_points for s in shots)}-"
                                  f"{max(s.padded_points for s in shots)} points, {w.nt} steps",
                      "checkpoint": f"binomial, {n_snapshots} pairs per window"},
           "modes": rows,
           "value": rows["batched_graph"]["gpts"],
           "ratio_batched_vs_per_shot": round(rows["batched_graph"]["gpts"] /
                                              rows["per_shot"]["gpts"], 3)}
    print(json.dumps(out), flush=True)


def cnn_kernel_bench(n: int = 256, reps: int = 20):
    """Matrix-core throughput of the preconditioner's kernels on an n^3 volume:
    forward convolution of every layer, the 16 -> 16 data and weight
    gradients (the latter with its fixed-order reduction), and the whole
    forward and backward passes; useful flops = 2 * 27 * cin * cout per voxel."""
    import numpy as np
    import torch
    from paper_2502_12350_amd.precond import LAYERS, Preconditioner

    P = Preconditioner(0, seed=1)
    rng = np.random.default_rng(0)
    shape = (n, n, n)
    g = torch.from_numpy(rng.standard_normal(shape).astype(np.float32)).cuda()
    il = torch.from_numpy(np.abs(rng.standard_normal(shape)).astype(np.float32)).cuda()
    x = P.pack_input(g, il)
    vox = n ** 3
    gen = torch.Generator(device="cuda").manual_seed(0)
    a16 = torch.randn(shape + (16,), generator=gen, device="cuda").to(torch.bfloat16)

    def timed(fn):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    out = {}
    for li, (ci, co) in enumerate(LAYERS):
        inp = x if ci == 2 else a16
        t = timed(lambda: P.conv(inp, li, relu=li < 3, out_f32=li == 3))
        fl = 2.0 * 27 * ci * co * vox
        out[f"conv_l{li}_{ci}x{co}"] = {"us": round(t * 1e6, 1), "TFLOPs": round(fl / t / 1e12, 1)}
    t = timed(lambda: P.conv(a16, 1, relu=False, flip=True, bias=False, mask=a16))
    out["dgrad_16x16"] = {"us": round(t * 1e6, 1),
                          "TFLOPs": round(2.0 * 27 * 256 * vox / t / 1e12, 1)}
    import ctypes as C
    nb = C.c_size_t()
    P.L.wfd_cnn_wgrad_workspace_bytes(n, n, n, C.byref(nb))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    b16 = torch.randn(shape + (16,), generator=gen, device="cuda").to(torch.bfloat16)
    stream = torch.cuda.current_stream().cuda_stream

    def wgrad():
        rc = P.L.wfd_cnn_wgrad(a16.data_ptr(), b16.data_ptr(), n, n, n, 16, 16,
                               P.dw[1].data_ptr(), P.db[1].data_ptr(), work.data_ptr(), nb.value,
                               C.c_void_p(stream))
        assert rc == 0, rc

    t = timed(wgrad)
    out["wgrad_16x16"] = {"us": round(t * 1e6, 1),
                          "TFLOPs": round(2.0 * 27 * 256 * vox / t / 1e12, 1)}
    tgt = torch.zeros(shape, device="cuda")
    y = P.forward(x, keep=True)
    t = timed(lambda: P.backward(y, tgt))
    fl_fwd = sum(2.0 * 27 * ci * co * vox for ci, co in LAYERS)
    fl_bwd = fl_fwd + sum(2.0 * 27 * ci * co * vox for ci, co in LAYERS[1:])
    out["backward_all_layers"] = {"us": round(t * 1e6, 1), "TFLOPs": round(fl_bwd / t / 1e12, 1)}
    t = timed(lambda: P.forward(x))
    out["forward_all_layers"] = {"us": round(t * 1e6, 1), "TFLOPs": round(fl_fwd / t / 1e12, 1)}
    peak = 2500.0
    l1 = out["conv_l1_16x16"]
    res = {"metric": "CNN preconditioner matrix-core throughput", "unit": "TFLOP/s",
           "value": l1["TFLOPs"], "higher_is_better": True, "n_gpus": 1, "dtype": "bf16",
           "data": "synthetic", "config": {"workload": f"3-D CNN 2-16-16-16-1, 3x3x3, {n}^3 volume"},
           "roofline": {"bound": "mfma", "achieved": l1["TFLOPs"], "peak": peak,
                        "unit": "TFLOP/s", "frac": round(l1["TFLOPs"] / peak, 4),
                        "traffic": None, "kernel": "k_conv16<16>"},
           "kernels": out}
    print(json.dumps(res), flush=True)


def precond_fwi_bench(n_iter: int, methods=("sd", "cnn", "cnn_span")):
    """FWI with the learned preconditioner against the plain method: the
    256^3 recipe of the training models (seed 5999, never trained on), 20-cell
    sponge, 1600 steps, 8 shots, 4096 receivers, constant density; start =
    layered background, truth = background + 1-4 blobs.  Both runs use
    steepest descent with the same quadratic line search; 'sd' steps along the
    illumination-compensated gradient, 'cnn' along the network's direction
    (falling back to the former when it does not descend), 'cnn_span' in the
    plane of both directions (three trial misfits and the exact slopes fix a
    two-dimensional quadratic)."""
    import numpy as np
    import torch
    import seisgen
    from paper_2502_12350_amd import GridSpec, Propagator
    from paper_2502_12350_amd.fwi import Shots, fwi
    from paper_2502_12350_amd.precond import Preconditioner, TRAINED

    w = seisgen.workload("c5_eval")
    g = GridSpec(**w.grid_kwargs())
    dev = torch.device("cuda", 0)
    P = Propagator(0)
    P.set_model(g, torch.from_numpy(w.extra["v_true"]).to(dev))
    wav = torch.from_numpy(w.wavelet).to(dev)
    dobs = [P.forward(wav, s, w.receivers).clone() for s in w.sources]
    torch.cuda.synchronize()
    P.release_workspace()
    shots = Shots(wav, np.asarray(w.sources), [w.receivers] * len(w.sources), dobs)
    v0 = torch.from_numpy(w.vel).to(dev)
    vt = w.extra["v_true"]
    net = Preconditioner.load(TRAINED)
    vt_d = torch.from_numpy(vt).to(dev)
    err0 = float(torch.linalg.vector_norm((v0 - vt_d).double()))
    runs = {}
    for method in methods:
        print(f"[bench-precond] {method}", file=sys.stderr, flush=True)
        errs = [1.0]

        def progress(it, J, t, v):
            errs.append(float(torch.linalg.vector_norm((v - vt_d).double())) / err0)
            print(f"[bench-precond] {method} iteration {it + 1}: misfit {J:.4e}, model error "
                  f"{errs[-1]:.5f} at {t:.1f} GPU-s", file=sys.stderr, flush=True)

        v, tr = fwi(P, g, v0, None, shots, n_iter=n_iter, method=method, bounds=(1500.0, 4500.0),
                    zero_top_planes=10, precond=net, progress=progress)
        runs[method] = {
            "model_error_rel_per_iteration": [round(e, 6) for e in errs],
            "misfit": [float(x) for x in tr.misfit],
            "gpu_seconds": [round(t, 3) for t in tr.gpu_seconds],
            "misfit_cut_per_gpu_s": tr.misfit_cut_per_gpu_s(),
            "gradients": tr.n_gradients, "forward_misfits": tr.n_misfits,
            "network_steps": tr.n_network,
            "model_error_rel": float(np.linalg.norm(v.cpu().numpy() - vt) /
                                     np.linalg.norm(w.vel - vt)),
            "_trace": tr}
    sd, cnn, span = runs["sd"], runs.get("cnn"), runs["cnn_span"]
    target = sd["misfit"][-1]  # equal final misfit: the plain method's
    t_sd = sd["_trace"].time_to_reach(target / sd["misfit"][0])
    t_cnn = cnn["_trace"].time_to_reach(target / cnn["misfit"][0]) if cnn else None
    t_span = span["_trace"].time_to_reach(target / span["misfit"][0])

    def t_err(r, e):  # GPU-seconds until the model error is at most e
        for t, x in zip(r["gpu_seconds"], r["model_error_rel_per_iteration"]):
            if x <= e:
                return t
        return None

    e_target = sd["model_error_rel_per_iteration"][-1]
    te_sd, te_span = t_err(sd, e_target), t_err(span, e_target)
    te_cnn = t_err(cnn, e_target) if cnn else None
    for r in runs.values():
        r.pop("_trace")
    out = {"metric": "FWI misfit cut per GPU-s: learned preconditioner vs illumination-compensated "
                     "gradient", "unit": "x", "higher_is_better": True, "n_gpus": 1,
           "dtype": "f32 (stencil), bf16 (network)", "data": "synthetic",
           "value": round(t_sd / t_span, 3) if t_span else None,
           "config": {"workload": "FWI, 256^3 layered model + 1-4 blobs (seed 5999) + 20-cell "
                                  "sponge, 1600 steps, 8 shots, 4096 receivers",
                      "iterations": n_iter, "zero_top_planes": 10,
                      "network": "2-16-16-16-1 3x3x3 BF16, trained on 512 solver pairs (128^3)"},
           "value_method": "cnn_span (the step in the plane of the plain and network "
                           "directions); GPU-s of the plain method to its final misfit over "
                           "GPU-s of this method to the same misfit",
           "gpu_s_to_plain_final_misfit": {"sd": t_sd, "cnn": t_cnn, "cnn_span": t_span},
           "gpu_s_to_plain_final_model_error": {"sd": te_sd, "cnn": te_cnn, "cnn_span": te_span},
           "model_error_speedup": {"cnn": round(te_sd / te_cnn, 3) if te_cnn else None,
                                   "cnn_span": round(te_sd / te_span, 3) if te_span else None},
           "methods": runs}
    print(json.dumps(out), flush=True)


def kernel_table_bench(steps: int = 200):
    """Per-kernel rates: forward and adjoint at the 576^3 size, constant and
    variable density (%HBM there), the cache-resident 64^3 and 240x240x200
    forwards (Gpt/s only), against the nominal 8 TB/s and a streaming rate
    measured on the same box."""
    import numpy as np
    import torch
    import seisgen
    from paper_2502_12350_amd import GridSpec, Propagator, K_FORWARD, K_ADJOINT

    dev = torch.device("cuda", 0)
    # streaming reference: torch addcmul over 1 GiB arrays (3 reads + 1 write)
    n = 1 << 28
    a, b, c = (torch.ones(n, device=dev) for _ in range(3))
    o = torch.empty(n, device=dev)
    torch.addcmul(a, b, c, out=o)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.addcmul(a, b, c, out=o)
    e1.record()
    torch.cuda.synchronize()
    stream_gbs = 16.0 * n * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b, c, o
    torch.cuda.empty_cache()
    rows = {}

    def run(name, w, rho, adjoint, hbm):
        g = GridSpec(**{**w.grid_kwargs(), "nt": steps})
        P = Propagator(0)
        P.set_model(g, torch.from_numpy(w.vel).to(dev),
                    None if rho is None else torch.from_numpy(rho).to(dev))
        wav = torch.from_numpy(w.wavelet[:steps]).to(dev)
        rec = w.receivers
        if adjoint:
            dobs = torch.zeros((len(rec), steps), device=dev)
            ck = ("revolve", 8)
            P.gradient(wav, w.sources[0], rec, dobs, ckpt=ck)
            P.set_profiling(True)
            P.gradient(wav, w.sources[0], rec, dobs, ckpt=ck)
            nl, ms = P.kernel_stats(K_ADJOINT)
        else:
            P.forward(wav, w.sources[0], rec)
            P.set_profiling(True)
            P.forward(wav, w.sources[0], rec)
            nl, ms = P.kernel_stats(K_FORWARD)
        P.set_profiling(False)
        us = 1e3 * ms / nl
        pts, mpts = w.padded_points, w.nx * w.ny * w.nz
        bpp = (32 if adjoint else 20) if rho is not None else (28 if adjoint else 16)
        r = {"us_per_step": round(us, 1), "gpts_padded": round(pts / us / 1e3, 1),
             "gpts_model": round(mpts / us / 1e3, 1), "bytes_per_point": bpp}
        if hbm:
            gbs = pts * bpp / us / 1e3
            r.update({"GBps": round(gbs, 0), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
                      "frac_of_streaming": round(gbs / stream_gbs, 4)})
        rows[name] = r
        print(f"[bench-kernels] {name}: {r}", file=sys.stderr, flush=True)
        P.release_workspace()
        del P
        torch.cuda.empty_cache()

    c2 = seisgen.workload("c2")
    run("forward_vd_576", c2, c2.rho, False, True)
    run("forward_cd_576", c2, None, False, True)
    run("adjoint_vd_576", c2, c2.rho, True, True)
    run("adjoint_cd_576", c2, None, True, True)
    del c2
    c1 = seisgen.workload("c1")
    run("forward_cd_c1_80cubed", c1, None, False, False)
    # the same forward with its time loop replayed as one HIP graph (a one-shot
    # batch): on this launch-bound grid the graph removes the launch gaps
    from paper_2502_12350_amd import ShotBatch
    gs1 = GridSpec(**{**c1.grid_kwargs(), "nt": steps})
    P1 = Propagator(0)
    P1.set_model(gs1, torch.from_numpy(c1.vel).to(dev))
    side = torch.cuda.Stream()  # graph capture needs a non-default stream
    wav1 = torch.from_numpy(c1.wavelet[:steps]).to(dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        b1 = ShotBatch([P1], wav1, [c1.sources[0]], [c1.receivers], stream=side)
    for use_graph, tune in ((False, False), (True, False), (True, True)):
        if tune:  # launch shapes picked by the autotuner for this grid
            b1.close()
            tuned, fus, _ = P1.autotune(steps=20)
            print(f"[bench-kernels] c1 autotuned {tuned}: forward {fus:.1f} us per step",
                  file=sys.stderr, flush=True)
            with torch.cuda.stream(side):
                b1 = ShotBatch([P1], wav1, [c1.sources[0]], [c1.receivers], stream=side)
        with torch.cuda.stream(side):
            b1.run(use_graph)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(side)
            for _ in range(5):
                b1.run(use_graph)
            e1.record(side)
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / 5 / steps
        name = "forward_cd_c1_80cubed_" + ("graph" if use_graph else "batch_eager") + \
            ("_autotuned" if tune else "")
        rows[name] = {"us_per_step": round(us, 2), "gpts_padded": round(c1.padded_points / us / 1e3, 1),
                      "gpts_model": round(c1.nx * c1.ny * c1.nz / us / 1e3, 1), "bytes_per_point": 16,
                      "note": "wall time per step incl. launch gaps (events around the whole loop)"}
        print(f"[bench-kernels] {name}: {rows[name]}", file=sys.stderr, flush=True)
    b1.close()
    c4 = seisgen.workload("c4")
    run("forward_cd_c4_240x240x200", c4, None, False, False)
    out = {"metric": "per-kernel Gpt/s and %HBM", "unit": "Gpt/s", "n_gpus": 1, "dtype": "f32",
           "data": "synthetic", "steps": steps,
           "streaming_reference_GBps": round(stream_gbs, 0),
           "config": {"workload": "576^3 padded (c2 model), constant and variable density; "
                                  "80^3 (c1) and 240x240x200 (c4) cache-resident forwards"},
           "kernels": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--nt", type=int, default=0, help="override the number of time steps")
    ap.add_argument("--snapshots", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--constant-density", action="store_true",
                    help="drop the density model (constant-density kernels; not the headline)")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--stream-probe", action="store_true",
                    help="achievable streaming bandwidth of plain float4 kernels")
    ap.add_argument("--fwi", type=int, default=0, metavar="ITERS",
                    help="run the FWI benchmark with this many iterations per method instead")
    ap.add_argument("--options", action="store_true",
                    help="cost of wavefield storage modes and of the CPML layer")
    ap.add_argument("--cpml-forward", type=int, default=0, metavar="STEPS",
                    help="the 576^3 forward with the CPML layer (profiling workload)")
    ap.add_argument("--batch-fwi", type=int, default=0, metavar="ITERS",
                    help="windowed FWI: batched vs per-shot gradients and trial misfits")
    ap.add_argument("--batch-gradient", action="store_true",
                    help="per-window gradients of narrow windows: batched vs per-shot")
    ap.add_argument("--kernels", action="store_true",
                    help="per-kernel table: forward/adjoint CD and VD at 576^3, cache-resident sizes")
    ap.add_argument("--precond-methods", default="sd,cnn,cnn_span",
                    help="--precond-fwi: methods to run (sd and cnn_span are required)")
    ap.add_argument("--precond-fwi", type=int, default=0, metavar="ITERS",
                    help="run FWI with the learned preconditioner against the plain method")
    ap.add_argument("--cnn", type=int, default=0, metavar="N",
                    help="time the CNN preconditioner kernels on an N^3 volume instead")
    ap.add_argument("--batch", action="store_true",
                    help="run the batched multi-shot forward benchmark instead")
    ap.add_argument("--autotune", action="store_true",
                    help="time every step-kernel launch shape at setup (untimed) and keep "
                         "the fastest (with --batch: per window)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py: one GPU only (one shot per GPU; a multi-GPU run would shard the "
              "shots and all-reduce the gradient once per evaluation) -- "
              f"--gpus {args.gpus} is not supported", file=sys.stderr, flush=True)
        sys.exit(2)
    if args.stream_probe:
        stream_probe()
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.fwi:
        fwi_bench(args.fwi)
        return
    if args.batch:
        batch_bench(max(args.steps, 1), args.warmup, args.autotune)
        return
    if args.cnn:
        cnn_kernel_bench(args.cnn)
        return
    if args.precond_fwi:
        precond_fwi_bench(args.precond_fwi, tuple(args.precond_methods.split(",")))
        return
    if args.kernels:
        kernel_table_bench()
        return
    if args.batch_fwi:
        batch_fwi_bench(args.batch_fwi)
        return
    if args.batch_gradient:
        batch_gradient_bench()
        return
    if args.options:
        options_bench()
        return
    if args.cpml_forward:
        cpml_forward_bench(args.cpml_forward)
        return

    import numpy as np
    import torch
    import seisgen
    from paper_2502_12350_amd import GridSpec, Propagator, K_FORWARD, K_ADJOINT, K_OTHER

    t_setup = time.perf_counter()
    w = seisgen.workload(args.workload)
    if args.nt:
        w.nt = args.nt
        w.wavelet = w.wavelet[:args.nt]
    grid = GridSpec(**w.grid_kwargs())
    dev = torch.device("cuda", 0)
    vel = torch.from_numpy(w.vel).to(dev)
    rho = None if (w.rho is None or args.constant_density) else torch.from_numpy(w.rho).to(dev)
    wav = torch.from_numpy(w.wavelet).to(dev)
    nrec = len(w.receivers)
    print(f"[bench] workload {w.name}: model {w.nx}x{w.ny}x{w.nz}, padded "
          f"{w.padded_shape[2]}x{w.padded_shape[1]}x{w.padded_shape[0]}, nt {w.nt}, "
          f"nrec {nrec}, density {'variable' if rho is not None else 'constant'}",
          file=sys.stderr, flush=True)

    # observed data: forward on a perturbed ("true") model
    true = seisgen.blob_anomalies(w.vel, seed=2503, n_blobs=8, amp=0.05, sigma_cells=(10, 30),
                                  centre_lo=(64, 64, 64), centre_hi=(w.nx - 64, w.ny - 64,
                                                                      w.nz - 64))
    P = Propagator(0)
    P.set_model(grid, torch.from_numpy(true).to(dev), rho)
    dobs = P.forward(wav, w.sources[0], w.receivers)
    torch.cuda.synchronize()
    P.release_workspace()
    P.set_model(grid, vel, rho)
    del true
    if args.autotune:
        tuned, fus, aus = P.autotune(steps=10)
        print(f"[bench] autotuned {tuned}: forward {fus:.1f} us, adjoint {aus:.1f} us per step",
              file=sys.stderr, flush=True)
    ckpt = ("revolve", min(args.snapshots, w.nt))
    grad = torch.zeros((w.nz, w.ny, w.nx), dtype=torch.float32, device=dev)
    misfit = torch.zeros((), dtype=torch.float64, device=dev)
    print(f"[bench] setup {time.perf_counter() - t_setup:.1f}s; workspace "
          f"{P.workspace_bytes(nrec, ckpt) / 2**30:.1f} GiB", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        P.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=ckpt, grad=grad, misfit=misfit)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    P.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        P.gradient(wav, w.sources[0], w.receivers, dobs, ckpt=ckpt, grad=grad, misfit=misfit)
        torch.cuda.synchronize()
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    nf, msf = P.kernel_stats(K_FORWARD)
    na, msa = P.kernel_stats(K_ADJOINT)
    no, mso = P.kernel_stats(K_OTHER)
    P.set_profiling(False)

    pts = w.padded_points
    vd = rho is not None
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = pts * 2.0 * w.nt / (ms_step * 1e-3) / 1e9
    kern = {
        "fd_step": {"launches": nf, "avg_us": 1e3 * msf / max(nf, 1),
                    "bytes_per_point": 20 if vd else 16, "share": msf / (msf + msa + mso)},
        "adjoint_imaging": {"launches": na, "avg_us": 1e3 * msa / max(na, 1),
                            "bytes_per_point": 32 if vd else 28,
                            "share": msa / (msf + msa + mso)},
    }
    for k in kern.values():
        k["gpts"] = pts / (k["avg_us"] * 1e-6) / 1e9
        k["GBps"] = k["gpts"] * k["bytes_per_point"]
        k["hbm_frac"] = k["GBps"] / HBM_PEAK_GBS
    dom_name = max(kern, key=lambda n: kern[n]["share"])
    dom = kern[dom_name]
    lib_kernel = {"fd_step": "k_forward", "adjoint_imaging": "k_adjoint"}[dom_name]
    traffic = committed_traffic(lib_kernel, "variable" if vd else "constant")
    out = {
        "metric": "Gpt/s & %HBM peak (fwd/adjoint 8th-order stencil); FWI misfit cut per GPU-s",
        "value": round(value, 3),
        "unit": "Gpt/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"one-shot forward + adjoint gradient pass, "
                               f"{'variable' if vd else 'constant'} density, "
                               f"{w.nx}x{w.ny}x{w.nz} model + {w.border}-cell sponge, "
                               f"{w.nt} steps, {nrec} receivers",
                   "padded_points": pts, "nt": w.nt, "nrec": nrec,
                   "checkpoint": f"binomial, {ckpt[1]} stored pairs",
                   "tuning": dict(zip(("fwd_variant", "fwd_rounds", "adj_variant",
                                       "adj_rounds"), P.tuning())),
                   "parallelism": "1 GPU, one shot"},
        "roofline": {"bound": "hbm", "achieved": round(dom["GBps"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom["hbm_frac"], 4),
                     "traffic": traffic, "kernel": dom_name,
                     "algorithmic_bytes_per_launch": dom["bytes_per_point"] * pts,
                     # both step kernels: the pass runs them for about equal times
                     "frac_per_kernel": {n: round(d["hbm_frac"], 4) for n, d in kern.items()},
                     "frac_min": round(min(d["hbm_frac"] for d in kern.values()), 4)},
        "kernels": {n: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
                    for n, d in kern.items()},
        "other_ms_per_step": round(mso / args.steps, 3),
        "model_point_gpts": round(w.nx * w.ny * w.nz * 2.0 * w.nt / (ms_step * 1e-3) / 1e9, 3),
        "misfit": float(misfit.item()) / (args.warmup + args.steps),
        "kernel_source": kernel_hash(),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
