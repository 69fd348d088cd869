"""Host-side logic of the C ABI, runnable without a GPU.

* the library loads and exports every function that include/wfd.h declares;
* position mapping and the stability ratio agree with the oracle;
* the checkpoint schedule is valid and reaches the closed-form optimum.
"""

import os
import re

import numpy as np
import pytest

import oracle
from paper_2502_12350_amd import _lib
from paper_2502_12350_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "wfd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wfd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = _header_functions()
    assert len(names) >= 15
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), f"{n} declared in wfd.h but not exported"
    assert sorted(_lib.exported_symbols()) == names


def test_error_paths_report_status_and_message():
    with pytest.raises(_lib.WfdError) as e:
        api.model_bytes(api.GridSpec(0, 4, 4, 10, 10, 10), False)
    assert e.value.name == "WFD_E_ARG" and "model size" in str(e.value)
    with pytest.raises(_lib.WfdError) as e:
        api.model_bytes(api.GridSpec(4, 4, 4, 10, 10, 10, border=-1), False)
    assert e.value.name == "WFD_E_ARG"
    with pytest.raises(_lib.WfdError) as e:
        api.checkpoint_plan(10, 0)
    assert e.value.name == "WFD_E_ARG"
    with pytest.raises(_lib.WfdError) as e:
        api.map_position(api.GridSpec(4, 4, 4, 10, 10, 10), [45.0, 0.0, 0.0])
    assert e.value.name == "WFD_E_RANGE"
    with pytest.raises(_lib.WfdError) as e:
        api.model_bytes(api.GridSpec(4, 4, 4, 10, 10, 10, dt=0.0), False)
    assert e.value.name == "WFD_E_ARG"


def test_pitched_plane_limit():
    # the step kernels address a pitched x-y plane (x rounded up to 64) with
    # 32-bit byte offsets: below 2^30 points it is accepted, at or above refused
    api.model_bytes(api.GridSpec(16384, 65535, 1, 10, 10, 10, border=0), False)
    with pytest.raises(_lib.WfdError) as e:  # 16385 x 65300 < 2^30, pitched 16448 x 65300 is not
        api.model_bytes(api.GridSpec(16385, 65300, 1, 10, 10, 10, border=0), False)
    assert e.value.name == "WFD_E_ARG" and "too large" in str(e.value)


def test_model_bytes_scales_with_density_option():
    g = api.GridSpec(30, 20, 10, 10, 10, 10, border=4)
    cd = api.model_bytes(g, False)
    vd = api.model_bytes(g, True)
    Nz, Ny, Nx = g.padded_shape
    vol = 64 * Ny * Nz * 4
    assert cd >= vol and vd >= 2 * vol + 30 * 20 * 10 * 4


def test_map_position_matches_oracle():
    rng = np.random.default_rng(1)
    g = api.GridSpec(37, 23, 19, 7.5, 10.0, 4.0, ox=-30.0, oy=100.0, oz=5.0, border=6)
    og = oracle.Grid(**{k: v for k, v in g.__dict__.items() if k in oracle.Grid.__dataclass_fields__})
    for _ in range(400):
        xyz = [rng.uniform(-40, 250), rng.uniform(90, 330), rng.uniform(0, 85)]
        # also exact half-way points
        if rng.random() < 0.3:
            xyz[0] = -30.0 + 7.5 * (rng.integers(0, 37) + 0.5)
        try:
            iz, iy, ix = oracle.node_index(og, xyz)
            ok = True
        except ValueError:
            ok = False
        if ok:
            assert api.map_position(g, xyz) == (ix, iy, iz)
        else:
            with pytest.raises(_lib.WfdError):
                api.map_position(g, xyz)


def test_cfl_ratio_matches_oracle():
    for h, dt, v, m2 in [((10, 10, 10), 1e-3, 2000, 0.0), ((5, 7, 9), 4e-4, 4500, 1e-3),
                         ((10, 10, 10), 8.889e-4, 4500, -2e-3)]:
        g = api.GridSpec(8, 8, 8, *h, dt=dt)
        og = oracle.Grid(8, 8, 8, *h, dt=dt)
        assert abs(api.cfl_ratio(g, v, m2) - oracle.cfl_ratio(og, v, m2)) <= 1e-14


def _simulate(actions, nt, S):
    cur = 0
    slots = {}
    visits = []
    steps = 0
    first_visit_seen = False
    chain_end = 0
    for op, a, b in actions:
        stored = set(slots.values()) | {0}
        if op == 0:
            assert a == cur or a in stored, (op, a, b)
            assert b > a
            steps += b - a
            if not first_visit_seen:
                assert a == chain_end, "first sweep must be one contiguous chain"
                chain_end = b
            cur = b
        elif op == 1:
            assert a == cur and 0 <= b < S and b not in slots
            slots[b] = a
        elif op == 2:
            assert a == cur or a in stored or a + 1 == cur
            if not first_visit_seen:
                assert chain_end == nt, "all data must be recorded before the first visit"
            first_visit_seen = True
            visits.append(a)
        elif op == 3:
            assert slots.get(b) == a
            del slots[b]
        else:
            raise AssertionError(op)
    assert visits == list(range(nt, 0, -1))
    return steps


@pytest.mark.parametrize("nt,S", [(1, 1), (2, 1), (7, 1), (10, 3), (50, 4), (200, 6),
                                  (300, 299), (64, 64), (1200, 20), (2000, 130)])
def test_checkpoint_plan_valid_and_optimal(nt, S):
    actions, nsteps = api.checkpoint_plan(nt, S)
    steps = _simulate(actions, nt, S)
    assert steps == nsteps
    # x_0 needs no slot, so S stored pairs reverse nt+1 states with S+1 snapshots
    assert nsteps == oracle.forward_steps_closed_form(nt + 1, S + 1)


def test_checkpoint_plan_counts_for_the_gradient_workload():
    # 1200 steps with 20 stored pairs: 3327 forward steps instead of 1200
    _, n = api.checkpoint_plan(1200, 20)
    assert n == 3327
    _, n_full = api.checkpoint_plan(1200, 1200)
    assert n_full == 1200


def test_cnn_packed_sizes_and_workspace():
    import ctypes as C
    from paper_2502_12350_amd import _lib
    L = _lib.lib()
    n = C.c_int64()
    for (ci, co, flip), k in {(2, 16, 0): 64, (16, 16, 0): 448, (16, 1, 0): 448,
                              (16, 1, 1): 32, (2, 16, 1): 448, (16, 16, 1): 448}.items():
        assert L.wfd_cnn_packed_elems(ci, co, flip, C.byref(n)) == 0
        assert n.value == 16 * k
    assert L.wfd_cnn_packed_elems(3, 16, 0, C.byref(n)) == -1       # no such layer
    assert L.wfd_cnn_packed_elems(16, 16, 2, C.byref(n)) == -1
    b = C.c_size_t()
    # one partial row of 27 * 256 + 16 floats per wavefront (4 per block, one
    # block per 64 x 4 x 16 tile, at most 512 blocks), then one row per
    # segment of 32 rows
    row = (27 * 256 + 16) * 4
    assert L.wfd_cnn_wgrad_workspace_bytes(70, 7, 5, C.byref(b)) == 0
    tiles = 2 * 2 * 1
    assert b.value == (4 * tiles + 1) * row
    assert L.wfd_cnn_wgrad_workspace_bytes(128, 128, 128, C.byref(b)) == 0
    assert b.value == (4 * 512 + 64) * row                            # 2 x 32 x 8 tiles
    assert L.wfd_cnn_wgrad_workspace_bytes(256, 256, 256, C.byref(b)) == 0
    assert b.value == (4 * 512 + 64) * row                            # capped at 512 blocks
    assert L.wfd_cnn_conv(None, 8, 8, 8, 3, 16, None, None, 0, None, None, 0, None, None,
                          None) == -1
    # argument checks that fail before any device work (pointers never dereferenced)
    big = 1 << 30
    assert L.wfd_cnn_wgrad(256, 256, 2 ** 30, 2 ** 30, 2 ** 30, 16, 16, 256, 256, 256, big,
                           None) == -1                                    # too many tiles
    assert L.wfd_cnn_wgrad(256, 258, 8, 8, 8, 16, 16, 256, 256, 256, big, None) == -1  # dz
    assert L.wfd_cnn_wgrad(258, 256, 8, 8, 8, 16, 16, 256, 256, 256, big, None) == -1  # in
    assert L.wfd_cnn_wgrad(256, 256, 8, 8, 8, 16, 16, 256, 256, 256, 16, None) == -4   # work
    assert L.wfd_cnn_conv(256, 8, 8, 8, 16, 16, 256, None, 0, 260, None, 0, 256, None,
                          None) == -1                                     # mask alignment
    # 32-bit plane offsets: an x-y plane holds at most 2^24 voxels
    assert L.wfd_cnn_conv(256, 4097, 4096, 1, 16, 16, 256, None, 0, None, None, 0, 256, None,
                          None) == -1
    assert L.wfd_cnn_conv(256, 8, 8, 8, 16, 1, 256, None, 0, None, 256, 17, 256, None,
                          None) == -1                                     # residual channels
    assert L.wfd_cnn_wgrad(256, 256, 4097, 4096, 1, 16, 16, 256, 256, 256, big,
                           None) == -1                                    # plane > 2^24


def test_smoothing_and_resampling_host_paths():
    import ctypes as C
    from paper_2502_12350_amd import _lib
    L = _lib.lib()
    b = C.c_size_t()
    assert L.wfd_smooth_workspace_bytes(_lib.SMOOTH_LAPLACE, 10, 20, 30, C.byref(b)) == 0
    assert b.value >= 2 * (10 + 20 + 30) * 8
    assert L.wfd_smooth_workspace_bytes(_lib.SMOOTH_BESSEL, 10, 20, 30, C.byref(b)) == 0
    assert b.value >= 3 * 10 * 20 * 30 * 4
    assert L.wfd_smooth_workspace_bytes(7, 10, 20, 30, C.byref(b)) == -1
    assert L.wfd_smooth_workspace_bytes(_lib.SMOOTH_BESSEL, 0, 20, 30, C.byref(b)) == -1
    # argument errors are found before anything touches a device
    assert L.wfd_resample(9, None, 1, 10, 1e-3, None, 10, 1e-3, None) == -1
    assert L.wfd_resample(_lib.RESAMPLE_SINC, None, 1, 10, 0.0, None, 10, 1e-3, None) == -1
    assert L.wfd_resample(_lib.RESAMPLE_SINC, None, 0, 10, 1e-3, None, 10, 1e-3, None) == 0
    lens = (C.c_double * 3)(10.0, 10.0, 10.0)
    hs = (C.c_double * 3)(10.0, 0.0, 10.0)
    assert L.wfd_smooth(_lib.SMOOTH_LAPLACE, 1, 2, 4, 4, 4, lens, hs, 1e-6, 10, 3, 64, None,
                        None) == -1                                       # zero spacing


def test_free_surface_flag_is_validated():
    import ctypes as C
    from paper_2502_12350_amd import _lib
    L = _lib.lib()
    g = _lib.wfd_grid(16, 16, 16, 10.0, 10.0, 10.0, 0.0, 0.0, 0.0, 4, 1e-3, 10, 2)
    n = C.c_size_t()
    assert L.wfd_model_bytes(C.byref(g), 0, C.byref(n)) == -1
    g.free_surface = 1
    assert L.wfd_model_bytes(C.byref(g), 0, C.byref(n)) == 0


def test_cpml_fields_are_validated_and_sized():
    import ctypes as C
    from paper_2502_12350_amd import _lib
    L = _lib.lib()
    g = _lib.wfd_grid(16, 16, 16, 10.0, 10.0, 10.0, 0.0, 0.0, 0.0, 4, 1e-3, 10, 0, 0, 0.0, 0.0)
    n0, n1 = C.c_size_t(), C.c_size_t()
    assert L.wfd_model_bytes(C.byref(g), 0, C.byref(n0)) == 0
    g.cpml = 2
    assert L.wfd_model_bytes(C.byref(g), 0, C.byref(n1)) == -1
    g.cpml = 1
    g.fpeak = -1.0
    assert L.wfd_model_bytes(C.byref(g), 0, C.byref(n1)) == -1
    assert "fpeak" in L.wfd_last_error().decode()
    g.fpeak = 12.0
    g.cpml_vmax = float("nan")
    assert L.wfd_model_bytes(C.byref(g), 0, C.byref(n1)) == -1
    g.cpml_vmax = 3000.0
    assert L.wfd_model_bytes(C.byref(g), 0, C.byref(n1)) == 0
    # six 1-D coefficient tables of 24 floats each, 256-byte aligned
    assert n1.value - n0.value == 6 * 256


def test_library_holds_no_measurement_probe():
    """The streaming probe is bench.py's measurement code (bench_probe.hip),
    not part of the library."""
    from paper_2502_12350_amd import _lib
    assert not hasattr(_lib.lib(), "wfd_stream_probe")


def test_bench_one_gpu_only_and_probe_argument_checks():
    """bench.py refuses more than one GPU before touching one, and the
    bench-side probe entry points reject bad arguments before any launch."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU only" in (r.stdout + r.stderr)
    sys.path.insert(0, root)
    import bench
    L = bench._probe_lib()
    assert L.bench_march_probe(4, 1, None, 576, 576, 576, 192, None) != 0   # no buffer
    assert L.bench_march_probe(4, 1, 256, 0, 576, 576, 192, None) != 0      # empty grid
    assert L.bench_stream_probe(4, 1, 1, None, 1024, 256, None) != 0        # no buffer
    assert L.bench_stream_probe(4, 1, 1, 256, 1023, 256, None) != 0         # n % 4 != 0

