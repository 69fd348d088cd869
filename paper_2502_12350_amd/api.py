"""Python face of the C ABI: torch supplies device memory and the stream.

Every numerical step runs in the HIP library; this module only checks
dtypes / shapes / devices, allocates buffers through torch and passes raw
pointers.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import check, wfd_ckpt, wfd_grid


@dataclass
class GridSpec:
    """Model grid, sponge and time axis (mirrors wfd_grid)."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    ox: float = 0.0
    oy: float = 0.0
    oz: float = 0.0
    border: int = 0
    dt: float = 1.0e-3
    nt: int = 1
    free_surface: bool = False
    cpml: bool = False          # CPML layer in the border cells instead of the sponge
    fpeak: float = 0.0          # CPML: source peak frequency (Hz), alpha_max = pi fpeak
    cpml_vmax: float = 0.0      # CPML: velocity of d0 (m/s); 0 = the model's maximum

    def c(self) -> wfd_grid:
        return wfd_grid(int(self.nx), int(self.ny), int(self.nz), float(self.dx), float(self.dy),
                        float(self.dz), float(self.ox), float(self.oy), float(self.oz),
                        int(self.border), float(self.dt), int(self.nt), int(bool(self.free_surface)),
                        int(bool(self.cpml)), float(self.fpeak), float(self.cpml_vmax))

    @property
    def padded_shape(self) -> Tuple[int, int, int]:
        b = 2 * self.border
        return (self.nz + b, self.ny + b, self.nx + b)


def _grid(g) -> GridSpec:
    if isinstance(g, GridSpec):
        return g
    if isinstance(g, dict):
        return GridSpec(**g)
    return GridSpec(**{k: getattr(g, k) for k in GridSpec.__dataclass_fields__ if hasattr(g, k)})


def _xyz(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _ckpt(ckpt) -> wfd_ckpt:
    """'full' | ('revolve', n_snapshots) | ('revolve', 0, mem_fraction) |
    ('host', pinned_cpu_tensor) | wfd_ckpt ('host' alone is resolved by the
    Propagator, which then keeps a pinned store of its own)."""
    if isinstance(ckpt, wfd_ckpt):
        return ckpt
    if isinstance(ckpt, tuple) and ckpt[0] == "host":
        store = ckpt[1]
        if getattr(store, "is_cuda", True) or not store.is_contiguous():
            raise ValueError("the host store must be a contiguous CPU tensor (pin_memory=True)")
        return wfd_ckpt(_lib.CKPT_HOST, 0, 0.8, store.data_ptr(),
                        store.numel() * store.element_size())
    if ckpt == "host":
        return wfd_ckpt(_lib.CKPT_HOST, 0, 0.8, None, 0)
    if ckpt in (None, "full"):
        return wfd_ckpt(_lib.CKPT_FULL, 0, 0.8)
    if isinstance(ckpt, tuple) and ckpt[0] == "revolve":
        n = int(ckpt[1]) if len(ckpt) > 1 else 0
        frac = float(ckpt[2]) if len(ckpt) > 2 else 0.8
        return wfd_ckpt(_lib.CKPT_REVOLVE, n, frac)
    raise ValueError(f"bad checkpoint policy {ckpt!r}")


# ---------------------------------------------------------------------------
# host-only helpers (no GPU needed)
# ---------------------------------------------------------------------------
def map_position(grid, xyz) -> Tuple[int, int, int]:
    """Padded-grid node (ix, iy, iz) of a position in metres."""
    g = _grid(grid).c()
    p = _xyz(xyz)[0]
    out = (C.c_int32 * 3)()
    check(_lib.lib().wfd_map_position(C.byref(g), _dptr(p), out))
    return (out[0], out[1], out[2])


def cfl_ratio(grid, vmax: float, m2max: float = 0.0) -> float:
    g = _grid(grid).c()
    r = C.c_double()
    check(_lib.lib().wfd_cfl_ratio(C.byref(g), float(vmax), float(m2max), C.byref(r)))
    return r.value


def checkpoint_plan(nt: int, n_snapshots: int):
    """(actions [n][3] int32, forward step count) of the library's schedule."""
    L = _lib.lib()
    na, ns = C.c_int64(), C.c_int64()
    check(L.wfd_checkpoint_plan(int(nt), int(n_snapshots), None, 0, C.byref(na), C.byref(ns)))
    buf = np.zeros((na.value, 3), dtype=np.int32)
    check(L.wfd_checkpoint_plan(int(nt), int(n_snapshots),
                                buf.ctypes.data_as(C.POINTER(C.c_int32)), na.value,
                                C.byref(na), C.byref(ns)))
    return buf, ns.value


def smooth(x, mode: str, lengths, spacing, *, tol: float = 1e-6, max_iter: int = 500, out=None):
    """The paper's gradient smoothing (GradientPreconditioning) of a device
    volume x [nz][ny][nx] FP32: mode "laplace" or "bessel", lengths and
    spacing (x, y, z) in metres.  Returns (smoothed volume, CG iterations)."""
    import torch
    L = _lib.lib()
    m = {"laplace": _lib.SMOOTH_LAPLACE, "bessel": _lib.SMOOTH_BESSEL}[mode]
    if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 3):
        raise ValueError("x must be a contiguous 3-D float32 CUDA tensor")
    nz, ny, nx = x.shape
    if out is None:
        out = torch.empty_like(x)
    nb = C.c_size_t()
    check(L.wfd_smooth_workspace_bytes(m, nx, ny, nz, C.byref(nb)))
    work = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
    lens = np.ascontiguousarray(lengths, dtype=np.float64)
    hs = np.ascontiguousarray(spacing, dtype=np.float64)
    it = C.c_int32()
    check(L.wfd_smooth(m, _ptr(x), _ptr(out), nx, ny, nz, _dptr(lens), _dptr(hs), float(tol),
                       int(max_iter), _ptr(work), nb.value, C.byref(it),
                       C.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)))
    return out, it.value


def resample(traces, dt_in: float, nt_out: int, dt_out: float, mode: str = "sinc"):
    """Resample device traces [nrec][nt] (sample k at (k + 1) dt) to nt_out
    samples of step dt_out by "nearest" or "sinc" interpolation."""
    import torch
    L = _lib.lib()
    m = {"nearest": _lib.RESAMPLE_NEAREST, "sinc": _lib.RESAMPLE_SINC}[mode]
    if not (traces.is_cuda and traces.dtype == torch.float32 and traces.is_contiguous()
            and traces.dim() == 2):
        raise ValueError("traces must be a contiguous 2-D float32 CUDA tensor")
    nrec, nt_in = traces.shape
    out = torch.empty((nrec, int(nt_out)), dtype=torch.float32, device=traces.device)
    check(L.wfd_resample(m, _ptr(traces), nrec, nt_in, float(dt_in), _ptr(out), int(nt_out),
                         float(dt_out),
                         C.c_void_p(torch.cuda.current_stream(traces.device).cuda_stream)))
    return out


def model_bytes(grid, variable_density: bool) -> int:
    g = _grid(grid).c()
    n = C.c_size_t()
    check(_lib.lib().wfd_model_bytes(C.byref(g), int(bool(variable_density)), C.byref(n)))
    return n.value


# ---------------------------------------------------------------------------
# device API
# ---------------------------------------------------------------------------
class Propagator:
    """One context on one GPU; all work goes to torch's current stream."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.L = _lib.lib()
        self._ctx = C.c_void_p()
        check(self.L.wfd_create(C.byref(self._ctx), int(device), self._stream()))
        self.grid: Optional[GridSpec] = None
        self._model = None
        self._work = None
        self._host = None

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_stream(self):
        check(self.L.wfd_set_stream(self._ctx, self._stream()))

    def close(self):
        if self._ctx:
            check(self.L.wfd_destroy(self._ctx))
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, t, name, shape=None, dtype=None):
        torch = self.torch
        if t is None:
            raise ValueError(f"{name} is required")
        if not (t.is_cuda and t.device == self.device):
            raise ValueError(f"{name} must live on {self.device}")
        if dtype is not None and t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _buffer(self, nbytes: int):
        torch = self.torch
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        return buf, buf.data_ptr() + off

    def set_model(self, grid, vel, rho=None):
        """Precompute coefficients and check stability (waits on the stream once)."""
        torch = self.torch
        g = _grid(grid)
        shape = (g.nz, g.ny, g.nx)
        vel = self._dev(vel, "vel", shape, torch.float32)
        if rho is not None:
            rho = self._dev(rho, "rho", shape, torch.float32)
        nbytes = model_bytes(g, rho is not None)
        buf, ptr = self._buffer(nbytes)
        self._sync_stream()
        gc = g.c()
        check(self.L.wfd_set_model(self._ctx, C.byref(gc), _ptr(vel), _ptr(rho), ptr, nbytes))
        self.grid = g
        self._model = buf
        return self

    def workspace_bytes(self, nrec: int, ckpt=None) -> int:
        n = C.c_size_t()
        ck = None if ckpt is None else _ckpt(ckpt)
        check(self.L.wfd_workspace_bytes(self._ctx, int(nrec), None if ck is None else C.byref(ck),
                                         C.byref(n)))
        return n.value

    def _workspace(self, nbytes: int):
        if self._work is None or self._work[2] < nbytes:
            self._work = None
            buf, ptr = self._buffer(nbytes)
            self._work = (buf, ptr, nbytes)
        return self._work[1], self._work[2]

    def release_workspace(self):
        self._work = None
        self._host = None

    def host_store_bytes(self) -> int:
        """Bytes of the pinned host store of the 'host' checkpoint mode."""
        n = C.c_size_t()
        check(self.L.wfd_host_store_bytes(self._ctx, C.byref(n)))
        return n.value

    def _host_store(self):
        """A pinned host store of this model's size, kept between calls."""
        nbytes = self.host_store_bytes()
        if getattr(self, "_host", None) is None or self._host.numel() * 4 < nbytes:
            self._host = None
            self._host = self.torch.empty((nbytes + 3) // 4, dtype=self.torch.float32,
                                          pin_memory=True)
        return self._host

    def forward(self, wavelet, src_xyz, rec_xyz, *, final: bool = False, seis=None):
        """Seismograms [nrec][nt] (and, if final, [2][Nz][Ny][Nx] = w^nt, w^(nt-1))."""
        torch = self.torch
        g = self.grid
        if g is None:
            raise RuntimeError("set_model first")
        wavelet = self._dev(wavelet, "wavelet", (g.nt,), torch.float32)
        src = _xyz(src_xyz)
        rec = _xyz(rec_xyz) if rec_xyz is not None and len(rec_xyz) else np.zeros((0, 3))
        nrec = rec.shape[0]
        if seis is None:
            seis = torch.empty((nrec, g.nt), dtype=torch.float32, device=self.device)
        else:
            self._dev(seis, "seis", (nrec, g.nt), torch.float32)
        fin = (torch.empty((2,) + g.padded_shape, dtype=torch.float32, device=self.device)
               if final else None)
        wptr, wbytes = self._workspace(self.workspace_bytes(nrec))
        self._sync_stream()
        check(self.L.wfd_forward(self._ctx, _ptr(wavelet), _dptr(src), nrec,
                                 _dptr(rec) if nrec else None, _ptr(seis) if nrec else None,
                                 _ptr(fin), wptr, wbytes))
        return (seis, fin) if final else seis

    def forward_misfit(self, wavelet, src_xyz, rec_xyz, dobs, *, misfit=None, seis: bool = False):
        """Accumulate one shot's misfit from a forward sweep only; returns misfit[, seis]."""
        torch = self.torch
        g = self.grid
        if g is None:
            raise RuntimeError("set_model first")
        wavelet = self._dev(wavelet, "wavelet", (g.nt,), torch.float32)
        src = _xyz(src_xyz)
        rec = _xyz(rec_xyz)
        nrec = rec.shape[0]
        dobs = self._dev(dobs, "dobs", (nrec, g.nt), torch.float32)
        if misfit is None:
            misfit = torch.zeros((), dtype=torch.float64, device=self.device)
        else:
            self._dev(misfit, "misfit", (), torch.float64)
        out_seis = (torch.empty((nrec, g.nt), dtype=torch.float32, device=self.device)
                    if seis else None)
        n = C.c_size_t()
        check(self.L.wfd_misfit_workspace_bytes(self._ctx, nrec, C.byref(n)))
        wptr, wbytes = self._workspace(n.value)
        self._sync_stream()
        check(self.L.wfd_forward_misfit(self._ctx, _ptr(wavelet), _dptr(src), nrec, _dptr(rec),
                                        _ptr(dobs), _ptr(out_seis), _ptr(misfit), wptr, wbytes))
        return (misfit, out_seis) if seis else misfit

    def gradient(self, wavelet, src_xyz, rec_xyz, dobs, *, ckpt="full", grad=None, misfit=None,
                 illum=None, seis: bool = False, wavelet_grad=None, out_exp2: int = 0,
                 field_exp2=None):
        """Accumulate one shot's misfit and dJ/dv; returns (misfit, grad[, seis]).

        wavelet_grad: optional [nt] float32 device tensor, += dJ/df (the
        gradient with respect to the wavelet samples); out_exp2: grad, illum
        and wavelet_grad accumulate 2^out_exp2 times their value; field_exp2:
        optional int32 device scalar that receives the call's field exponent."""
        torch = self.torch
        g = self.grid
        if g is None:
            raise RuntimeError("set_model first")
        wavelet = self._dev(wavelet, "wavelet", (g.nt,), torch.float32)
        src = _xyz(src_xyz)
        rec = _xyz(rec_xyz)
        nrec = rec.shape[0]
        dobs = self._dev(dobs, "dobs", (nrec, g.nt), torch.float32)
        if grad is None:
            grad = torch.zeros((g.nz, g.ny, g.nx), dtype=torch.float32, device=self.device)
        else:
            self._dev(grad, "grad", (g.nz, g.ny, g.nx), torch.float32)
        if misfit is None:
            misfit = torch.zeros((), dtype=torch.float64, device=self.device)
        else:
            self._dev(misfit, "misfit", (), torch.float64)
        if illum is not None:
            self._dev(illum, "illum", (g.nz, g.ny, g.nx), torch.float32)
        out_seis = (torch.empty((nrec, g.nt), dtype=torch.float32, device=self.device)
                    if seis else None)
        if wavelet_grad is not None:
            self._dev(wavelet_grad, "wavelet_grad", (g.nt,), torch.float32)
        if field_exp2 is not None:
            self._dev(field_exp2, "field_exp2", (), torch.int32)
        opts = _lib.wfd_gradient_opts(_ptr(wavelet_grad), int(out_exp2), _ptr(field_exp2))
        ck = _ckpt(("host", self._host_store()) if isinstance(ckpt, str) and ckpt == "host"
                   else ckpt)
        wptr, wbytes = self._workspace(self.workspace_bytes(nrec, ck))
        self._sync_stream()
        check(self.L.wfd_gradient_ex(self._ctx, _ptr(wavelet), _dptr(src), nrec, _dptr(rec),
                                     _ptr(dobs), C.byref(ck), _ptr(out_seis), _ptr(misfit),
                                     _ptr(grad), _ptr(illum), C.byref(opts), wptr, wbytes))
        return (misfit, grad, out_seis) if seis else (misfit, grad)

    def gradient_finish(self, grad, zero_top_planes: int):
        torch = self.torch
        g = self.grid
        self._dev(grad, "grad", (g.nz, g.ny, g.nx), torch.float32)
        self._sync_stream()
        check(self.L.wfd_gradient_finish(self._ctx, _ptr(grad), int(zero_top_planes)))
        return grad

    # launch tuning -----------------------------------------------------------
    def set_tuning(self, fwd_variant: int = 0, fwd_rounds: int = 0, adj_variant: int = 0,
                   adj_rounds: int = 0):
        """Tile shapes of the step kernels and their z-chunk rounds (wfd_tuning)."""
        t = _lib.wfd_tuning(int(fwd_variant), int(fwd_rounds), int(adj_variant), int(adj_rounds))
        check(self.L.wfd_set_tuning(self._ctx, C.byref(t)))

    def tuning(self) -> Tuple[int, int, int, int]:
        """(fwd_variant, fwd_rounds, adj_variant, adj_rounds)."""
        t = _lib.wfd_tuning()
        check(self.L.wfd_get_tuning(self._ctx, C.byref(t)))
        return t.fwd_variant, t.fwd_rounds, t.adj_variant, t.adj_rounds

    def autotune(self, steps: int = 20):
        """Time every launch shape on the current model and keep the fastest;
        returns (tuning tuple, forward us/step, adjoint us/step)."""
        if self.grid is None:
            raise RuntimeError("set_model first")
        wptr, wbytes = self._workspace(self.workspace_bytes(0, ("revolve", 1)))
        self._sync_stream()
        t = _lib.wfd_tuning()
        us = (C.c_double * 2)()
        check(self.L.wfd_autotune(self._ctx, int(steps), wptr, wbytes, C.byref(t), us))
        return (t.fwd_variant, t.fwd_rounds, t.adj_variant, t.adj_rounds), us[0], us[1]

    # measurement -------------------------------------------------------------
    def set_profiling(self, on: bool):
        check(self.L.wfd_set_profiling(self._ctx, int(bool(on))))

    def kernel_stats(self, kernel_class: int) -> Tuple[int, float]:
        n, ms = C.c_int64(), C.c_double()
        check(self.L.wfd_kernel_stats(self._ctx, int(kernel_class), C.byref(n), C.byref(ms)))
        return n.value, ms.value


class ShotBatch:
    """Forward sweeps of several shots advanced together (one launch per step
    over all shots' tiles), optionally replayed as one HIP graph.

    Each shot has its own Propagator (its own model, typically the window
    around its source) on one device; all of them launch on `stream` (torch's
    current stream if None; graph replay needs a non-default stream).
    """

    def __init__(self, props: Sequence[Propagator], wavelet, src_xyz, rec_xyz, stream=None):
        if not props:
            raise ValueError("no shots")
        torch = props[0].torch
        p0 = props[0]
        self.torch = torch
        self.props = list(props)
        # the batch's step descriptors point into each context's model buffer:
        # hold those buffers for the batch's lifetime (a later set_model on a
        # member makes wfd_batch_run fail with WFD_E_STATE instead)
        self._models = [p._model for p in self.props]
        self.stream = stream if stream is not None else torch.cuda.current_stream(p0.device)
        nt = p0.grid.nt if p0.grid is not None else 0
        self.wavelet = p0._dev(wavelet, "wavelet", (nt,), torch.float32)
        n = len(self.props)
        if len(src_xyz) != n or len(rec_xyz) != n:
            raise ValueError("one source and one receiver array per shot")
        self._src = np.ascontiguousarray(np.concatenate([_xyz(s) for s in src_xyz]),
                                         dtype=np.float64)
        self._rec = [_xyz(r) if r is not None and len(r) else np.zeros((0, 3)) for r in rec_xyz]
        nrec = [r.shape[0] for r in self._rec]
        self.seis = [torch.empty((k, nt), dtype=torch.float32, device=p0.device) for k in nrec]
        self._work = []
        ctxs = (C.c_void_p * n)()
        works = (C.c_void_p * n)()
        wbytes = (C.c_size_t * n)()
        seisp = (C.c_void_p * n)()
        recp = (_lib._D3 * n)()
        for i, p in enumerate(self.props):
            if p.grid is None:
                raise RuntimeError(f"shot {i}: set_model first")
            check(p.L.wfd_set_stream(p._ctx, C.c_void_p(self.stream.cuda_stream)))
            nb = p.workspace_bytes(nrec[i])
            buf, ptr = p._buffer(nb)
            self._work.append(buf)
            ctxs[i], works[i], wbytes[i] = p._ctx.value, ptr, nb
            seisp[i] = _ptr(self.seis[i]) if nrec[i] else None
            if nrec[i]:
                recp[i] = _dptr(self._rec[i])
        nr = (C.c_int32 * n)(*nrec)
        self._b = C.c_void_p()
        check(p0.L.wfd_batch_create(C.byref(self._b), n, ctxs, _ptr(self.wavelet),
                                    _dptr(self._src), nr, recp, seisp, works, wbytes))
        self.L = p0.L

    def run(self, use_graph: bool = False):
        """Enqueue all shots on the batch stream; returns the per-shot traces."""
        check(self.L.wfd_batch_run(self._b, int(bool(use_graph))))
        return self.seis

    def close(self):
        if getattr(self, "_b", None):
            check(self.L.wfd_batch_destroy(self._b))
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GradientBatch:
    """Misfits and velocity gradients of several shots computed together: every
    forward and adjoint step of the shared binomial checkpointing schedule is
    one launch over all shots' tiles, optionally replayed as one HIP graph.

    Each shot has its own Propagator (its own model, typically the window
    around its source) on one device; the results equal each Propagator's
    gradient(..., ckpt=("revolve", n_snapshots)) bitwise.  run() adds every
    shot's misfit and gradient (and illumination) into the tensors it returns.
    """

    def __init__(self, props: Sequence[Propagator], wavelet, src_xyz, rec_xyz, dobs,
                 n_snapshots: int, illum: bool = False, stream=None):
        if not props:
            raise ValueError("no shots")
        torch = props[0].torch
        p0 = props[0]
        self.torch = torch
        self.props = list(props)
        self._models = [p._model for p in self.props]
        self.stream = stream if stream is not None else torch.cuda.current_stream(p0.device)
        nt = p0.grid.nt if p0.grid is not None else 0
        self.wavelet = p0._dev(wavelet, "wavelet", (nt,), torch.float32)
        n = len(self.props)
        if len(src_xyz) != n or len(rec_xyz) != n or len(dobs) != n:
            raise ValueError("one source, receiver array and data array per shot")
        self._src = np.ascontiguousarray(np.concatenate([_xyz(s) for s in src_xyz]),
                                         dtype=np.float64)
        self._rec = [_xyz(r) if r is not None and len(r) else np.zeros((0, 3)) for r in rec_xyz]
        nrec = [r.shape[0] for r in self._rec]
        self.dobs = [p._dev(d, "dobs", (k, nt), torch.float32) if k else None
                     for p, d, k in zip(self.props, dobs, nrec)]
        self.misfit = torch.zeros(n, dtype=torch.float64, device=p0.device)
        self.grad = [torch.zeros((p.grid.nz, p.grid.ny, p.grid.nx), dtype=torch.float32,
                                 device=p0.device) for p in self.props]
        self.illum = ([torch.zeros_like(g) for g in self.grad] if illum else None)
        self._work = []
        ctxs = (C.c_void_p * n)()
        works = (C.c_void_p * n)()
        wbytes = (C.c_size_t * n)()
        dob = (C.c_void_p * n)()
        mis = (C.c_void_p * n)()
        grd = (C.c_void_p * n)()
        ill = (C.c_void_p * n)()
        recp = (_lib._D3 * n)()
        for i, p in enumerate(self.props):
            if p.grid is None:
                raise RuntimeError(f"shot {i}: set_model first")
            check(p.L.wfd_set_stream(p._ctx, C.c_void_p(self.stream.cuda_stream)))
            nb = p.workspace_bytes(nrec[i], ("revolve", int(n_snapshots)))
            buf, ptr = p._buffer(nb)
            self._work.append(buf)
            ctxs[i], works[i], wbytes[i] = p._ctx.value, ptr, nb
            dob[i] = _ptr(self.dobs[i])
            mis[i] = self.misfit.data_ptr() + 8 * i
            grd[i] = _ptr(self.grad[i])
            ill[i] = _ptr(self.illum[i]) if illum else None
            if nrec[i]:
                recp[i] = _dptr(self._rec[i])
        nr = (C.c_int32 * n)(*nrec)
        self._b = C.c_void_p()
        check(p0.L.wfd_gbatch_create(C.byref(self._b), n, ctxs, _ptr(self.wavelet),
                                     _dptr(self._src), nr, recp, dob, int(n_snapshots), mis, grd,
                                     ill if illum else None, works, wbytes))
        self.L = p0.L

    def run(self, use_graph: bool = False):
        """Enqueue every shot's gradient on the batch stream (accumulating into
        self.misfit [nshot], self.grad and self.illum); returns (misfit, grad)."""
        check(self.L.wfd_gbatch_run(self._b, int(bool(use_graph))))
        return self.misfit, self.grad

    def close(self):
        if getattr(self, "_b", None):
            check(self.L.wfd_gbatch_destroy(self._b))
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
