"""Learned gradient preconditioner: a 4-layer 3-D CNN on the library's
BF16 matrix-core kernels (include/wfd.h, wfd_cnn_*).

The paper preconditions the FWI gradient with a fixed smoothing filter (its
GradientPreconditioning option).  Here a small network maps the plain
illumination-compensated gradient g / (I + eps max I) and the source
illumination I (each scaled by its maximum) to a model-update direction:

    conv 3x3x3  2 -> 16, ReLU;  16 -> 16, ReLU;  16 -> 16, ReLU;  16 -> 1,
    plus the first input channel (the network learns a correction of the
    scaled plain direction)

BF16 weights and activations, FP32 accumulation, FP32 master weights trained
with Adam on the mean squared error against the scaled true perturbation.
Every convolution, gradient, loss and optimizer step runs in the library's
kernels; this module holds the buffers (torch tensors) and sequences calls.
The plain illumination-compensated gradient g / (I + eps max I) stays the
fallback: `direction` returns it whenever the network's direction is not a
descent direction.
"""

from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import check

LAYERS: Tuple[Tuple[int, int], ...] = ((2, 16), (16, 16), (16, 16), (16, 1))

# Weights trained by `python -m paper_2502_12350_amd.precond` on solver pairs
# (the training record, with its command, is beside them).
TRAINED = __import__("os").environ.get("WFD_PRECOND_WEIGHTS") or __import__("os").path.join(
    __import__("os").path.dirname(__file__), "weights", "precond_c5.npz")


def _p(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Preconditioner:
    """Network parameters and training state on one GPU (torch's current stream)."""

    def __init__(self, device: int = 0, seed: int = 0, params=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.L = _lib.lib()
        rng = np.random.default_rng(seed)
        self.w: List = []
        self.b: List = []
        for li, (ci, co) in enumerate(LAYERS):
            if params is not None:
                w = np.asarray(params[f"w{li}"], dtype=np.float32).reshape(27, ci, co)
                b = np.asarray(params[f"b{li}"], dtype=np.float32).reshape(co)
            else:  # He-uniform
                lim = np.sqrt(6.0 / (27 * ci))
                w = rng.uniform(-lim, lim, size=(27, ci, co)).astype(np.float32)
                b = np.zeros(co, dtype=np.float32)
            self.w.append(torch.from_numpy(np.ascontiguousarray(w)).to(self.device))
            self.b.append(torch.from_numpy(b).to(self.device))
        self.packed = []
        for ci, co in LAYERS:
            n = [C.c_int64(), C.c_int64()]
            for f in (0, 1):
                check(self.L.wfd_cnn_packed_elems(ci, co, f, C.byref(n[f])))
            self.packed.append(tuple(torch.empty(int(n[f].value), dtype=torch.bfloat16,
                                                 device=self.device) for f in (0, 1)))
        self.dw = [torch.zeros_like(w) for w in self.w]
        self.db = [torch.zeros_like(b) for b in self.b]
        self.m = [torch.zeros_like(t) for t in self.w + self.b]
        self.v = [torch.zeros_like(t) for t in self.w + self.b]
        self.step_count = 0
        self._reduce = torch.empty(_lib.CNN_REDUCE_BYTES, dtype=torch.uint8, device=self.device)
        self._acts = None
        self.pack()

    # -- plumbing -----------------------------------------------------------------
    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def pack(self):
        """Re-pack the BF16 matrix-core weights from the FP32 master weights."""
        s = self._stream()
        for li, (ci, co) in enumerate(LAYERS):
            for f in (0, 1):
                check(self.L.wfd_cnn_pack_weights(_p(self.w[li]), ci, co, f,
                                                  _p(self.packed[li][f]), s))

    def conv(self, x, li: int, *, relu: bool, out_f32: bool = False, flip: bool = False,
             mask=None, bias: bool = True, residual=None):
        """One convolution of layer li (or its data gradient with flip=True)."""
        torch = self.torch
        nz, ny, nx = x.shape[:3]
        ci, co = LAYERS[li]
        if flip:
            ci, co = co, ci
        assert x.shape[3] == ci and x.dtype == torch.bfloat16 and x.is_contiguous()
        ob = None if out_f32 else torch.empty((nz, ny, nx, co), dtype=torch.bfloat16,
                                              device=self.device)
        of = torch.empty((nz, ny, nx, co), dtype=torch.float32, device=self.device) \
            if out_f32 else None
        check(self.L.wfd_cnn_conv(_p(x), nx, ny, nz, ci, co, _p(self.packed[li][int(flip)]),
                                  _p(self.b[li]) if (bias and not flip) else None, int(relu),
                                  _p(mask), _p(residual),
                                  0 if residual is None else residual.shape[-1],
                                  _p(ob), _p(of), self._stream()))
        return of if out_f32 else ob

    # -- network ------------------------------------------------------------------
    def pack_input(self, grad, illum, eps_illum: float = 1e-3):
        """[nz][ny][nx][2] BF16 network input from FP32 gradient and illumination:
        the illumination-compensated gradient and the illumination, each scaled."""
        torch = self.torch
        out = torch.empty(tuple(grad.shape) + (2,), dtype=torch.bfloat16, device=self.device)
        # contiguous copies (if any) are held until the call: a copy freed
        # before it could hand its memory to the next one
        g, il = grad.contiguous(), illum.contiguous()
        check(self.L.wfd_cnn_pack_input(_p(g), _p(il), grad.numel(), eps_illum, _p(out),
                                        _p(self._reduce), self._reduce.numel(), self._stream()))
        return out

    def forward(self, x, keep: bool = False):
        """Network output [nz][ny][nx] FP32 for a BF16 input [nz][ny][nx][2]."""
        acts = [x]
        for li in range(3):
            acts.append(self.conv(acts[-1], li, relu=True))
        y = self.conv(acts[-1], 3, relu=False, out_f32=True, residual=x)[..., 0]
        self._acts = acts if keep else None
        return y

    def backward(self, y, target):
        """Gradients of mean((y - target)^2) into self.dw / self.db; returns the
        loss (device FP64 scalar).  Needs forward(..., keep=True) first."""
        torch = self.torch
        acts = self._acts
        assert acts is not None, "forward(keep=True) first"
        nz, ny, nx = y.shape
        loss = torch.zeros((), dtype=torch.float64, device=self.device)
        dz = torch.empty((nz, ny, nx, 1), dtype=torch.bfloat16, device=self.device)
        tc = target.contiguous()
        check(self.L.wfd_cnn_mse(_p(y), _p(tc), y.numel(), _p(dz), _p(loss), _p(self._reduce),
                                 self._reduce.numel(), self._stream()))
        nb = C.c_size_t()
        check(self.L.wfd_cnn_wgrad_workspace_bytes(nx, ny, nz, C.byref(nb)))
        work = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        for li in range(3, -1, -1):
            ci, co = LAYERS[li]
            check(self.L.wfd_cnn_wgrad(_p(acts[li]), _p(dz), nx, ny, nz, ci, co, _p(self.dw[li]),
                                       _p(self.db[li]), _p(work), nb.value, self._stream()))
            if li > 0:  # gradient of the layer input, masked by its ReLU
                dz = self.conv(dz, li, relu=False, flip=True, mask=acts[li], bias=False)
        return loss

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        """One Adam step on all weights and biases, then re-pack."""
        self.step_count += 1
        s = self._stream()
        for p, g, m, v in zip(self.w + self.b, self.dw + self.db, self.m, self.v):
            check(self.L.wfd_cnn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, beta1, beta2,
                                      eps, self.step_count, s))
        self.pack()

    def train_step(self, x, target, lr: float = 1e-3):
        y = self.forward(x, keep=True)
        loss = self.backward(y, target)
        self.adam(lr)
        self._acts = None
        return loss

    # -- use in FWI ----------------------------------------------------------------
    def direction(self, grad, illum, eps_illum: float = 1e-3):
        """Descent direction for the gradient `grad` [nz][ny][nx]: the network
        output (it predicts the scaled model perturbation), or the
        illumination-compensated fallback when that does not descend.
        Returns (direction, used_net)."""
        torch = self.torch
        d = self.forward(self.pack_input(grad, illum, eps_illum))
        if float(torch.sum(d.double() * grad.double())) < 0.0:
            return d, True
        return -grad / (illum + eps_illum * illum.max()), False

    # -- persistence -----------------------------------------------------------------
    def state(self) -> dict:
        out = {}
        for li in range(len(LAYERS)):
            out[f"w{li}"] = self.w[li].cpu().numpy()
            out[f"b{li}"] = self.b[li].cpu().numpy()
        return out

    def save(self, path: str):
        np.savez(path, **self.state())

    @classmethod
    def load(cls, path: str = TRAINED, device: int = 0):
        with np.load(path, allow_pickle=False) as z:
            params = {k: z[k] for k in z.files}
        return cls(device, params=params)


# ---------------------------------------------------------------------------
# training on pairs generated by the solver
# ---------------------------------------------------------------------------
def solver_pair(prop, w, zero_top_planes: int = 10):
    """Gradient and illumination at w.vel (the start model) for data modelled
    on w.extra["v_true"], and the true perturbation: (grad, illum, dv) as FP32
    device volumes [nz][ny][nx]."""
    import torch
    from .api import GridSpec
    g = GridSpec(**w.grid_kwargs())
    dev = prop.device
    wav = torch.from_numpy(w.wavelet).to(dev)
    vt = torch.from_numpy(w.extra["v_true"]).to(dev)
    v0 = torch.from_numpy(w.vel).to(dev)
    prop.set_model(g, vt)
    dobs = [prop.forward(wav, s, w.receivers).clone() for s in w.sources]
    prop.set_model(g, v0)
    grad = torch.zeros_like(v0)
    illum = torch.zeros_like(v0)
    for s, d in zip(w.sources, dobs):
        prop.gradient(wav, s, w.receivers, d, ckpt="full", grad=grad, illum=illum)
    if zero_top_planes:
        prop.gradient_finish(grad, zero_top_planes)
    return grad, illum, vt - v0


def cosine(a, b) -> float:
    import torch
    a, b = a.double(), b.double()
    return float(torch.sum(a * b) / (torch.linalg.vector_norm(a) * torch.linalg.vector_norm(b)))


def fallback_direction(grad, illum, eps_illum: float = 1e-3):
    """The plain illumination-compensated descent direction -g / (I + eps max I)."""
    return -grad / (illum + eps_illum * illum.max())


def recipe_model(size: int, seed: int):
    """Training-recipe model of a given size: 128^3 (4 shots, 1000 steps) or
    the 256^3 evaluation geometry (8 shots, 1600 steps, 20-cell sponge)."""
    import seisgen
    if size >= 256:
        return seisgen.c5_model(seed, n=size, border=20, nt=1600, shots_xy=(4, 2))
    return seisgen.c5_model(seed, n=size)


SEED_BASE = {128: 5000, 256: 6000}  # training seeds; validation continues after them


def main(argv=None):
    """python -m paper_2502_12350_amd.precond --data 128:512:1 --epochs E --out weights.npz

    Generates training pairs with the solver (for each size:models:crops
    entry, models of that size with seeds SEED_BASE[size] + i, each giving
    `crops` random crops of --crop cells, or the whole volume when crops is
    1 and the size equals the crop), trains the network, and reports the
    validation cosine between each direction and the true perturbation
    (network vs the plain illumination-compensated gradient) on whole
    validation volumes."""
    import argparse
    import json
    import sys
    import time
    import torch
    from .api import Propagator

    ap = argparse.ArgumentParser()
    ap.add_argument("--data", default="128:512:1", help="comma list of size:models:crops")
    ap.add_argument("--val", default="128:16", help="comma list of size:models")
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--decay", type=float, default=0.75, help="learning-rate factor per epoch")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="precond.npz")
    args = ap.parse_args(argv)

    prop = Propagator(0)
    net = Preconditioner(0, seed=args.seed)
    rng = np.random.default_rng(args.seed)
    xs, ts, val = [], [], []
    t0 = time.perf_counter()
    done = 0

    def pair(size, seed):
        nonlocal done
        w = recipe_model(size, seed)
        grad, illum, dv = solver_pair(prop, w)
        done += 1
        if done % 16 == 0:
            torch.cuda.synchronize()
            print(f"[precond] {done} pairs in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
        return grad, illum, dv

    counts = {}
    for item in args.data.split(","):
        size, models, crops = (int(v) for v in item.split(":"))
        counts[size] = models
        for i in range(models):
            grad, illum, dv = pair(size, SEED_BASE[size] + i)
            x = net.pack_input(grad, illum)
            t = dv / dv.abs().max()
            c = args.crop
            if crops == 1 and size <= c:
                xs.append(x)
                ts.append(t.contiguous())
                continue
            for _ in range(crops):
                z0, y0, x0 = (int(v) for v in rng.integers(0, size - c + 1, 3))
                xs.append(x[z0:z0 + c, y0:y0 + c, x0:x0 + c].contiguous())
                ts.append(t[z0:z0 + c, y0:y0 + c, x0:x0 + c].contiguous())
    for item in args.val.split(","):
        size, models = (int(v) for v in item.split(":"))
        for i in range(models):
            grad, illum, dv = pair(size, SEED_BASE[size] + counts.get(size, 0) + i)
            val.append((net.pack_input(grad, illum), dv / dv.abs().max(), grad, illum, dv, size))
    prop.release_workspace()
    t_data = time.perf_counter() - t0

    def validate():
        res = {}
        for x, t, grad, illum, dv, size in val:
            y = net.forward(x)
            r = res.setdefault(size, ([], [], []))
            r[0].append(float(torch.mean((y - t) ** 2)))
            r[1].append(cosine(y, dv))
            r[2].append(cosine(fallback_direction(grad, illum), dv))
        return {str(k): {"loss": float(np.mean(v[0])), "cos_net": float(np.mean(v[1])),
                         "cos_fallback": float(np.mean(v[2]))} for k, v in res.items()}

    def show(tag, h):
        print(f"[precond] {tag}: " + "; ".join(
            f"{k}^3 val loss {v['loss']:.4e}, cos net {v['cos_net']:.3f}, "
            f"cos fallback {v['cos_fallback']:.3f}" for k, v in h.items()),
            file=sys.stderr, flush=True)

    def score(h):  # mean validation cosine of the network's direction over the sizes
        return float(np.mean([v["cos_net"] for v in h.values()]))

    hist = [validate()]
    show("before training", hist[0])
    best = (score(hist[0]), 0, [t.clone() for t in net.w + net.b])
    t1 = time.perf_counter()
    steps = 0
    for ep in range(args.epochs):
        lr = args.lr * (args.decay ** ep)
        for k in rng.permutation(len(xs)):
            net.train_step(xs[k], ts[k], lr=lr)
            steps += 1
        torch.cuda.synchronize()
        hist.append(validate())
        show(f"epoch {ep + 1} ({time.perf_counter() - t1:.1f} s)", hist[-1])
        if score(hist[-1]) > best[0]:
            best = (score(hist[-1]), ep + 1, [t.clone() for t in net.w + net.b])
    t_train = time.perf_counter() - t1
    for dst, src in zip(net.w + net.b, best[2]):  # keep the best epoch's weights
        dst.copy_(src)
    net.pack()
    print(f"[precond] kept epoch {best[1]} (mean validation cosine {best[0]:.3f})",
          file=sys.stderr, flush=True)
    net.save(args.out)
    print(json.dumps({"data": args.data, "val": args.val, "crop": args.crop,
                      "epochs": args.epochs, "lr": args.lr, "decay": args.decay,
                      "samples": len(xs), "train_steps": steps, "kept_epoch": best[1],
                      "data_seconds": round(t_data, 1), "train_seconds": round(t_train, 1),
                      "history": hist}), flush=True)


if __name__ == "__main__":
    main()
