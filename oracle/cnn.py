"""FP64 oracle of the learned gradient preconditioner (a small 3-D CNN).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product library.  It shares no
code with the GPU path.

The paper smooths the FWI gradient with a fixed filter (its
GradientPreconditioning option: Bessel or Laplace).  The learned replacement
is a 4-layer 3-D convolutional network mapping two input channels to one
output channel, the model update direction.  The inputs are the gradient
divided by the regularised source illumination, g / (I + eps max I) (the
plain preconditioned gradient the network has to improve on), and the
illumination I itself, each scaled by its largest magnitude:

    z1 = C(a0; W1, b1)   a1 = q(relu(z1))        2 -> 16 channels
    z2 = C(a1; W2, b2)   a2 = q(relu(z2))       16 -> 16
    z3 = C(a2; W3, b3)   a3 = q(relu(z3))       16 -> 16
    y  = C(a3; W4, b4) + a0[..., 0]             16 -> 1

The last term passes the first input channel (the scaled plain direction)
through, so the network learns a correction to it.

C is a 3 x 3 x 3 cross-correlation with zero padding ("same" size) plus a
per-channel bias.  Weights and stored activations are BF16 (q = round to
nearest even from FP32), products are exact and sums are taken in FP64 here
(FP32 on the GPU).  Training minimises L = mean((y - t)^2) against the scaled
true perturbation t; the backward pass is the chain rule through the same
graph, with the output gradient and the masked activation gradients rounded
to BF16 where the GPU stores them.

Volumes are channels-last [z][y][x][c]; weights are W[kz][ky][kx][ci][co]
with tap (kz, ky, kx) reading the input at offset (kz - 1, ky - 1, kx - 1).

Pins (tests/test_oracle_cnn.py): BF16 rounding against torch's bfloat16 cast
and hand-worked ties; the convolution against a brute-force loop, a centred
delta (identity) and a shifted delta; the data gradient against the adjoint
identity <C(x), y> = <x, C^T(y)>; the weight gradient against
<C(x; V), y> = <V, dW(x, y)>; the whole network gradient against central
differences; Adam against its closed form after one step.
"""

from __future__ import annotations

import numpy as np

CHANNELS = (2, 16, 16, 16, 1)


# ---------------------------------------------------------------------------
# BF16 storage
# ---------------------------------------------------------------------------
def bf16(a) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even) via FP32; returns FP64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# convolution and its two gradients
# ---------------------------------------------------------------------------
def conv3d(x, w, b=None) -> np.ndarray:
    """y[p, co] = b[co] + sum_{k, ci} x[p + k - 1, ci] w[k, ci, co], zero outside."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((D, H, W, w.shape[-1]))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                y += xp[kz:kz + D, ky:ky + H, kx:kx + W, :] @ w[kz, ky, kx]
    if b is not None:
        y += np.asarray(b, dtype=np.float64)
    return y


def conv3d_dgrad(dy, w) -> np.ndarray:
    """Transpose of conv3d in x: dx[p, ci] = sum_{k, co} dy[p - k + 1, co] w[k, ci, co]."""
    dy = np.asarray(dy, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    D, H, W, _ = dy.shape
    dp = np.pad(dy, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dx = np.zeros((D, H, W, w.shape[-2]))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                dx += dp[2 - kz:2 - kz + D, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W, :] @ \
                    w[kz, ky, kx].T
    return dx


def conv3d_wgrad(x, dy) -> np.ndarray:
    """dW[k, ci, co] = sum_p x[p + k - 1, ci] dy[p, co]."""
    x = np.asarray(x, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    D, H, W, ci = x.shape
    co = dy.shape[-1]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    d2 = dy.reshape(-1, co)
    dw = np.zeros((3, 3, 3, ci, co))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                dw[kz, ky, kx] = xp[kz:kz + D, ky:ky + H, kx:kx + W, :].reshape(-1, ci).T @ d2
    return dw


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def init_params(seed: int):
    """He-uniform weights (BF16) and zero biases, as lists per layer."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        lim = np.sqrt(6.0 / (27 * ci))
        Ws.append(bf16(rng.uniform(-lim, lim, size=(3, 3, 3, ci, co))))
        bs.append(np.zeros(co))
    return Ws, bs


def pack_input(grad, illum, eps: float = 1e-3) -> np.ndarray:
    """Network input [z][y][x][2] in BF16: c = grad / (illum + eps max|illum|)
    scaled by max|c|, and illum scaled by max|illum| (a channel whose maximum
    is 0 is left unscaled)."""
    g = np.asarray(grad, dtype=np.float64)
    i = np.asarray(illum, dtype=np.float64)
    im = np.max(np.abs(i))
    c = g / (i + eps * im) if im > 0 else g
    cm = np.max(np.abs(c))
    a = np.stack([c / cm if cm > 0 else c, i / im if im > 0 else i], axis=-1)
    return bf16(a)


def forward(a0, Ws, bs, quantize: bool = True):
    """Activations [a0, a1, a2, a3] and the output y [z][y][x][1]."""
    q = bf16 if quantize else (lambda v: v)
    acts = [np.asarray(a0, dtype=np.float64)]
    for layer in range(3):
        z = conv3d(acts[-1], Ws[layer], bs[layer])
        acts.append(q(np.maximum(z, 0.0)))
    y = conv3d(acts[-1], Ws[3], bs[3]) + acts[0][..., :1]
    return acts, y


def loss(y, t) -> float:
    """Mean squared error over all voxels."""
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d))


def backward(acts, y, t, Ws, quantize: bool = True):
    """Gradients (dWs, dbs) of loss(y, t) through the network of forward()."""
    q = bf16 if quantize else (lambda v: v)
    y = np.asarray(y, dtype=np.float64)
    dz = q(2.0 * (y - np.asarray(t, dtype=np.float64)) / y.size)
    dWs, dbs = [None] * 4, [None] * 4
    for layer in range(3, -1, -1):
        dWs[layer] = conv3d_wgrad(acts[layer], dz)
        dbs[layer] = dz.reshape(-1, dz.shape[-1]).sum(axis=0)
        if layer > 0:
            da = conv3d_dgrad(dz, Ws[layer])
            dz = q(da * (acts[layer] > 0))
    return dWs, dbs


def adam_step(w, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, Alg. 1) from step-1 moments m, v; returns
    (w, m, v) after the update."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
