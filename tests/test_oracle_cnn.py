"""Pins of the CNN preconditioner oracle (oracle/cnn.py) against facts that do
not come from the oracle itself: a library BF16 cast, hand-worked rounding
ties, brute-force loops, delta kernels, adjoint identities, central
differences and the closed form of one Adam step."""

import numpy as np
import pytest

from oracle import cnn


def _rand(rng, *shape):
    return rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# BF16 rounding
# ---------------------------------------------------------------------------
def test_bf16_matches_torch_cast():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-20, 20, 20000),
                        [0.0, -0.0, 1.0, -3.5, 65504.0, 1e-30]]).astype(np.float32)
    # exact ties between two BF16 neighbours (low 16 bits = 0x8000)
    u = rng.integers(0, 2 ** 31, 4000, dtype=np.uint64).astype(np.uint32)
    ties = ((u & np.uint32(0x7F7F0000)) | np.uint32(0x8000)).view(np.float32)
    a = np.concatenate([a, ties[np.isfinite(ties)]])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(a), ref)


def test_bf16_hand_worked_ties():
    # spacing of BF16 near 1 is 2^-7; 1 + 2^-8 lies half-way between 1 and
    # 1 + 2^-7 and goes to the even mantissa (1); 1 + 3 * 2^-8 lies half-way
    # between 1 + 2^-7 (odd) and 1 + 2^-6 (even) and goes up
    assert cnn.bf16(1.0 + 2.0 ** -8) == 1.0
    assert cnn.bf16(1.0 + 3.0 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert cnn.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert cnn.bf16(-2.0 ** -130) == -2.0 ** -130          # subnormal, exact
    assert cnn.bf16(3.0) == 3.0


# ---------------------------------------------------------------------------
# convolution
# ---------------------------------------------------------------------------
def _brute_conv(x, w, b):
    D, H, W, ci = x.shape
    co = w.shape[-1]
    y = np.zeros((D, H, W, co))
    for z in range(D):
        for yy in range(H):
            for xx in range(W):
                for o in range(co):
                    s = b[o]
                    for kz in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                zz, y2, x2 = z + kz - 1, yy + ky - 1, xx + kx - 1
                                if 0 <= zz < D and 0 <= y2 < H and 0 <= x2 < W:
                                    for c in range(ci):
                                        s += x[zz, y2, x2, c] * w[kz, ky, kx, c, o]
                    y[z, yy, xx, o] = s
    return y


def test_conv_matches_brute_force():
    rng = np.random.default_rng(2)
    x, w, b = _rand(rng, 3, 4, 5, 2), _rand(rng, 3, 3, 3, 2, 3), _rand(rng, 3)
    assert np.allclose(cnn.conv3d(x, w, b), _brute_conv(x, w, b), rtol=0, atol=1e-12)


def test_conv_delta_kernels():
    rng = np.random.default_rng(3)
    x = _rand(rng, 4, 5, 6, 3)
    w = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        w[1, 1, 1, c, c] = 1.0
    assert np.array_equal(cnn.conv3d(x, w), x)
    # tap (kz, ky, kx) = (2, 1, 0) reads x[z + 1, y, x - 1]
    w = np.zeros((3, 3, 3, 3, 1))
    w[2, 1, 0, 1, 0] = 1.0
    y = cnn.conv3d(x, w)[..., 0]
    ref = np.zeros_like(y)
    ref[:-1, :, 1:] = x[1:, :, :-1, 1]
    assert np.array_equal(y, ref)


def test_dgrad_is_the_adjoint():
    rng = np.random.default_rng(4)
    x, w, y = _rand(rng, 5, 4, 6, 16), _rand(rng, 3, 3, 3, 16, 7), _rand(rng, 5, 4, 6, 7)
    lhs = np.sum(cnn.conv3d(x, w) * y)
    rhs = np.sum(x * cnn.conv3d_dgrad(y, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) * 100


def test_wgrad_is_the_weight_derivative():
    rng = np.random.default_rng(5)
    x, y, v = _rand(rng, 4, 6, 5, 2), _rand(rng, 4, 6, 5, 16), _rand(rng, 3, 3, 3, 2, 16)
    lhs = np.sum(cnn.conv3d(x, v) * y)
    rhs = np.sum(v * cnn.conv3d_wgrad(x, y))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_network_gradient_matches_central_differences():
    rng = np.random.default_rng(6)
    Ws, bs = cnn.init_params(7)
    bs = [rng.standard_normal(b.shape) * 0.05 for b in bs]
    a0 = _rand(rng, 5, 6, 4, 2)
    t = _rand(rng, 5, 6, 4, 1)
    acts, y = cnn.forward(a0, Ws, bs, quantize=False)
    dWs, dbs = cnn.backward(acts, y, t, Ws, quantize=False)
    dirs_w = [rng.standard_normal(w.shape) for w in Ws]
    dirs_b = [rng.standard_normal(b.shape) for b in bs]
    h = 1e-5

    def J(s):
        W2 = [w + s * d for w, d in zip(Ws, dirs_w)]
        b2 = [b + s * d for b, d in zip(bs, dirs_b)]
        return cnn.loss(cnn.forward(a0, W2, b2, quantize=False)[1], t)

    fd = (J(h) - J(-h)) / (2 * h)
    an = sum(np.sum(g * d) for g, d in zip(dWs, dirs_w)) + \
        sum(np.sum(g * d) for g, d in zip(dbs, dirs_b))
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_quantized_backward_rounds_where_stored():
    """With quantize=True every stored activation and activation gradient is a
    BF16 value, and the result equals the unquantized chain applied to them."""
    rng = np.random.default_rng(8)
    Ws, bs = cnn.init_params(9)
    a0 = cnn.bf16(_rand(rng, 4, 4, 4, 2))
    t = _rand(rng, 4, 4, 4, 1)
    acts, y = cnn.forward(a0, Ws, bs)
    for a in acts:
        assert np.array_equal(a, cnn.bf16(a))
    dWs, _ = cnn.backward(acts, y, t, Ws)
    dz = cnn.bf16(2.0 * (y - t) / y.size)
    assert np.allclose(dWs[3], cnn.conv3d_wgrad(acts[3], dz), rtol=0, atol=0)


def test_untrained_output_layer_passes_the_first_channel_through():
    rng = np.random.default_rng(11)
    Ws, bs = cnn.init_params(12)
    Ws[3] = np.zeros_like(Ws[3])
    a0 = cnn.bf16(_rand(rng, 3, 5, 4, 2))
    _, y = cnn.forward(a0, Ws, bs)
    assert np.array_equal(y[..., 0], a0[..., 0])


def test_pack_input_scales_each_channel():
    rng = np.random.default_rng(10)
    g, i = _rand(rng, 3, 4, 5) * 1e-20, np.abs(_rand(rng, 3, 4, 5)) * 1e3
    a = cnn.pack_input(g, i)
    assert a.shape == (3, 4, 5, 2)
    assert np.max(np.abs(a[..., 0])) == 1.0 and np.max(a[..., 1]) == 1.0
    assert np.array_equal(a, cnn.bf16(a))
    # constant illumination: channel 0 is the gradient scaled by its maximum
    a = cnn.pack_input(g, np.full(g.shape, 7.0))
    assert np.array_equal(a[..., 0], cnn.bf16(g / np.max(np.abs(g))))
    assert np.all(a[..., 1] == 1.0)
    # the compensation divides by I + eps max I: a point with I = 0 gets
    # 1 / (eps max I) times its gradient, a point with I = max I about 1 / max I
    g2 = np.array([1.0, 1.0]).reshape(1, 1, 2)
    i2 = np.array([0.0, 4.0]).reshape(1, 1, 2)
    a = cnn.pack_input(g2, i2, eps=1e-3)
    assert a[0, 0, 0, 0] == 1.0
    assert a[0, 0, 1, 0] == cnn.bf16((1.0 / 4.004) / (1.0 / 0.004))
    # zero illumination everywhere: raw gradient, unscaled illumination
    a = cnn.pack_input(g2, np.zeros_like(g2))
    assert np.array_equal(a[..., 0], cnn.bf16(g2 / 1.0)) and np.all(a[..., 1] == 0.0)


def test_adam_first_step_closed_form():
    # after one step from zero moments the bias-corrected ratio is g / |g|,
    # so every weight moves by lr * g / (|g| + eps)
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = cnn.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
