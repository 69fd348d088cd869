"""CNN preconditioner kernels on the GPU against the FP64 oracle (oracle/cnn.py).

Each kernel is fed the same BF16-valued inputs as the oracle.  Products of
BF16 values are exact in FP32, so the FP32 results differ from the oracle's
FP64 sums only by summation order: rel-L2 <= 1e-5 (at most 432 terms).
Where a result is stored as BF16, the GPU's FP32 sum and the oracle's FP64 sum
can fall on either side of a rounding boundary, so BF16 outputs must match the
rounded oracle except for at most 1 in 1000 values, each within one BF16 step.
The volume 70 x 7 x 5 spans two 64-wide x tiles with a ragged tail, and
ragged y and z tiles.
"""

import numpy as np
import pytest

from oracle import cnn
from gpu_util import gpu_or_skip, rel_l2, say

pytestmark = pytest.mark.gpu

NZ, NY, NX = 5, 7, 70
TOL = 1e-5


def _bf(torch, a):
    """Oracle BF16-valued array -> device bfloat16 tensor (exact)."""
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


def _bf16_close(got, ref):
    """BF16 outputs: equal to the rounded oracle up to rare one-step flips."""
    ref_q = cnn.bf16(ref)
    diff = got != ref_q
    frac = float(np.mean(diff))
    # one BF16 step at the value (values within 1e-5 of the largest count as
    # that size: near zero the FP32 and FP64 sums can differ in sign)
    step = np.maximum(np.abs(ref_q), 1e-5 * np.max(np.abs(ref_q))) * 2.0 ** -7 + 1e-38
    worst = float(np.max(np.abs(got - ref_q)[diff] / step[diff])) if diff.any() else 0.0
    return frac, worst


def _net(torch, seed=0):
    from paper_2502_12350_amd.precond import Preconditioner
    P = Preconditioner(0, seed=seed)
    rng = np.random.default_rng(seed + 100)
    for b in P.b:  # non-zero biases exercise the bias path
        b.copy_(torch.from_numpy(rng.standard_normal(b.numel()).astype(np.float32) * 0.1))
    Ws = [cnn.bf16(w.cpu().numpy().astype(np.float64).reshape(3, 3, 3, *w.shape[1:]))
          for w in P.w]
    bs = [b.cpu().numpy().astype(np.float64) for b in P.b]
    return P, Ws, bs


@pytest.mark.parametrize("li", [0, 1, 3])
def test_conv_forward_matches_oracle(li):
    torch = gpu_or_skip()
    P, Ws, bs = _net(torch, seed=li)
    ci, co = [(2, 16), (16, 16), (16, 16), (16, 1)][li]
    say(f"[cnn conv] layer {li}: {ci} -> {co} on {NX}x{NY}x{NZ}")
    rng = np.random.default_rng(20 + li)
    x = cnn.bf16(rng.standard_normal((NZ, NY, NX, ci)))
    xd = _bf(torch, x)
    ref = cnn.conv3d(x, Ws[li], bs[li])
    got_f = _np(P.conv(xd, li, relu=False, out_f32=True))
    e = rel_l2(got_f, ref)
    say(f"  FP32 output rel-L2 {e:.2e}")
    assert e <= TOL
    if co == 16:
        got_b = _np(P.conv(xd, li, relu=True))
        frac, worst = _bf16_close(got_b, np.maximum(ref, 0.0))
        say(f"  BF16 relu output: {frac:.1e} of values one step off (worst {worst:.2f} steps)")
        assert frac <= 1e-3 and worst <= 1.0


@pytest.mark.parametrize("li", [1, 2, 3])
def test_data_gradient_matches_oracle(li):
    torch = gpu_or_skip()
    P, Ws, _ = _net(torch, seed=10 + li)
    ci, co = [(2, 16), (16, 16), (16, 16), (16, 1)][li]
    say(f"[cnn dgrad] layer {li}: {co} -> {ci}")
    rng = np.random.default_rng(30 + li)
    dz = cnn.bf16(rng.standard_normal((NZ, NY, NX, co)))
    mask = cnn.bf16(np.maximum(rng.standard_normal((NZ, NY, NX, ci)), 0.0))
    ref = cnn.conv3d_dgrad(dz, Ws[li])
    got = _np(P.conv(_bf(torch, dz), li, relu=False, flip=True, bias=False, out_f32=True))
    e = rel_l2(got, ref)
    say(f"  rel-L2 {e:.2e}")
    assert e <= TOL
    got_m = _np(P.conv(_bf(torch, dz), li, relu=False, flip=True, bias=False,
                       mask=_bf(torch, mask)))
    frac, worst = _bf16_close(got_m, ref * (mask > 0))
    assert frac <= 1e-3 and worst <= 1.0


@pytest.mark.parametrize("li", [0, 1, 3])
def test_weight_gradient_matches_oracle(li):
    torch = gpu_or_skip()
    import ctypes as C
    from paper_2502_12350_amd import _lib
    ci, co = [(2, 16), (16, 16), (16, 16), (16, 1)][li]
    say(f"[cnn wgrad] layer {li}: {ci} -> {co}")
    rng = np.random.default_rng(40 + li)
    x = cnn.bf16(rng.standard_normal((NZ, NY, NX, ci)))
    dz = cnn.bf16(rng.standard_normal((NZ, NY, NX, co)))
    L = _lib.lib()
    nb = C.c_size_t()
    _lib.check(L.wfd_cnn_wgrad_workspace_bytes(NX, NY, NZ, C.byref(nb)))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.full((27, ci, co), float("nan"), device="cuda")
    db = torch.full((co,), float("nan"), device="cuda")
    xd, dzd = _bf(torch, x), _bf(torch, dz)
    _lib.check(L.wfd_cnn_wgrad(xd.data_ptr(), dzd.data_ptr(), NX, NY, NZ, ci, co, dw.data_ptr(),
                               db.data_ptr(), work.data_ptr(), nb.value, None))
    torch.cuda.synchronize()
    ref = cnn.conv3d_wgrad(x, dz).reshape(27, ci, co)
    e = rel_l2(_np(dw), ref)
    eb = rel_l2(_np(db), dz.reshape(-1, co).sum(axis=0))
    say(f"  dW rel-L2 {e:.2e}, db rel-L2 {eb:.2e}")
    assert e <= TOL and eb <= TOL


@pytest.mark.parametrize("ci,co", [(16, 16), (2, 16), (16, 1)])
def test_weight_gradient_many_tiles_per_block(ci, co):
    # 200 x 130 x 70: 4 x 33 x 5 marching tiles (ragged in x, y and z), more
    # than the 512 blocks of the persistent grid, so blocks visit several
    # tiles and 2048 wavefront rows are reduced.  Each wavefront sums up to
    # 8192 exact BF16 products per entry in FP32, each rounding at most 2^-24
    # of a running sum; the bound 2e-5 leaves a factor 4 over sqrt(8192) 2^-24.
    torch = gpu_or_skip()
    import ctypes as C
    from paper_2502_12350_amd import _lib
    nz, ny, nx = 70, 130, 200
    say(f"[cnn wgrad] {nx}x{ny}x{nz}: {ci} -> {co}")
    rng = np.random.default_rng(7 + ci + co)
    x = cnn.bf16(rng.standard_normal((nz, ny, nx, ci)))
    dz = cnn.bf16(rng.standard_normal((nz, ny, nx, co)))
    L = _lib.lib()
    nb = C.c_size_t()
    _lib.check(L.wfd_cnn_wgrad_workspace_bytes(nx, ny, nz, C.byref(nb)))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.full((27, ci, co), float("nan"), device="cuda")
    db = torch.full((co,), float("nan"), device="cuda")
    xd, dzd = _bf(torch, x), _bf(torch, dz)
    res = []
    for _ in range(2):
        _lib.check(L.wfd_cnn_wgrad(xd.data_ptr(), dzd.data_ptr(), nx, ny, nz, ci, co,
                                   dw.data_ptr(), db.data_ptr(), work.data_ptr(), nb.value, None))
        torch.cuda.synchronize()
        res.append((dw.clone(), db.clone()))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])
    ref = cnn.conv3d_wgrad(x, dz).reshape(27, ci, co)
    e = rel_l2(_np(dw), ref)
    eb = rel_l2(_np(db), dz.reshape(-1, co).astype(np.float64).sum(axis=0))
    say(f"  dW rel-L2 {e:.2e}, db rel-L2 {eb:.2e}")
    assert e <= 2e-5 and eb <= 2e-5


@pytest.mark.parametrize("li,flip", [(1, False), (3, False), (1, True)])
def test_convolution_over_several_z_chunks(li, flip):
    # 70 x 7 x 37: three 16-plane chunks per column, the last one ragged; the
    # 16-input-channel kernel carries partial sums of three output planes
    # across its input planes, so chunk starts and ends are the cases to see
    torch = gpu_or_skip()
    nz, ny, nx = 37, 7, 70
    P, Ws, bs = _net(torch, seed=li + 10)
    ci, co = [(2, 16), (16, 16), (16, 16), (16, 1)][li]
    rng = np.random.default_rng(60 + li)
    say(f"[cnn conv] {nx}x{ny}x{nz} layer {li} flip {flip}")
    if flip:  # data gradient: dz (co channels) -> input-gradient (ci channels), ReLU mask
        dz = cnn.bf16(rng.standard_normal((nz, ny, nx, co)))
        act = cnn.bf16(rng.standard_normal((nz, ny, nx, ci)))
        got = P.conv(_bf(torch, dz), li, relu=False, flip=True, bias=False, mask=_bf(torch, act))
        ref = cnn.conv3d_dgrad(dz, Ws[li]) * (act > 0)
    else:
        x = cnn.bf16(rng.standard_normal((nz, ny, nx, ci)))
        got = P.conv(_bf(torch, x), li, relu=li < 3, out_f32=True)
        ref = cnn.conv3d(x, Ws[li], bs[li])
        if li < 3:
            ref = np.maximum(ref, 0.0)
    torch.cuda.synchronize()
    g = _np(got).reshape(ref.shape)
    if got.dtype == torch.bfloat16:
        frac, worst = _bf16_close(g, ref)
        say(f"  BF16 mismatches {frac:.2e}, worst {worst:.2f} steps")
        assert frac <= 1e-3 and worst <= 1.0
    else:
        e = rel_l2(g, ref)
        say(f"  rel-L2 {e:.2e}")
        assert e <= TOL


@pytest.mark.parametrize("shape", [(1, 1, 3), (2, 5, 1), (3, 1, 65), (17, 4, 64)])
def test_tiny_and_degenerate_volumes(shape):
    # one plane, one row, one voxel wide, exactly one tile: every convolution
    # shape (forward, masked data gradient) and every weight gradient
    torch = gpu_or_skip()
    import ctypes as C
    from paper_2502_12350_amd import _lib
    nz, ny, nx = shape
    say(f"[cnn tiny] {nx}x{ny}x{nz}")
    P, Ws, bs = _net(torch, seed=3)
    rng = np.random.default_rng(90 + nz + ny + nx)
    L = _lib.lib()
    nb = C.c_size_t()
    _lib.check(L.wfd_cnn_wgrad_workspace_bytes(nx, ny, nz, C.byref(nb)))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    for li, (ci, co) in enumerate([(2, 16), (16, 16), (16, 16), (16, 1)]):
        x = cnn.bf16(rng.standard_normal((nz, ny, nx, ci)))
        got = _np(P.conv(_bf(torch, x), li, relu=False, out_f32=True)).reshape(nz, ny, nx, co)
        assert rel_l2(got, cnn.conv3d(x, Ws[li], bs[li])) <= TOL
        dz = cnn.bf16(rng.standard_normal((nz, ny, nx, co)))
        if li > 0:
            got = _np(P.conv(_bf(torch, dz), li, relu=False, flip=True, bias=False,
                             out_f32=True)).reshape(nz, ny, nx, ci)
            assert rel_l2(got, cnn.conv3d_dgrad(dz, Ws[li])) <= TOL
        if li != 2:
            dw = torch.full((27, ci, co), float("nan"), device="cuda")
            db = torch.full((co,), float("nan"), device="cuda")
            xd, dzd = _bf(torch, x), _bf(torch, dz)  # alive until the kernels have run
            _lib.check(L.wfd_cnn_wgrad(xd.data_ptr(), dzd.data_ptr(), nx, ny, nz, ci, co,
                                       dw.data_ptr(), db.data_ptr(), work.data_ptr(), nb.value,
                                       None))
            torch.cuda.synchronize()
            assert rel_l2(_np(dw), cnn.conv3d_wgrad(x, dz).reshape(27, ci, co)) <= TOL
            assert rel_l2(_np(db), dz.reshape(-1, co).astype(np.float64).sum(axis=0)) <= TOL


def test_full_size_256_sampled_outputs_and_weight_gradient():
    # the 256^3 volume of the kernel benchmark, in its launch configuration:
    # the 16 -> 16 convolution and its data gradient at 2000 sampled voxels
    # (plus the 8 corners), each against the oracle on the voxel's 3x3x3
    # neighbourhood (zero outside the volume); the 16 -> 16 weight gradient in
    # full against the oracle's FP64 sums over all 16.7 M voxels
    torch = gpu_or_skip()
    import ctypes as C
    from paper_2502_12350_amd import _lib
    n = 256
    P, Ws, bs = _net(torch, seed=5)
    rng = np.random.default_rng(256)
    x = cnn.bf16(rng.standard_normal((n, n, n, 16), dtype=np.float32))
    xd = _bf(torch, x)
    y = P.conv(xd, 1, relu=False, out_f32=True)
    dg = P.conv(xd, 1, relu=False, flip=True, bias=False, out_f32=True)
    torch.cuda.synchronize()
    pts = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(2000)]
    pts += [(a, b, c) for a in (0, n - 1) for b in (0, n - 1) for c in (0, n - 1)]
    idx = torch.tensor(pts, device="cuda")
    gy = y[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    gd = dg[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    worst_y = worst_d = 0.0
    for i, (z, yy, xx) in enumerate(pts):
        sub = np.zeros((3, 3, 3, 16))
        z0, z1, y0, y1, x0, x1 = max(z - 1, 0), min(z + 2, n), max(yy - 1, 0), min(yy + 2, n), \
            max(xx - 1, 0), min(xx + 2, n)
        sub[z0 - z + 1:z1 - z + 1, y0 - yy + 1:y1 - yy + 1, x0 - xx + 1:x1 - xx + 1] = \
            x[z0:z1, y0:y1, x0:x1]
        ry = cnn.conv3d(sub, Ws[1], bs[1])[1, 1, 1]
        rd = cnn.conv3d_dgrad(sub, Ws[1])[1, 1, 1]
        worst_y = max(worst_y, float(np.linalg.norm(gy[i] - ry) / np.linalg.norm(ry)))
        worst_d = max(worst_d, float(np.linalg.norm(gd[i] - rd) / np.linalg.norm(rd)))
    say(f"[cnn 256^3] worst sampled rel error: conv {worst_y:.2e}, data gradient {worst_d:.2e}")
    assert worst_y <= TOL and worst_d <= TOL
    del y, dg
    dz = cnn.bf16(rng.standard_normal((n, n, n, 16), dtype=np.float32))
    dzd = _bf(torch, dz)
    L = _lib.lib()
    nb = C.c_size_t()
    _lib.check(L.wfd_cnn_wgrad_workspace_bytes(n, n, n, C.byref(nb)))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.full((27, 16, 16), float("nan"), device="cuda")
    db = torch.full((16,), float("nan"), device="cuda")
    _lib.check(L.wfd_cnn_wgrad(xd.data_ptr(), dzd.data_ptr(), n, n, n, 16, 16, dw.data_ptr(),
                               db.data_ptr(), work.data_ptr(), nb.value, None))
    torch.cuda.synchronize()
    e = rel_l2(_np(dw), cnn.conv3d_wgrad(x, dz).reshape(27, 16, 16))
    eb = rel_l2(_np(db), dz.reshape(-1, 16).sum(axis=0))
    say(f"  weight gradient rel-L2 {e:.2e}, bias gradient {eb:.2e}")
    # FP32 partial sums over up to 8 tiles x 16 planes x 64 voxels per wavefront,
    # then 2048 rows: the bound of the 200x130x70 case
    assert e <= 2e-5 and eb <= 2e-5


def test_mse_adam_and_input_packing_match_oracle():
    torch = gpu_or_skip()
    import ctypes as C
    from paper_2502_12350_amd import _lib
    L = _lib.lib()
    rng = np.random.default_rng(50)
    n = NZ * NY * NX
    y = rng.standard_normal(n).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    work = torch.empty(_lib.CNN_REDUCE_BYTES, dtype=torch.uint8, device="cuda")
    yd, td = torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda()
    dy = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    _lib.check(L.wfd_cnn_mse(yd.data_ptr(), td.data_ptr(), n, dy.data_ptr(), loss.data_ptr(),
                             work.data_ptr(), work.numel(), None))
    torch.cuda.synchronize()
    ref = cnn.loss(y, t)
    assert abs(float(loss.item()) - ref) <= 1e-12 * ref
    assert np.array_equal(_np(dy), cnn.bf16(2.0 * (y.astype(np.float64) - t) / n))
    # Adam: three steps against the oracle's closed form
    w = rng.standard_normal(1000).astype(np.float32)
    wd = torch.from_numpy(w).cuda()
    md, vd = torch.zeros_like(wd), torch.zeros_like(wd)
    wo, mo, vo = w.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step in (1, 2, 3):
        g = rng.standard_normal(1000).astype(np.float32)
        gd = torch.from_numpy(g).cuda()  # alive until the kernel has run
        _lib.check(L.wfd_cnn_adam(wd.data_ptr(), gd.data_ptr(), md.data_ptr(), vd.data_ptr(),
                                  1000, 1e-2, 0.9, 0.999, 1e-8, step, None))
        torch.cuda.synchronize()
        wo, mo, vo = cnn.adam_step(wo, g.astype(np.float64), mo, vo, step, 1e-2)
    assert rel_l2(_np(wd), wo) <= 1e-6
    # network input
    g = (rng.standard_normal((NZ, NY, NX)) * 1e-12).astype(np.float32)
    il = (np.abs(rng.standard_normal((NZ, NY, NX))) * 1e4).astype(np.float32)
    from paper_2502_12350_amd.precond import Preconditioner
    P = Preconditioner(0)
    got = _np(P.pack_input(torch.from_numpy(g).cuda(), torch.from_numpy(il).cuda()))
    c = g.astype(np.float64) / (il + 1e-3 * il.max())
    frac, worst = _bf16_close(got, np.stack([c / np.abs(c).max(), il / il.max()], axis=-1))
    assert frac <= 1e-3 and worst <= 1.0


def test_network_forward_backward_matches_oracle():
    """The whole network: forward output and every weight/bias gradient against
    the oracle's quantized chain rule (BF16 rounding flips of stored
    activations propagate, so the bound is 1e-2)."""
    torch = gpu_or_skip()
    P, Ws, bs = _net(torch, seed=3)
    say("[cnn network] forward + backward")
    rng = np.random.default_rng(60)
    a0 = cnn.bf16(rng.standard_normal((NZ, NY, NX, 2)))
    t = rng.standard_normal((NZ, NY, NX, 1))
    acts, y_ref = cnn.forward(a0, Ws, bs)
    dWs, dbs = cnn.backward(acts, y_ref, t, Ws)
    y = P.forward(_bf(torch, a0), keep=True)
    loss = P.backward(y, torch.from_numpy(t[..., 0].astype(np.float32)).cuda())
    torch.cuda.synchronize()
    ey = rel_l2(_np(y), y_ref[..., 0])
    say(f"  output rel-L2 {ey:.2e}; loss {float(loss.item()):.6e} vs {cnn.loss(y_ref, t):.6e}")
    assert ey <= 1e-2
    for li in range(4):
        ew = rel_l2(_np(P.dw[li]), dWs[li].reshape(P.dw[li].shape))
        eb = rel_l2(_np(P.db[li]), dbs[li])
        say(f"  layer {li}: dW rel-L2 {ew:.2e}, db rel-L2 {eb:.2e}")
        assert ew <= 1e-2 and eb <= 1e-2


def test_training_lowers_the_loss_and_is_deterministic():
    torch = gpu_or_skip()
    from paper_2502_12350_amd.precond import Preconditioner
    say("[cnn training] 60 Adam steps on a fixed pair")
    rng = np.random.default_rng(70)
    shape = (12, 20, 40)
    g = rng.standard_normal(shape).astype(np.float32)
    il = np.abs(rng.standard_normal(shape)).astype(np.float32)
    runs = []
    for _ in range(2):
        P = Preconditioner(0, seed=5)
        x = P.pack_input(torch.from_numpy(g).cuda(), torch.from_numpy(il).cuda())
        tgt = (-0.5 * x[..., 0].float()).contiguous()   # a linear map of the first channel
        losses = [float(P.train_step(x, tgt, lr=3e-3).item()) for _ in range(60)]
        runs.append((losses, P.w[0].clone()))
    (l1, w1), (l2, w2) = runs
    say(f"  loss {l1[0]:.4e} -> {l1[-1]:.4e}")
    assert l1[-1] < 0.2 * l1[0]
    assert l1 == l2 and torch.equal(w1, w2)
