"""The surrogate's HIP kernels against the FP64 CPU reference (oracle/cno.py).

Single kernels: the reference is fed the operands the matrix cores see
(rounded to BF16, round-to-nearest-even), so GPU and reference differ only by
FP32 accumulation order -- any indexing or layout mistake shows at once.
Whole network: output and every parameter gradient of the U-Net against the
reference U-Net with the same weights (BF16 rounding of every layer's
operands bounds the agreement, here a few 1e-3 in relative L2)."""
import numpy as np
import pytest

from oracle import cno

pytestmark = pytest.mark.gpu


def bf16(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    r = ((u + np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def host(t):
    return t.double().cpu().numpy()


@pytest.mark.parametrize("shape", [(2, 16, 32, 32, 48), (1, 8, 20, 16, 192), (3, 4, 16, 64, 16), (1, 6, 72, 32, 96),
                                   (2, 3, 128, 16, 64)])
def test_conv_kernels_match_reference(shape):
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream
    B, H, W, ci, co = shape
    rng = np.random.default_rng(sum(shape))
    x = rng.normal(size=(B, H, W, ci)).astype(np.float32)
    w = (rng.normal(size=(9, ci, co)) / np.sqrt(9 * ci)).astype(np.float32)
    b = rng.normal(size=co).astype(np.float32)
    g = rng.normal(size=(B, H, W, co)).astype(np.float32)
    L, st = lib(), _stream()
    dw_, wf, wd = dev(w), torch.empty(w.size, dtype=torch.int16, device="cuda"), torch.empty(w.size, dtype=torch.int16, device="cuda")
    assert L.eelbm_cno_pack_weights(_p(dw_), ci, co, _p(wf), _p(wd), st) == 0
    dx_, db_, dg_ = dev(x), dev(b), dev(g)
    out = torch.empty((B, H, W, co), dtype=torch.float32, device="cuda")
    assert L.eelbm_cno_conv_fwd(_p(dx_), B, H, W, ci, _p(wf), _p(db_), co, _p(out), 0, 0.1, st) == 0
    ref = cno.conv3x3(bf16(x), bf16(w), b.astype(np.float64))
    assert rel(host(out), ref) < 2e-6
    act = torch.empty_like(out)
    assert L.eelbm_cno_conv_fwd(_p(dx_), B, H, W, ci, _p(wf), _p(db_), co, _p(act), 1, 0.1, st) == 0
    assert rel(host(act), cno.leaky(ref, 0.1)) < 2e-6
    din = torch.empty_like(dx_)
    assert L.eelbm_cno_conv_bwd_data(_p(dg_), B, H, W, co, _p(wd), ci, _p(din), st) == 0
    rdx, _, _ = cno.conv3x3_backward(bf16(x), bf16(w), bf16(g))
    assert rel(host(din), rdx) < 2e-6
    gw = torch.zeros_like(dw_)
    gb = torch.zeros_like(db_)
    assert L.eelbm_cno_conv_bwd_weight(_p(dx_), _p(dg_), B, H, W, ci, co, _p(gw), _p(gb), st) == 0
    _, rdw, _ = cno.conv3x3_backward(bf16(x), bf16(w), bf16(g))
    assert rel(host(gw), rdw) < 2e-6
    assert rel(host(gb), g.astype(np.float64).sum(axis=(0, 1, 2))) < 1e-5


@pytest.mark.parametrize("case", [(2, 8, 16, 96, 48, 48, 1), (1, 3, 10, 48, 32, 32, 1), (2, 16, 36, 32, 16, 32, 0),
                                  (1, 4, 40, 192, 96, 96, 1)])
def test_fused_upsample_concat_conv_matches_reference(case):
    """eelbm_cno_conv_fwd_cat: src0 read with nearest 2x upsampling (or as is)
    and concatenated with src1 along channels, in the convolution's loads,
    against the reference convolution of the explicitly built input."""
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream
    B, Hs, Ws, c0, c1, co, up = case
    H, W = (2 * Hs, 2 * Ws) if up else (Hs, Ws)
    rng = np.random.default_rng(sum(case))
    h = rng.normal(size=(B, Hs, Ws, c0)).astype(np.float32)
    skip = rng.normal(size=(B, H, W, c1)).astype(np.float32)
    ci = c0 + c1
    w = (rng.normal(size=(9, ci, co)) / np.sqrt(9 * ci)).astype(np.float32)
    b = rng.normal(size=co).astype(np.float32)
    L, st = lib(), _stream()
    dw_ = dev(w)
    wf = torch.empty(w.size, dtype=torch.int16, device="cuda")
    wd = torch.empty(w.size, dtype=torch.int16, device="cuda")
    assert L.eelbm_cno_pack_weights(_p(dw_), ci, co, _p(wf), _p(wd), st) == 0
    dh, ds, db_ = dev(h), dev(skip), dev(b)
    out = torch.empty((B, H, W, co), dtype=torch.float32, device="cuda")
    assert L.eelbm_cno_conv_fwd_cat(_p(dh), c0, up, _p(ds), c1, B, H, W, _p(wf), _p(db_), co, _p(out), 1, 0.1, st) == 0
    src = cno.up2(h.astype(np.float64)) if up else h.astype(np.float64)
    x = np.concatenate([src, skip.astype(np.float64)], axis=3)
    ref = cno.leaky(cno.conv3x3(bf16(x), bf16(w), b.astype(np.float64)), 0.1)
    assert rel(host(out), ref) < 2e-6
    # an odd image cannot be the 2x upsampling of another
    if up:
        assert L.eelbm_cno_conv_fwd_cat(_p(dh), c0, 1, _p(ds), c1, B, H - 1, W, _p(wf), _p(db_), co, _p(out), 1, 0.1,
                                        st) != 0


@pytest.mark.parametrize("mt", [1, 2, 4])
@pytest.mark.parametrize("chans", [(48, 32), (16, 16)])
def test_every_conv_tile_matches_reference(mt, chans):
    """Each tile the forward convolution can take (MT x 16 pixels per
    wavefront, NT x 16 output channels per workgroup), forced, on a ragged
    image (72 = 64 + 8 columns, 66 = 16 x 4 + 2 rows) with 3 input chunks of
    32 channels (the last one half full: the next chunk's loads overlap the
    products) or one (the weights stay in LDS), and more tiles than the chip
    holds workgroups (each workgroup loops over several); the automatic
    choice restored after."""
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream
    B, H, W, co = 3, 66, 72, 192
    c0, c1 = chans
    rng = np.random.default_rng(mt + c0)
    h = rng.normal(size=(B, H // 2, W // 2, c0)).astype(np.float32)
    skip = rng.normal(size=(B, H, W, c1)).astype(np.float32)
    ci = c0 + c1
    w = (rng.normal(size=(9, ci, co)) / np.sqrt(9 * ci)).astype(np.float32)
    b = rng.normal(size=co).astype(np.float32)
    L, st = lib(), _stream()
    dw_ = dev(w)
    wf = torch.empty(w.size, dtype=torch.int16, device="cuda")
    wd = torch.empty(w.size, dtype=torch.int16, device="cuda")
    assert L.eelbm_cno_pack_weights(_p(dw_), ci, co, _p(wf), _p(wd), st) == 0
    dh, ds, db_ = dev(h), dev(skip), dev(b)
    x = np.concatenate([cno.up2(h.astype(np.float64)), skip.astype(np.float64)], axis=3)
    ref = cno.leaky(cno.conv3x3(bf16(x), bf16(w), b.astype(np.float64)), 0.1)
    out = torch.empty((B, H, W, co), dtype=torch.float32, device="cuda")
    try:
        for nt in (1, 2, 3, 4):
            assert L.eelbm_cno_conv_set_tile(mt, nt) == 0
            out.fill_(float("nan"))
            assert L.eelbm_cno_conv_fwd_cat(_p(dh), c0, 1, _p(ds), c1, B, H, W, _p(wf), _p(db_), co, _p(out), 1, 0.1,
                                            st) == 0, (mt, nt)
            assert rel(host(out), ref) < 2e-6, (mt, nt)
        # 48 output channels: 3 N-tiles, which 2 and 4 do not divide
        assert L.eelbm_cno_conv_set_tile(mt, 2) == 0
        assert L.eelbm_cno_conv_fwd_cat(_p(dh), c0, 1, _p(ds), c1, B, H, W, _p(wf), _p(db_), 48, _p(out), 1, 0.1,
                                        st) != 0
    finally:
        assert L.eelbm_cno_conv_set_tile(0, 0) == 0
    assert L.eelbm_cno_conv_set_tile(3, 1) != 0 and L.eelbm_cno_conv_set_tile(1, 5) != 0


@pytest.mark.parametrize("shape", [(3, 40, 24), (1, 3, 1), (2, 256, 300)])
def test_volume_defect_matches_reference(shape):
    """eelbm_cno_volume_defect against the FP64 reference on random channel
    fields (a 300-wide case: more columns than threads; ny = 3: the rows the
    flux estimate reads overlap)."""
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream
    N, ny, nx = shape
    rng = np.random.default_rng(ny)
    f0 = np.zeros((N, 6, ny, nx), dtype=np.float32)
    f0[:, 0] = rng.uniform(0.01, 0.2, size=(N, ny, nx))
    f0[:, 1:5] = rng.normal(0, 0.01, size=(N, 4, ny, nx))
    f1 = f0 + rng.normal(0, 1e-4, size=f0.shape).astype(np.float32)
    chi = rng.uniform(0.01, 0.3, size=N).astype(np.float32)
    out = torch.empty(N, dtype=torch.float64, device="cuda")
    L = lib()
    assert L.eelbm_cno_volume_defect(_p(dev(f0)), _p(dev(f1)), N, ny, nx, 100, _p(dev(chi)), _p(out), _stream()) == 0
    ref = cno.volume_defect(f0, f1, 100, chi.astype(np.float64))
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-9, atol=1e-13)
    assert L.eelbm_cno_volume_defect(_p(dev(f0)), _p(dev(f1)), N, 2, nx, 100, _p(dev(chi)), _p(out), _stream()) != 0


def test_weight_gradient_is_deterministic():
    """The weight and bias gradients are sums of per-chunk partials added in a
    fixed order: two calls give the same bits."""
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream
    B, H, W, ci, co = 4, 64, 64, 48, 96
    rng = np.random.default_rng(11)
    x, g = dev(rng.normal(size=(B, H, W, ci))), dev(rng.normal(size=(B, H, W, co)))
    L, st = lib(), _stream()
    res = []
    for _ in range(2):
        gw = torch.zeros((9, ci, co), dtype=torch.float32, device="cuda")
        gb = torch.zeros(co, dtype=torch.float32, device="cuda")
        assert L.eelbm_cno_conv_bwd_weight(_p(x), _p(g), B, H, W, ci, co, _p(gw), _p(gb), st) == 0
        res.append((host(gw), host(gb)))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_elementwise_kernels_match_reference():
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream
    L, st = lib(), _stream()
    rng = np.random.default_rng(7)
    B, H, W, C = 2, 8, 12, 16
    x = rng.normal(size=(B, H, W, C)).astype(np.float32)
    y = torch.empty((B, H // 2, W // 2, C), dtype=torch.float32, device="cuda")
    assert L.eelbm_cno_pool(_p(dev(x)), B, H, W, C, _p(y), 0, st) == 0
    assert rel(host(y), cno.pool2(x.astype(np.float64))) < 1e-7
    gy = rng.normal(size=(B, H // 2, W // 2, C)).astype(np.float32)
    gx = torch.empty((B, H, W, C), dtype=torch.float32, device="cuda")
    assert L.eelbm_cno_pool(_p(dev(gy)), B, H, W, C, _p(gx), 1, st) == 0
    assert rel(host(gx), cno.pool2_backward(gy.astype(np.float64))) < 1e-7
    u = torch.empty((B, 2 * H, 2 * W, C), dtype=torch.float32, device="cuda")
    assert L.eelbm_cno_up(_p(dev(x)), B, H, W, C, _p(u), 0, st) == 0
    assert np.array_equal(host(u), cno.up2(x.astype(np.float64)))
    gu = rng.normal(size=(B, 2 * H, 2 * W, C)).astype(np.float32)
    gux = torch.empty((B, H, W, C), dtype=torch.float32, device="cuda")
    assert L.eelbm_cno_up(_p(dev(gu)), B, H, W, C, _p(gux), 1, st) == 0
    assert rel(host(gux), cno.up2_backward(gu.astype(np.float64))) < 1e-6
    a2 = rng.normal(size=(B, H, W, 32)).astype(np.float32)
    cat = torch.empty((B, H, W, 48), dtype=torch.float32, device="cuda")
    assert L.eelbm_cno_concat(_p(dev(x)), C, _p(dev(a2)), 32, B * H * W, _p(cat), st) == 0
    assert np.array_equal(host(cat), np.concatenate([x, a2], axis=3).astype(np.float64))
    da, dbb = torch.empty((B, H, W, C), dtype=torch.float32, device="cuda"), dev(np.ones((B, H, W, 32)))
    assert L.eelbm_cno_split_add(_p(cat), C, 32, B * H * W, _p(da), _p(dbb), st) == 0
    assert np.array_equal(host(da), x.astype(np.float64)) and np.allclose(host(dbb), a2 + 1.0)
    dyv = rng.normal(size=x.shape).astype(np.float32)
    dxv = torch.empty_like(dev(x))
    assert L.eelbm_cno_act_bwd(_p(dev(x)), _p(dev(dyv)), x.size, 0.1, _p(dxv), st) == 0
    assert np.allclose(host(dxv), cno.leaky_backward(x, dyv, 0.1), rtol=1e-6)
    t = rng.normal(size=x.shape).astype(np.float32)
    part = torch.empty(64, dtype=torch.float64, device="cuda")
    dp = torch.empty_like(dev(x))
    assert L.eelbm_cno_mse(_p(dev(x)), _p(dev(t)), B * H * W, C, 6, _p(part), 64, _p(dp), st) == 0
    rl, rg = cno.mse(x.astype(np.float64), t.astype(np.float64), 6)
    assert abs(float(part.sum()) - rl) < 1e-9 * rl and rel(host(dp), rg) < 1e-6
    w0, g0 = rng.normal(size=50).astype(np.float32), rng.normal(size=50).astype(np.float32)
    wt, mt, vt = dev(w0), dev(np.zeros(50)), dev(np.zeros(50))
    for step in (1, 2):
        assert L.eelbm_cno_adam(_p(wt), _p(dev(g0)), _p(mt), _p(vt), 50, 1e-2, 0.9, 0.999, 1e-8, step, 0.0, st) == 0
    rw, rm, rv = cno.adam(w0.astype(np.float64), g0, 0, 0, 1, 1e-2)
    rw, rm, rv = cno.adam(rw, g0, rm, rv, 2, 1e-2)
    assert np.allclose(host(wt), rw, atol=1e-6)


def _net_and_reference(widths, seed_w=5):
    from paper_2409_10399_amd.surrogate import CNO
    net = CNO(cin=9, cout=6, widths=widths, seed=3)
    ref = cno.UNet(cin=16, cout=16, widths=widths, slope=0.1, rng=np.random.default_rng(seed_w))
    ref.params = [(bf16(w), b) for w, b in ref.params]  # the weights the matrix cores see
    net.set_params(ref.params)
    return net, ref


def _compare(net, ref, x, target):
    out = net.forward(dev(x))
    r_out = ref.forward(x)
    part = net.loss(out, dev(target))
    r_loss, r_g = cno.mse(r_out, target, 6)
    net.backward(net.dloss)
    r_grads, _ = ref.backward(r_g)
    ew = [rel(host(tw), gw) for (gw, _), tw in zip(r_grads, net.gW)]
    eb = [rel(host(tb), gb) for (_, gb), tb in zip(r_grads, net.gb) if np.linalg.norm(gb) > 0]
    return rel(host(out), r_out), abs(float(part.sum()) - r_loss) / r_loss, max(ew), max(eb)


@pytest.mark.parametrize("emulate", [True, False])
def test_network_output_and_gradients_match_reference(monkeypatch, emulate):
    """emulate: the reference rounds every convolution operand to BF16 as the
    matrix cores do (forward: input and weights; input gradient: output
    gradient and weights; weight gradient: input and output gradient), so
    only FP32 summation order differs -- and the BF16 roundings it flips
    (2^-8 relative on single elements).  Otherwise: the plain FP64
    reference, off by BF16 rounding through 11 layers."""
    rng = np.random.default_rng(11)
    if emulate:
        conv, back = cno.conv3x3, cno.conv3x3_backward
        monkeypatch.setattr(cno, "conv3x3", lambda x, w, b=None: conv(bf16(x), bf16(w), b))

        def back_rounded(x, w, dout):
            dx, _, db = back(x, bf16(w), bf16(dout))
            _, dw, _ = back(bf16(x), w, bf16(dout))
            return dx, dw, db
        monkeypatch.setattr(cno, "conv3x3_backward", back_rounded)
    net, ref = _net_and_reference([16, 32, 48])
    x = np.zeros((2, 16, 16, 16))
    x[..., :9] = rng.normal(size=(2, 16, 16, 9))
    target = rng.normal(size=(2, 16, 16, 16))
    e_out, e_loss, e_w, e_b = _compare(net, ref, x, target)
    print(f"  emulate={emulate}: output {e_out:.1e} loss {e_loss:.1e} worst weight grad {e_w:.1e} "
          f"worst bias grad {e_b:.1e}", flush=True)
    bound = (1e-3, 1e-4, 1e-2, 1e-2) if emulate else (2e-2, 2e-2, 1.5e-1, 1.5e-1)
    assert e_out < bound[0] and e_loss < bound[1] and e_w < bound[2] and e_b < bound[3]


def test_training_steps_reduce_loss():
    from paper_2409_10399_amd.surrogate import CNO
    rng = np.random.default_rng(12)
    net = CNO(cin=9, cout=6, widths=[16, 32, 48], seed=1)
    x = np.zeros((4, 32, 32, 16))
    x[..., :9] = rng.normal(size=(4, 32, 32, 9))
    target = np.zeros((4, 32, 32, 16))
    target[..., :6] = 0.5 * np.tanh(x[..., :6]) + 0.2 * x[..., 3:9]
    xd, td = dev(x), dev(target)
    losses = []
    for it in range(60):
        out = net.forward(xd)
        losses.append(float(net.loss(out, td).sum()))
        net.backward(net.dloss)
        net.adam(3e-3)
    assert np.isfinite(losses).all() and losses[-1] < 0.5 * losses[0], losses[::10]


def _bf16_bits(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    return (((u + np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))) >> 16) & np.uint32(0xFFFF)).astype(np.uint16)


def _bits_to_f32(b):
    return (b.astype(np.uint32) << 16).view(np.float32)


@pytest.mark.parametrize("in_bf16,out_bf16", [(1, 1), (0, 1), (1, 0)])
def test_bf16_activation_conv_equals_rounded_fp32(in_bf16, out_bf16):
    """BF16 activations: with inputs that BF16 holds exactly, the convolution
    reading BF16 and/or writing BF16 gives the FP32 path's values, rounded to
    BF16 where the output is BF16 -- bit for bit (the fused upsample and
    concatenation included)."""
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream
    B, Hs, Ws, c0, c1, co = 2, 10, 36, 48, 32, 96
    H, W = 2 * Hs, 2 * Ws
    rng = np.random.default_rng(in_bf16 + 2 * out_bf16)
    h = _bits_to_f32(_bf16_bits(rng.normal(size=(B, Hs, Ws, c0))))
    skip = _bits_to_f32(_bf16_bits(rng.normal(size=(B, H, W, c1))))
    ci = c0 + c1
    w = (rng.normal(size=(9, ci, co)) / np.sqrt(9 * ci)).astype(np.float32)
    L, st = lib(), _stream()
    dw_ = dev(w)
    wf = torch.empty(w.size, dtype=torch.int16, device="cuda")
    wd = torch.empty(w.size, dtype=torch.int16, device="cuda")
    assert L.eelbm_cno_pack_weights(_p(dw_), ci, co, _p(wf), _p(wd), st) == 0
    db_ = dev(rng.normal(size=co).astype(np.float32))
    ref = torch.empty((B, H, W, co), dtype=torch.float32, device="cuda")
    assert L.eelbm_cno_conv_fwd_cat(_p(dev(h)), c0, 1, _p(dev(skip)), c1, B, H, W, _p(wf), _p(db_), co, _p(ref), 1,
                                    0.1, st) == 0
    if in_bf16:
        sh = torch.tensor(_bf16_bits(h).view(np.int16), device="cuda")
        ss = torch.tensor(_bf16_bits(skip).view(np.int16), device="cuda")
    else:
        sh, ss = dev(h), dev(skip)
    out = torch.empty((B, H, W, co), dtype=torch.int16 if out_bf16 else torch.float32, device="cuda")
    assert L.eelbm_cno_conv_fwd_cat_dt(_p(sh), c0, 1, _p(ss), c1, B, H, W, _p(wf), _p(db_), co, _p(out), 1, 0.1,
                                       in_bf16, out_bf16, st) == 0
    r = ref.cpu().numpy()
    if out_bf16:
        assert np.array_equal(out.cpu().numpy().view(np.uint16), _bf16_bits(r))
    else:
        assert np.array_equal(out.cpu().numpy(), r)


def test_bf16_pool_and_inference_pass():
    """2x2 pooling of BF16 activations against the same sum in FP32 rounded
    to BF16; the inference pass (BF16 activations) against forward() (FP32
    activations), which it differs from only where pooling sees rounded
    inputs."""
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import CNO, _p, _stream
    rng = np.random.default_rng(4)
    B, H, W, C = 2, 12, 20, 32
    x = _bf16_bits(rng.normal(size=(B, H, W, C)))
    xf = _bits_to_f32(x)
    out = torch.empty((B, H // 2, W // 2, C), dtype=torch.int16, device="cuda")
    assert lib().eelbm_cno_pool_bf16(_p(torch.tensor(x.view(np.int16), device="cuda")), B, H, W, C, _p(out),
                                     _stream()) == 0
    s = ((xf[:, 0::2, 0::2] + xf[:, 0::2, 1::2]) + xf[:, 1::2, 0::2]) + xf[:, 1::2, 1::2]
    assert np.array_equal(out.cpu().numpy().view(np.uint16), _bf16_bits(np.float32(0.25) * s))
    net = CNO(9, 6, [16, 32, 48], seed=3)
    xin = torch.randn((2, 64, 64, net.cin), device="cuda")
    a = net.forward(xin, keep=False).clone()
    b = net.infer(xin).clone()
    assert float((a - b).norm() / a.norm()) < 1e-2
