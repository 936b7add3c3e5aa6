"""Surrogate-network kernels on the GPU against the FP64 numpy oracle.

Inputs are drawn in FP64, rounded to BF16 and given to both sides, so the
only differences are FP32 accumulation order and the rounding of BF16
outputs.  Accumulation bound: |gpu - ref| <= 2e-5 * (same sum of absolute
terms) + 1e-6, the sum of absolute terms coming from the oracle applied to
|x| and |w|."""
import numpy as np
import pytest

from oracle import nn_oracle as N

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available()
    from paper_1511_04633_amd import unet
    unet.nn()


def bits_of(a):
    f = N.bf16_round(a).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def to_bf(a):
    import torch
    return torch.tensor(bits_of(a).view(np.int16)).view(torch.bfloat16).cuda()


def from_bf(t):
    import torch
    b = t.view(torch.int16).cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def to_f32(a):
    import torch
    return torch.tensor(np.asarray(a, np.float32)).cuda()


def rnd(shape, seed, scale=1.0):
    return N.bf16_round(np.random.default_rng(seed).standard_normal(shape) * scale)


def S():
    from paper_1511_04633_amd import unet
    return unet.stream_ptr()


def call(name, *a):
    from paper_1511_04633_amd import unet
    unet.call(name, *a)
    import torch
    torch.cuda.synchronize()


def P(t):
    from paper_1511_04633_amd import unet
    return unet.P(t)


SHAPES = [(2, 6, 6, 6), (1, 5, 4, 7), (1, 9, 10, 35)]  # the last: 3 ragged bricks per axis
CHANNELS = [(16, 16), (48, 16), (16, 32), (32, 96), (160, 64), (16, 160), (16, 256)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("ci,co", CHANNELS)
def test_conv_forward(shape, ci, co):
    import torch
    print(f"case: conv fwd {shape} {ci}->{co}", flush=True)
    B, D, H, W = shape
    x, w, b = rnd((B, D, H, W, ci), 1), rnd((co, 27, ci), 2, 0.1), rnd((co,), 3)
    ref = N.conv3d(x, w, b)
    bound = 2e-5 * (N.conv3d(np.abs(x), np.abs(w), np.abs(b))) + 1e-6
    tx, tw, tb = to_bf(x), to_bf(w), to_f32(b)  # keep the device buffers alive
    out = torch.empty((B, D, H, W, co), dtype=torch.float32, device="cuda")
    call("lbmx_nn_conv3d_fwd", P(tx), P(tw), P(tb), P(out), 1, B, D, H, W, ci, co, S())
    err = np.abs(out.cpu().numpy() - ref)
    assert np.all(err <= bound), (err.max(), (err / bound).max())
    ob = torch.empty((B, D, H, W, co), dtype=torch.bfloat16, device="cuda")
    call("lbmx_nn_conv3d_fwd", P(tx), P(tw), P(tb), P(ob), 0, B, D, H, W, ci, co, S())
    assert np.all(np.abs(from_bf(ob) - ref) <= 2 ** -8 * np.abs(ref) + bound)


@pytest.mark.parametrize("ci,co", [(16, 16), (48, 16), (16, 32), (32, 96)])
def test_conv_forward_many_bricks(ci, co):
    """4 x 36 x 34 x 40 voxels: 972 bricks of 16 x 4 x 4 (ragged in x, y
    and z), several waves of blocks on the GPU (one and several rounds of 16
    input channels, one and two channel tiles per block, one and several
    tile groups), at a size whose full FP64 convolution is too slow for the
    oracle: checked on 600 seeded voxels plus the corners against the
    oracle's pointwise sum."""
    import torch
    print(f"case: conv fwd many bricks {ci}->{co}", flush=True)
    B, D, H, W = 4, 36, 34, 40
    x, w, b = rnd((B, D, H, W, ci), 11), rnd((co, 27, ci), 12, 0.1), rnd((co,), 13)
    tx, tw, tb = to_bf(x), to_bf(w), to_f32(b)
    out = torch.empty((B, D, H, W, co), dtype=torch.float32, device="cuda")
    call("lbmx_nn_conv3d_fwd", P(tx), P(tw), P(tb), P(out), 1, B, D, H, W, ci, co, S())
    got = out.cpu().numpy()
    rng = np.random.default_rng(14)
    pts = [(int(rng.integers(B)), int(rng.integers(D)), int(rng.integers(H)), int(rng.integers(W)))
           for _ in range(600)]
    pts += [(bi, z, y, xx) for bi in (0, B - 1) for z in (0, D - 1) for y in (0, H - 1)
            for xx in (0, W - 1)]
    ref = N.conv3d_at(x, w, b, pts)
    bound = 2e-5 * N.conv3d_at(np.abs(x), np.abs(w), np.abs(b), pts) + 1e-6
    g = np.array([got[p] for p in pts])
    assert np.all(np.abs(g - ref) <= bound), (np.abs(g - ref).max(), (np.abs(g - ref) / bound).max())


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("ci,co", [(16, 16), (48, 16), (32, 96), (160, 64)])
def test_conv_data_gradient(shape, ci, co):
    import torch
    print(f"case: conv dgrad {shape} {ci}->{co}", flush=True)
    B, D, H, W = shape
    g, w = rnd((B, D, H, W, co), 4), rnd((co, 27, ci), 5, 0.1)
    ref = N.conv3d_dgrad(g, w)
    bound = 2e-5 * N.conv3d_dgrad(np.abs(g), np.abs(w)) + 1e-6
    tw, tg = to_bf(w), to_bf(g)
    wt = torch.empty((ci, 27, co), dtype=torch.bfloat16, device="cuda")
    call("lbmx_nn_conv3d_flip", P(tw), P(wt), ci, co, S())
    out = torch.empty((B, D, H, W, ci), dtype=torch.float32, device="cuda")
    call("lbmx_nn_conv3d_fwd", P(tg), P(wt), None, P(out), 1, B, D, H, W, co, ci, S())
    err = np.abs(out.cpu().numpy() - ref)
    assert np.all(err <= bound), (err.max(), (err / bound).max())


@pytest.mark.parametrize("shape", SHAPES + [(2, 16, 16, 16)])
@pytest.mark.parametrize("ci,co", [(16, 16), (48, 16), (32, 96), (160, 64), (96, 96)])
def test_conv_weight_gradient(shape, ci, co):
    """Against the oracle, shapes with partial 16 x 4 x 4 bricks in every
    direction (1 x 9 x 10 x 35: three bricks along each axis, the last ones
    ragged) and one brick smaller than a brick (1 x 5 x 4 x 7)."""
    import torch
    print(f"case: conv wgrad {shape} {ci}->{co}", flush=True)
    B, D, H, W = shape
    x, g = rnd((B, D, H, W, ci), 6), rnd((B, D, H, W, co), 7)
    gw_ref, gb_ref = N.conv3d_wgrad(x, g)
    bw, bb = N.conv3d_wgrad(np.abs(x), np.abs(g))
    gw = torch.full((co, 27, ci), 0.5, dtype=torch.float32, device="cuda")  # accumulates
    gb = torch.full((co,), -0.25, dtype=torch.float32, device="cuda")
    tx, tg = to_bf(x), to_bf(g)
    call("lbmx_nn_conv3d_wgrad", P(tx), P(tg), P(gw), P(gb), B, D, H, W, ci, co, S())
    err = np.abs(gw.cpu().numpy() - 0.5 - gw_ref)
    assert np.all(err <= 2e-5 * bw + 1e-5), (err.max(), (err / (2e-5 * bw + 1e-5)).max())
    assert np.all(np.abs(gb.cpu().numpy() + 0.25 - gb_ref) <= 2e-5 * bb + 1e-5)


def test_pool_upsample_concat():
    import torch
    B, D, H, W, C = 2, 4, 6, 8, 32
    x = rnd((B, D, H, W, C), 8)
    p = torch.empty((B, D // 2, H // 2, W // 2, C), dtype=torch.bfloat16, device="cuda")
    tx = to_bf(x)
    call("lbmx_nn_pool2", P(tx), P(p), B, D, H, W, C, 0, S())
    ref = N.pool2(x)
    assert np.all(np.abs(from_bf(p) - ref) <= 2 ** -8 * np.abs(ref) + 1e-7)
    gy = rnd((B, D // 2, H // 2, W // 2, C), 9)
    gx = torch.empty((B, D, H, W, C), dtype=torch.bfloat16, device="cuda")
    tgy = to_bf(gy)
    call("lbmx_nn_pool2", P(tgy), P(gx), B, D, H, W, C, 1, S())
    assert np.array_equal(from_bf(gx), N.pool2_bwd(gy))  # division by 8 is exact
    u = torch.empty((B, 2 * D, 2 * H, 2 * W, C), dtype=torch.bfloat16, device="cuda")
    call("lbmx_nn_up2", P(tx), P(u), B, D, H, W, C, 0, S())
    assert np.array_equal(from_bf(u), N.up2(x))
    gu = rnd((B, 2 * D, 2 * H, 2 * W, C), 10)
    gd = torch.empty((B, D, H, W, C), dtype=torch.bfloat16, device="cuda")
    tgu = to_bf(gu)
    call("lbmx_nn_up2", P(tgu), P(gd), B, D, H, W, C, 1, S())
    ref = N.up2_bwd(gu)
    assert np.all(np.abs(from_bf(gd) - ref) <= 2 ** -8 * np.abs(ref) + 1e-6)
    a, b = rnd((B, D, H, W, 16), 11), rnd((B, D, H, W, 32), 12)
    cat = torch.empty((B, D, H, W, 48), dtype=torch.bfloat16, device="cuda")
    ta, tb = to_bf(a), to_bf(b)
    call("lbmx_nn_concat", P(ta), P(tb), P(cat), B * D * H * W, 16, 32, 0, S())
    assert np.array_equal(from_bf(cat), np.concatenate([a, b], axis=-1))
    ga = torch.empty_like(ta)
    gb = torch.empty_like(tb)
    call("lbmx_nn_concat", P(ga), P(gb), P(cat), B * D * H * W, 16, 32, 1, S())
    assert np.array_equal(from_bf(ga), a) and np.array_equal(from_bf(gb), b)


def test_silu_add_mse_adam_layout_input():
    import torch
    z, ga = rnd((5000,), 13, 3.0), rnd((5000,), 14)
    a = torch.empty(5000, dtype=torch.bfloat16, device="cuda")
    tz, tga = to_bf(z), to_bf(ga)
    call("lbmx_nn_silu", P(tz), P(a), 5000, S())
    ref = N.silu(z)
    assert np.all(np.abs(from_bf(a) - ref) <= 2 ** -8 * np.abs(ref) + 1e-6)
    gz = torch.empty(5000, dtype=torch.bfloat16, device="cuda")
    call("lbmx_nn_silu_bwd", P(tz), P(tga), P(gz), 5000, S())
    ref = N.silu_bwd(z, ga)
    assert np.all(np.abs(from_bf(gz) - ref) <= 2 ** -8 * np.abs(ref) + 1e-5)
    s = torch.empty(5000, dtype=torch.bfloat16, device="cuda")
    call("lbmx_nn_add", P(tz), P(tga), P(s), 5000, S())
    ref = z + ga
    assert np.all(np.abs(from_bf(s) - ref) <= 2 ** -8 * np.abs(ref) + 1e-7)
    # squared error
    V = 3000
    pred, tgt = np.random.default_rng(15).standard_normal((V, 16)), np.random.default_rng(16).standard_normal((V, 4))
    grad = torch.empty((V, 16), dtype=torch.bfloat16, device="cuda")
    part = torch.zeros(64, dtype=torch.float64, device="cuda")
    tp, tt = to_f32(pred), to_f32(tgt)
    call("lbmx_nn_mse", P(tp), P(tt), P(grad), P(part), 64, V, 16, 4, S())
    p32, t32 = pred.astype(np.float32).astype(np.float64), tgt.astype(np.float32).astype(np.float64)
    loss, g = N.mse(p32, t32, 4)
    assert abs(part.cpu().numpy().sum() / (V * 4) - loss) <= 1e-6 * loss
    assert np.all(np.abs(from_bf(grad) - g) <= 2 ** -8 * np.abs(g) + 1e-12)
    # Adam
    n = 1000
    rng = np.random.default_rng(17)
    w, gr = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    tw, tg = to_f32(w), to_f32(gr)
    tm, tv = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    wb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    wr, mr, vr = w.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        tg.copy_(torch.tensor(gr * step))
        call("lbmx_nn_adam", P(tw), P(tg), P(tm), P(tv), P(wb), n, 1e-2, 0.9, 0.999, 1e-8, step,
             1e-3, S())
        wr, mr, vr = N.adam(wr, gr.astype(np.float64) * step, mr, vr, 1e-2, 0.9, 0.999, 1e-8, step, 1e-3)
    assert np.abs(tw.cpu().numpy() - wr).max() < 1e-6
    assert np.array_equal(from_bf(wb), N.bf16_round(tw.cpu().numpy()))
    assert np.abs(tg.cpu().numpy()).max() == 0  # gradient cleared
    # layout with scale
    B, K, C, V = 2, 4, 16, 50
    a = np.random.default_rng(18).standard_normal((B, K, V))
    sc = np.array([1.0, 2.0, 0.5, 4.0], np.float32)
    cl = torch.empty((B, V, C), dtype=torch.float32, device="cuda")
    ta, tsc, tinv = to_f32(a), to_f32(sc), to_f32(1 / sc)
    call("lbmx_nn_layout", P(ta), P(cl), B, V, K, C, 1, P(tsc), S())
    ref = np.zeros((B, V, C))
    ref[..., :K] = np.transpose(a.astype(np.float32), (0, 2, 1)) * sc
    assert np.abs(cl.cpu().numpy() - ref).max() < 1e-6
    back = torch.empty((B, K, V), dtype=torch.float32, device="cuda")
    call("lbmx_nn_layout", P(cl), P(back), B, V, K, C, 0, P(tinv), S())
    assert np.abs(back.cpu().numpy() - a).max() < 1e-6
    # network input (m = 70: rows longer than the kernel's 64 threads)
    cond = to_f32(np.array([[0.25, 2.0], [-1.0, 3.0]]))
    for m in (8, 70):
        x = torch.empty((2, m, m, m, 16), dtype=torch.bfloat16, device="cuda")
        call("lbmx_nn_make_input", P(cond), P(x), 2, m, S())
        xv = from_bf(x)
        assert np.all(xv[0, ..., 0] == 0.25) and np.all(xv[1, ..., 0] == -1.0)
        assert np.all(xv[0, ..., 2] == 1) and np.all(xv[0, ..., 1] == 0) and np.all(xv[0, ..., 3] == 0)
        assert np.all(xv[1, ..., 3] == 1) and np.all(xv[1, ..., 1:3] == 0)
        c = N.bf16_round((2 * np.arange(m) + 1.0) / m - 1.0)
        assert np.array_equal(xv[..., 4], np.broadcast_to(c[None, None, None, :], xv.shape[:4]))
        assert np.array_equal(xv[..., 5], np.broadcast_to(c[None, None, :, None], xv.shape[:4]))
        assert np.array_equal(xv[..., 6], np.broadcast_to(c[None, :, None, None], xv.shape[:4]))
        assert np.all(xv[..., 7:] == 0)


def test_flip_many_and_mse_paths():
    """lbmx_nn_conv3d_flip_many equals the per-layer flips bit for bit, and
    lbmx_nn_adam_flip equals lbmx_nn_adam followed by it; the loss kernel's
    vector path (C % 8 == 0, K <= 8) and scalar path give the oracle's loss
    and gradient."""
    import ctypes
    import torch
    shapes = [(16, 16), (48, 16), (32, 96)]
    ws = [rnd((co, 27, ci), 60 + k) for k, (ci, co) in enumerate(shapes)]
    flat = np.concatenate([w.reshape(-1) for w in ws])
    offs = np.concatenate([[0], np.cumsum([w.size for w in ws])[:-1]])
    tf = to_bf(flat)
    out = torch.empty_like(tf)
    call("lbmx_nn_conv3d_flip_many", P(tf), P(out), len(shapes),
         (ctypes.c_int64 * 3)(*offs.tolist()), (ctypes.c_int32 * 3)(*[c for c, _ in shapes]),
         (ctypes.c_int32 * 3)(*[c for _, c in shapes]), S())
    for k, (ci, co) in enumerate(shapes):
        one = torch.empty((ci, 27, co), dtype=torch.bfloat16, device="cuda")
        tw = to_bf(ws[k])
        call("lbmx_nn_conv3d_flip", P(tw), P(one), ci, co, S())
        o = int(offs[k])
        assert np.array_equal(from_bf(out)[o:o + ws[k].size], from_bf(one).reshape(-1))
    # Adam writing the flipped copies equals Adam + flip_many, bit for bit;
    # a tail of elements outside every layer gets no flipped copy
    tab = ((ctypes.c_int64 * 3)(*offs.tolist()), (ctypes.c_int32 * 3)(*[c for c, _ in shapes]),
           (ctypes.c_int32 * 3)(*[c for _, c in shapes]))
    n = flat.size + 37
    rng = np.random.default_rng(66)
    w0, g0 = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    res = []
    for fused in (True, False):
        tw, tg = to_f32(w0), to_f32(g0)
        tm, tv = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
        wb = torch.zeros(n, dtype=torch.bfloat16, device="cuda")
        wf = torch.zeros(n, dtype=torch.bfloat16, device="cuda")
        for step in (1, 2):
            tg.copy_(to_f32(g0 * step))
            if fused:
                call("lbmx_nn_adam_flip", P(tw), P(tg), P(tm), P(tv), P(wb), P(wf), n, 1e-3, 0.9,
                     0.999, 1e-8, step, 0.01, 3, *tab, S())
            else:
                call("lbmx_nn_adam", P(tw), P(tg), P(tm), P(tv), P(wb), n, 1e-3, 0.9, 0.999, 1e-8,
                     step, 0.01, S())
                call("lbmx_nn_conv3d_flip_many", P(wb), P(wf), 3, *tab, S())
        res.append([bits_of(from_bf(wb)), bits_of(from_bf(wf)), tw.cpu().numpy(), tm.cpu().numpy()])
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    assert not np.any(res[0][1][flat.size:])  # the tail: no flipped copy
    from paper_1511_04633_amd import lbmx as LB
    bad = (ctypes.c_int64 * 3)(int(offs[1]), int(offs[0]), int(offs[2]))  # not ascending
    with pytest.raises(LB.LbmxError):
        call("lbmx_nn_adam_flip", P(tw), P(tg), P(tm), P(tv), P(wb), P(wf), n, 1e-3, 0.9, 0.999,
             1e-8, 3, 0.0, 3, bad, tab[1], tab[2], S())
    for C, K in ((16, 4), (24, 5), (12, 3)):
        V = 3001
        pr, tg = np.random.default_rng(C).standard_normal((V, C)), np.random.default_rng(K).standard_normal((V, K))
        tp, tt = to_f32(pr), to_f32(tg)
        grad = torch.empty((V, C), dtype=torch.bfloat16, device="cuda")
        part = torch.zeros(64, dtype=torch.float64, device="cuda")
        call("lbmx_nn_mse", P(tp), P(tt), P(grad), P(part), 64, V, C, K, S())
        loss, g = N.mse(pr.astype(np.float32), tg.astype(np.float32), K)
        assert abs(part.cpu().numpy().sum() / (V * K) - loss) <= 1e-6 * loss
        assert np.all(np.abs(from_bf(grad) - g) <= 2 ** -8 * np.abs(g) + 1e-12)


def ulp_bf(a):
    """Spacing of BF16 at |a| (2^-7 relative to the power of two below)."""
    a = np.abs(np.asarray(a, np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
    return 2.0 ** (e - 7)


def bf_tensor(shape):
    import torch
    return torch.empty(shape, dtype=torch.bfloat16, device="cuda")


@pytest.mark.parametrize("shape,ci,co", [((2, 6, 6, 6), 16, 32), ((1, 9, 10, 35), 48, 16),
                                         ((1, 5, 4, 7), 32, 96)])
def test_conv_epilogue_options(shape, ci, co):
    """lbmx_nn_conv3d_fwd_ep: (act) z equals the plain convolution and a the
    SiLU kernel applied to it; (gate) the output equals the convolution
    followed by the SiLU-backward kernel; (split) the two outputs are the
    plain output's channel ranges -- all bit for bit (same BF16 roundings in
    the same order); and a, the gated output against the oracle on the
    GPU's own z within one BF16 spacing."""
    print(f"case: conv epilogue {shape} {ci}->{co}", flush=True)
    B, D, H, W = shape
    x, w, b = rnd((B, D, H, W, ci), 31), rnd((co, 27, ci), 32, 0.1), rnd((co,), 33)
    zg = rnd((B, D, H, W, co), 34, 2.0)
    tx, tw, tb, tzg = to_bf(x), to_bf(w), to_f32(b), to_bf(zg)
    plain = bf_tensor((B, D, H, W, co))
    call("lbmx_nn_conv3d_fwd", P(tx), P(tw), P(tb), P(plain), 0, B, D, H, W, ci, co, S())
    n = plain.numel()
    # act
    z, a = bf_tensor(plain.shape), bf_tensor(plain.shape)
    call("lbmx_nn_conv3d_fwd_ep", P(tx), P(tw), P(tb), P(z), P(a), None, None, 0, B, D, H, W, ci,
         co, S())
    a_sep = bf_tensor(plain.shape)
    call("lbmx_nn_silu", P(plain), P(a_sep), n, S())
    assert np.array_equal(bits_of(from_bf(z)), bits_of(from_bf(plain)))
    assert np.array_equal(bits_of(from_bf(a)), bits_of(from_bf(a_sep)))
    ref_a = N.silu(from_bf(z))
    assert np.all(np.abs(from_bf(a) - ref_a) <= ulp_bf(ref_a) + 1e-30)
    # gate
    gated = bf_tensor(plain.shape)
    call("lbmx_nn_conv3d_fwd_ep", P(tx), P(tw), P(tb), P(gated), None, P(tzg), None, 0, B, D, H,
         W, ci, co, S())
    g_sep = bf_tensor(plain.shape)
    call("lbmx_nn_silu_bwd", P(tzg), P(plain), P(g_sep), n, S())
    assert np.array_equal(bits_of(from_bf(gated)), bits_of(from_bf(g_sep)))
    ref_g = N.silu_bwd(zg, from_bf(plain))
    assert np.all(np.abs(from_bf(gated) - ref_g) <= ulp_bf(ref_g) + 1e-30)
    # split
    if co >= 32:
        sp = 16
        o1, o2 = bf_tensor((B, D, H, W, sp)), bf_tensor((B, D, H, W, co - sp))
        call("lbmx_nn_conv3d_fwd_ep", P(tx), P(tw), P(tb), P(o1), None, None, P(o2), sp, B, D, H,
             W, ci, co, S())
        pv = from_bf(plain)
        assert np.array_equal(from_bf(o1), pv[..., :sp]) and np.array_equal(from_bf(o2), pv[..., sp:])
    # rejected combinations
    from paper_1511_04633_amd import lbmx as LB
    for args in ((P(a), P(tzg), None, 0), (None, None, P(a), 0), (None, None, P(a), 8),
                 (P(a), None, P(a), 16)):
        with pytest.raises(LB.LbmxError):
            call("lbmx_nn_conv3d_fwd_ep", P(tx), P(tw), P(tb), P(z), *args, B, D, H, W, ci, co,
                 S())


@pytest.mark.parametrize("shape", [(2, 10, 10, 36), (1, 4, 6, 14)])
def test_conv_with_upcat_input_read_in_place(shape):
    """lbmx_nn_conv3d_fwd_upcat / lbmx_nn_conv3d_wgrad_upcat (a decoder
    layer's input [up2(low) | skip] read in place) against lbmx_nn_upcat
    followed by the plain kernels: the forward bit for bit (same values, same
    summation order), the weight gradients up to the order of the FP32 atomic
    additions; both against the oracle.  (2, 10, 10, 36) has interior bricks
    and ragged ones (x: 16 + 16 + 4), (1, 4, 6, 14) only partial bricks."""
    print(f"case: conv with in-place upsample-and-concatenate input {shape}", flush=True)
    B, D, H, W = shape
    Cu, Cs, Co = 32, 16, 32
    low, sk = rnd((B, D // 2, H // 2, W // 2, Cu), 61), rnd((B, D, H, W, Cs), 62)
    w, b, g = rnd((Co, 27, Cu + Cs), 63, 0.1), rnd((Co,), 64), rnd((B, D, H, W, Co), 65)
    tl, ts, tw, tb, tg = to_bf(low), to_bf(sk), to_bf(w), to_f32(b), to_bf(g)
    cat = bf_tensor((B, D, H, W, Cu + Cs))
    call("lbmx_nn_upcat", P(tl), P(ts), P(cat), B, D // 2, H // 2, W // 2, Cu, Cs, S())
    z1, a1, z2, a2 = (bf_tensor((B, D, H, W, Co)) for _ in range(4))
    call("lbmx_nn_conv3d_fwd_upcat", P(tl), P(ts), P(tw), P(tb), P(z1), P(a1), B, D, H, W, Cu, Cs,
         Co, S())
    call("lbmx_nn_conv3d_fwd_ep", P(cat), P(tw), P(tb), P(z2), P(a2), None, None, 0, B, D, H, W,
         Cu + Cs, Co, S())
    assert np.array_equal(bits_of(from_bf(z1)), bits_of(from_bf(z2)))
    assert np.array_equal(bits_of(from_bf(a1)), bits_of(from_bf(a2)))
    x = np.concatenate([N.up2(low), sk], axis=-1)
    ref = N.conv3d(x, w, b)
    bnd = 2e-5 * N.conv3d(np.abs(x), np.abs(w), np.abs(b)) + 1e-6 + ulp_bf(ref)
    assert np.all(np.abs(from_bf(z1) - ref) <= bnd)
    import torch
    gw1, gw2 = (torch.zeros((Co, 27, Cu + Cs), device="cuda") for _ in range(2))
    gb1, gb2 = (torch.zeros(Co, device="cuda") for _ in range(2))
    call("lbmx_nn_conv3d_wgrad_upcat", P(tl), P(ts), P(tg), P(gw1), P(gb1), B, D, H, W, Cu, Cs, Co,
         S())
    call("lbmx_nn_conv3d_wgrad", P(cat), P(tg), P(gw2), P(gb2), B, D, H, W, Cu + Cs, Co, S())
    gw_ref, gb_ref = N.conv3d_wgrad(x, g)
    bw, bb = N.conv3d_wgrad(np.abs(x), np.abs(g))
    for gw, gb in ((gw1, gb1), (gw2, gb2)):
        assert np.all(np.abs(gw.cpu().numpy() - gw_ref) <= 2e-5 * bw + 1e-5)
        assert np.all(np.abs(gb.cpu().numpy() - gb_ref) <= 2e-5 * bb + 1e-5)
    assert np.abs(gw1.cpu().numpy() - gw2.cpu().numpy()).max() <= 1e-6 * (np.abs(gw_ref).max() + 1)
    # rejected: odd extents, upsampled channels not a multiple of 16 below the total
    from paper_1511_04633_amd import lbmx as LB
    for args in ((B, D, H, W + 1, Cu, Cs), (B, D, H, W, 8, Cs + 24), (B, D, H, W, 0, Cu + Cs)):
        with pytest.raises(LB.LbmxError):
            call("lbmx_nn_conv3d_fwd_upcat", P(tl), P(ts), P(tw), P(tb), P(z1), None, *args, Co, S())
        with pytest.raises(LB.LbmxError):
            call("lbmx_nn_conv3d_wgrad_upcat", P(tl), P(ts), P(tg), P(gw1), None, *args, Co, S())


@pytest.mark.parametrize("shape,K,npart", [((2, 9, 10, 35), 4, 1024), ((1, 5, 4, 7), 6, 1024),
                                           ((2, 8, 8, 32), 16, 8)])
def test_head_convolution_with_fused_loss(shape, K, npart):
    """lbmx_nn_conv3d_mse against lbmx_nn_conv3d_fwd (FP32 output) followed
    by lbmx_nn_mse: prediction and BF16 gradient bit for bit, the loss up to
    FP64 summation order; partial entries past the last block are cleared
    (the buffer starts non-zero); fewer partials than resident blocks
    (npart 8) shrinks the grid; and against the oracle."""
    import torch
    print(f"case: head conv + fused loss {shape} K={K} npartial={npart}", flush=True)
    B, D, H, W = shape
    ci, co = 16, 16
    x, w, b = rnd((B, D, H, W, ci), 71), rnd((co, 27, ci), 72, 0.1), rnd((co,), 73)
    nv = B * D * H * W
    tgt = np.random.default_rng(74).standard_normal((nv, K))
    tx, tw, tb, tt = to_bf(x), to_bf(w), to_f32(b), to_f32(tgt)
    pred1 = torch.empty((nv, co), dtype=torch.float32, device="cuda")
    grad1 = torch.empty((nv, co), dtype=torch.bfloat16, device="cuda")
    part1 = torch.full((npart,), 7.0, dtype=torch.float64, device="cuda")
    call("lbmx_nn_conv3d_mse", P(tx), P(tw), P(tb), P(tt), K, P(grad1), P(part1), npart, P(pred1),
         B, D, H, W, ci, co, S())
    pred2 = torch.empty((nv, co), dtype=torch.float32, device="cuda")
    grad2 = torch.empty((nv, co), dtype=torch.bfloat16, device="cuda")
    part2 = torch.zeros(64, dtype=torch.float64, device="cuda")
    call("lbmx_nn_conv3d_fwd", P(tx), P(tw), P(tb), P(pred2), 1, B, D, H, W, ci, co, S())
    call("lbmx_nn_mse", P(pred2), P(tt), P(grad2), P(part2), 64, nv, co, K, S())
    assert np.array_equal(pred1.cpu().numpy(), pred2.cpu().numpy())
    assert np.array_equal(bits_of(from_bf(grad1)), bits_of(from_bf(grad2)))
    s1, s2 = part1.cpu().numpy().sum(), part2.cpu().numpy().sum()
    assert abs(s1 - s2) <= 1e-12 * s2
    # against the oracle: the prediction, then the loss on the GPU's own prediction
    ref = N.conv3d(x, w, b).reshape(nv, co)
    bnd = 2e-5 * N.conv3d(np.abs(x), np.abs(w), np.abs(b)).reshape(nv, co) + 1e-6
    p1 = pred1.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(p1 - ref) <= bnd)
    loss, g = N.mse(p1, tgt.astype(np.float32).astype(np.float64), K)
    assert abs(s1 / (nv * K) - loss) <= 1e-6 * loss
    assert np.all(np.abs(from_bf(grad1) - g) <= 2 ** -8 * np.abs(g) + 1e-12)
    # without the prediction output: the same gradient
    grad3 = torch.empty((nv, co), dtype=torch.bfloat16, device="cuda")
    call("lbmx_nn_conv3d_mse", P(tx), P(tw), P(tb), P(tt), K, P(grad3), P(part1), npart, None,
         B, D, H, W, ci, co, S())
    assert np.array_equal(bits_of(from_bf(grad3)), bits_of(from_bf(grad1)))
    from paper_1511_04633_amd import lbmx as LB
    for k, n in ((0, npart), (co + 1, npart), (K, 0)):
        with pytest.raises(LB.LbmxError):
            call("lbmx_nn_conv3d_mse", P(tx), P(tw), P(tb), P(tt), k, P(grad3), P(part1), n, None,
                 B, D, H, W, ci, co, S())
    # fewer partials than output-channel tiles (32 channels, one partial)
    w32 = to_bf(rnd((32, 27, ci), 75, 0.1))
    g32 = torch.empty((nv, 32), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(LB.LbmxError):
        call("lbmx_nn_conv3d_mse", P(tx), P(w32), None, P(tt), K, P(g32), P(part1), 1, None,
             B, D, H, W, ci, 32, S())


def test_layout_with_symmetry_transform():
    """lbmx_nn_layout_flip against unet.transform_fields (the host reference,
    itself pinned to the oracle's fields on the CPU) followed by the
    channel-last layout and the per-channel scale, bit for bit, for every
    element of the training symmetry group; channels past K are zero."""
    import ctypes
    import torch
    from paper_1511_04633_amd import unet
    B, m, K, C = 2, 6, 4, 8
    a = np.random.default_rng(91).standard_normal((B, K, m, m, m)).astype(np.float32)
    sc = np.array([0.5, 2.0, -1.5, 3.0], np.float32)
    ta, tsc = to_f32(a), to_f32(sc)
    for g, (flip, signs) in enumerate(unet.SYMMETRIES):
        out = torch.full((B, m ** 3, C), 7.0, dtype=torch.float32, device="cuda")
        call("lbmx_nn_layout_flip", P(ta), P(out), B, m, K, C, flip,
             (ctypes.c_float * K)(*signs), P(tsc), S())
        ref = np.zeros((B, m ** 3, C), np.float32)
        t = unet.transform_fields(a, g).astype(np.float32)  # [B, K, z, y, x]
        ref[..., :K] = t.reshape(B, K, -1).transpose(0, 2, 1) * sc
        assert np.array_equal(out.cpu().numpy(), ref), g
    from paper_1511_04633_amd import lbmx as LB
    with pytest.raises(LB.LbmxError):
        call("lbmx_nn_layout_flip", P(ta), P(out), B, m, K, C, 8, (ctypes.c_float * K)(*signs),
             None, S())


def test_upcat_and_gated_gradients():
    """lbmx_nn_upcat equals up2 + concat (and the oracle's definitions) bit
    for bit; lbmx_nn_pool2_bwd_gate equals pool2 backward + add + SiLU
    backward, lbmx_nn_up2_bwd_gate up2 backward + SiLU backward, bit for bit,
    with and without the optional inputs; against the oracle within one BF16
    spacing per rounding."""
    import torch
    print("case: upcat, gated pooling and upsampling gradients", flush=True)
    B, D, H, W, Ch, Cs = 2, 3, 4, 5, 32, 16
    h, sk = rnd((B, D, H, W, Ch), 41), rnd((B, 2 * D, 2 * H, 2 * W, Cs), 42)
    th, tsk = to_bf(h), to_bf(sk)
    cat = bf_tensor((B, 2 * D, 2 * H, 2 * W, Ch + Cs))
    call("lbmx_nn_upcat", P(th), P(tsk), P(cat), B, D, H, W, Ch, Cs, S())
    assert np.array_equal(from_bf(cat), np.concatenate([N.up2(h), sk], axis=-1))
    # pooling gradient (fine grid 2D x 2H x 2W, coarse D x H x W), add and gate
    C = 32
    g = rnd((B, D, H, W, C), 43)
    add, z = rnd((B, 2 * D, 2 * H, 2 * W, C), 44), rnd((B, 2 * D, 2 * H, 2 * W, C), 45, 2.0)
    tg, tadd, tz = to_bf(g), to_bf(add), to_bf(z)
    for use_add in (False, True):
        for use_gate in (False, True):
            fused = bf_tensor(add.shape)
            call("lbmx_nn_pool2_bwd_gate", P(tg), P(tadd) if use_add else None,
                 P(tz) if use_gate else None, P(fused), B, 2 * D, 2 * H, 2 * W, C, S())
            sep = bf_tensor(add.shape)
            call("lbmx_nn_pool2", P(tg), P(sep), B, 2 * D, 2 * H, 2 * W, C, 1, S())
            ref = N.pool2_bwd(g)
            if use_add:
                call("lbmx_nn_add", P(sep), P(tadd), P(sep), sep.numel(), S())
                ref = N.bf16_round(ref + add)
            if use_gate:
                s2 = bf_tensor(add.shape)
                call("lbmx_nn_silu_bwd", P(tz), P(sep), P(s2), sep.numel(), S())
                sep = s2
                ref = N.silu_bwd(z, ref)
            assert np.array_equal(bits_of(from_bf(fused)), bits_of(from_bf(sep))), (use_add, use_gate)
            assert np.all(np.abs(from_bf(fused) - ref) <= 2 * ulp_bf(ref) + 1e-30)
    # upsampling gradient and gate
    gf = rnd((B, 2 * D, 2 * H, 2 * W, C), 46)
    zc = rnd((B, D, H, W, C), 47, 2.0)
    tgf, tzc = to_bf(gf), to_bf(zc)
    for use_gate in (False, True):
        fused = bf_tensor((B, D, H, W, C))
        call("lbmx_nn_up2_bwd_gate", P(tgf), P(tzc) if use_gate else None, P(fused), B, D, H, W,
             C, S())
        sep = bf_tensor((B, D, H, W, C))
        call("lbmx_nn_up2", P(tgf), P(sep), B, D, H, W, C, 1, S())
        ref = N.up2_bwd(gf)
        if use_gate:
            s2 = bf_tensor((B, D, H, W, C))
            call("lbmx_nn_silu_bwd", P(tzc), P(sep), P(s2), sep.numel(), S())
            sep = s2
            ref = N.silu_bwd(zc, N.bf16_round(ref))
        assert np.array_equal(bits_of(from_bf(fused)), bits_of(from_bf(sep))), use_gate
        assert np.all(np.abs(from_bf(fused) - ref) <= 2 * ulp_bf(ref) + 1e-6)


def test_unet_layers_elementwise_against_oracle():
    """Every layer of a training step (16^3, batch 2, fused kernels) replayed
    in the oracle on the GPU's own BF16 inputs, element by element: forward
    z = conv(x) + b and a = silu(z); weight and bias gradients from the
    GPU's x and dL/dz; data gradients (times the previous layer's SiLU
    derivative where fused, split where the input was a concatenation).
    Bounds: FP32 accumulation, 2e-5 of the same sum of absolute terms, plus
    one BF16 spacing per rounding to BF16."""
    import torch
    from paper_1511_04633_amd import unet

    print("case: unet per-layer replay 16^3 batch 2", flush=True)
    m, B = 16, 2
    net = unet.UNet(seed=3, m=m)
    net.record = []
    cond = to_f32(np.array([[0.3, 1.0], [-0.6, 3.0]]))
    target = to_f32(np.random.default_rng(21).standard_normal((B, m ** 3, 4)) * 0.5)
    pred = net.forward(cond, B, train=True)
    part = torch.zeros(1024, dtype=torch.float64, device="cuda")
    grad, cnt = unet.mse_loss(pred, target, part)
    net.backward(grad)
    torch.cuda.synchronize()
    W = {id(c): N.bf16_round(c.w.cpu().numpy()) for c in net.convs()}
    Bv = {id(c): c.b.cpu().numpy().astype(np.float64) for c in net.convs()}
    nf = nb = 0
    for rec in net.record:
        c = rec["conv"]
        if rec["up"] is not None:  # decoder input read in place: [up2(low) | skip]
            x = np.concatenate([N.up2(from_bf(rec["up"][0])), from_bf(rec["up"][1])], axis=-1)
        else:
            x = from_bf(rec["x"])
        w = W[id(c)]
        if rec["pass"] == "fwd":
            ref = N.conv3d(x, w, Bv[id(c)])
            bnd = 2e-5 * N.conv3d(np.abs(x), np.abs(w), np.abs(Bv[id(c)])) + 1e-6 + ulp_bf(ref)
            z = from_bf(rec["z"])
            assert np.all(np.abs(z - ref) <= bnd), (c.ci, c.co, (np.abs(z - ref) / bnd).max())
            ra = N.silu(z)
            assert np.all(np.abs(from_bf(rec["a"]) - ra) <= ulp_bf(ra) + 1e-30)
            nf += 1
            continue
        gz = from_bf(rec["gz"])
        gw_ref, gb_ref = N.conv3d_wgrad(x, gz)
        bw, bb = N.conv3d_wgrad(np.abs(x), np.abs(gz))
        gw, gb = c.gw.cpu().numpy(), c.gb.cpu().numpy()
        assert np.all(np.abs(gw - gw_ref) <= 2e-5 * bw + 1e-6), (c.ci, c.co, "gw")
        assert np.all(np.abs(gb - gb_ref) <= 2e-5 * bb + 1e-6), (c.ci, c.co, "gb")
        nb += 1
        if rec["dgrad"] is None:
            continue  # the first layer: no gradient w.r.t. the network input
        d = N.conv3d_dgrad(gz, w)
        bd = 2e-5 * N.conv3d_dgrad(np.abs(gz), np.abs(w)) + 1e-6
        if "gate" in rec:
            zp = from_bf(rec["gate"])
            ref = N.silu_bwd(zp, N.bf16_round(d))
            dmax = 1.1 * (bd + ulp_bf(d))  # |silu'| < 1.1
            got = from_bf(rec["dgrad"])
            assert np.all(np.abs(got - ref) <= dmax + ulp_bf(ref)), (c.ci, c.co, "gated")
        else:
            got = from_bf(rec["dgrad"])
            if "dgrad2" in rec:
                got = np.concatenate([got, from_bf(rec["dgrad2"])], axis=-1)
            assert np.all(np.abs(got - d) <= bd + ulp_bf(d)), (c.ci, c.co, "dgrad")
    assert nf == 14 and nb == 14


def test_unet_fused_matches_unfused():
    """The fused training step (epilogues, the decoder inputs read in place,
    the loss in the head's epilogue, gated pooling and upsampling
    gradients) against the separate kernels:
    the same prediction bit for bit, and the same weight gradients up to the
    order of the FP32 atomic additions."""
    import torch
    from paper_1511_04633_amd import unet

    print("case: unet fused vs unfused 16^3 batch 2", flush=True)
    m, B = 16, 2
    cond = to_f32(np.array([[0.1, 2.0], [0.8, 1.0]]))
    target = to_f32(np.random.default_rng(5).standard_normal((B, m ** 3, 4)) * 0.5)
    out = []
    for fused in (True, False):
        net = unet.UNet(seed=7, m=m)
        net.fused = fused
        pred = torch.empty((B, m ** 3, 16), dtype=torch.float32, device="cuda")
        part = torch.zeros(1024, dtype=torch.float64, device="cuda")
        grad, _ = net.forward_loss(cond, B, target, part, pred=pred)
        net.backward(grad)
        torch.cuda.synchronize()
        out.append((pred.cpu().numpy(), [(c.gw.cpu().numpy(), c.gb.cpu().numpy())
                                          for c in net.convs()], part.cpu().numpy().sum(),
                    bits_of(from_bf(grad))))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][3], out[1][3])  # the loss gradient, fused into the head or not
    assert abs(out[0][2] - out[1][2]) <= 1e-12 * out[1][2]
    for (gw1, gb1), (gw2, gb2) in zip(out[0][1], out[1][1]):
        sc = np.abs(gw2).max() + 1e-30
        assert np.abs(gw1 - gw2).max() <= 1e-4 * sc
        assert np.abs(gb1 - gb2).max() <= 1e-4 * (np.abs(gb2).max() + 1e-30)


def _oracle_unet_grads(net, cond_np, target, m):
    """The same network evaluated with the oracle in FP64, rounding to BF16
    wherever the GPU stores BF16; returns the loss and weight gradients."""
    from paper_1511_04633_amd.unet import Conv

    r16 = N.bf16_round
    convs = net.convs()
    W = {id(c): r16(c.w.cpu().numpy()) for c in convs}
    Bv = {id(c): c.b.cpu().numpy().astype(np.float64) for c in convs}
    B = cond_np.shape[0]
    ax = (2 * np.arange(m) + 1.0) / m - 1.0
    x = np.zeros((B, m, m, m, 16))
    for b in range(B):
        x[b, ..., 0] = cond_np[b, 0]
        x[b, ..., int(cond_np[b, 1])] = 1.0
        x[b, ..., 4] = ax[None, None, :]
        x[b, ..., 5] = ax[None, :, None]
        x[b, ..., 6] = ax[:, None, None]
    x = r16(x)
    tape = []

    def conv_act(c, h):
        z = r16(N.conv3d(h, W[id(c)], Bv[id(c)]))
        a = r16(N.silu(z))
        tape.append(("conv", c, h, z))
        return a

    h, skips = x, []
    for lvl, (ca, cb) in enumerate(net.enc):
        h = conv_act(ca, h)
        h = conv_act(cb, h)
        if lvl < 3:
            skips.append(h)
            tape.append(("pool", h.shape))
            h = r16(N.pool2(h))
    for ca, cb in net.dec:
        sk = skips.pop()
        cu = h.shape[-1]
        h = np.concatenate([N.up2(h), sk], axis=-1)
        tape.append(("upcat", cu))
        h = conv_act(ca, h)
        h = conv_act(cb, h)
    pred = N.conv3d(h, W[id(net.head)], Bv[id(net.head)]).astype(np.float32).astype(np.float64)
    loss, g = N.mse(pred.reshape(B, -1, 16), target, 4)
    g = r16(g.reshape(pred.shape))
    grads = {}
    grads[id(net.head)] = N.conv3d_wgrad(h, g)
    g = r16(N.conv3d_dgrad(g, W[id(net.head)]))
    sg = []
    for item in reversed(tape):
        if item[0] == "conv":
            _, c, hin, z = item
            gz = r16(N.silu_bwd(z, g))
            grads[id(c)] = N.conv3d_wgrad(hin, gz)
            g = r16(N.conv3d_dgrad(gz, W[id(c)]))
        elif item[0] == "upcat":
            cu = item[1]
            sg.append(g[..., cu:])
            g = r16(N.up2_bwd(g[..., :cu]))
        else:
            g = r16(r16(N.pool2_bwd(g)) + sg.pop())
    return loss, grads


def test_unet_gradients_against_oracle():
    """End to end: loss and every layer's weight gradient of a small U-Net
    (16^3 input, batch 2) against the oracle-composed network."""
    import torch
    from paper_1511_04633_amd import unet

    print("case: unet gradients 16^3 batch 2", flush=True)
    m, B = 16, 2
    net = unet.UNet(seed=3, m=m)
    cond_np = np.array([[0.3, 1.0], [-0.6, 3.0]])
    cond = to_f32(cond_np)
    rng = np.random.default_rng(21)
    target = rng.standard_normal((B, m ** 3, 4)) * 0.5
    pred = net.forward(cond, B, train=True)
    part = torch.zeros(1024, dtype=torch.float64, device="cuda")
    ttarget = to_f32(target)
    grad, cnt = unet.mse_loss(pred, ttarget, part)
    net.backward(grad)
    torch.cuda.synchronize()
    loss_gpu = part.cpu().numpy().sum() / cnt
    loss_ref, grads = _oracle_unet_grads(net, cond_np, target.astype(np.float32).astype(np.float64), m)
    assert abs(loss_gpu - loss_ref) <= 2e-3 * loss_ref
    for c in net.convs():
        gw_ref, gb_ref = grads[id(c)]
        gw = c.gw.cpu().numpy()
        rel = np.linalg.norm(gw - gw_ref) / np.linalg.norm(gw_ref)
        cos = (gw * gw_ref).sum() / (np.linalg.norm(gw) * np.linalg.norm(gw_ref))
        assert rel < 3e-2 and cos > 0.999, (c.ci, c.co, rel, cos)
        gb = c.gb.cpu().numpy()
        assert np.linalg.norm(gb - gb_ref) <= 3e-2 * np.linalg.norm(gb_ref) + 1e-9


def test_unet_training_reduces_loss():
    """A few Adam steps on one synthetic sample lower the loss (the training
    loop runs entirely through the library kernels).  Without the symmetry
    augmentation: these synthetic targets (w even about the centre) are not
    the cavity's symmetric fields."""
    from paper_1511_04633_amd import unet

    m = 16
    net = unet.UNet(seed=1, m=m)
    yy = (np.arange(m) + 0.5) / m
    th = np.broadcast_to((0.5 - yy)[None, :, None], (m, m, m))
    fields = np.zeros((4, 4, m, m, m), np.float32)
    fields[:, 3] = th
    fields[:, 2] = 0.1 * np.sin(np.pi * yy)[None, :, None]
    hist = unet.train(net, fields, np.array([3.5, 4.0, 5.0, 5.5]), np.array([1, 2, 3, 1]),
                      epochs=40, batch=2, lr=1e-3, augment=False)["loss"]
    assert hist[-1] < 0.2 * hist[0], hist
