"""Pins of the network oracle: against torch's FP64 CPU routines (an
independent library implementation), finite differences and adjoint
identities.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import nn_oracle as N


def rnd(*shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


def torch_conv(x, w, b):
    """torch.nn.functional.conv3d in FP64 on channel-last data, weights [Co][27][Ci]."""
    xt = torch.tensor(x).permute(0, 4, 1, 2, 3)
    Co, _, Ci = w.shape
    wt = torch.tensor(w).reshape(Co, 3, 3, 3, Ci).permute(0, 4, 1, 2, 3)  # [Co][Ci][kz][ky][kx]
    out = torch.nn.functional.conv3d(xt, wt, torch.tensor(b), padding=1)
    return out.permute(0, 2, 3, 4, 1).numpy()


def test_conv_matches_torch():
    x, w, b = rnd(2, 5, 4, 6, 3, seed=1), rnd(4, 27, 3, seed=2), rnd(4, seed=3)
    assert np.abs(N.conv3d(x, w, b) - torch_conv(x, w, b)).max() < 1e-12


def test_conv_at_points_is_the_convolution():
    """The pointwise form agrees with conv3d (itself pinned to torch above)
    at interior, face, edge and corner voxels of a ragged shape."""
    rng = np.random.default_rng(21)
    x = rng.standard_normal((2, 5, 4, 7, 3))
    w = rng.standard_normal((4, 27, 3))
    b = rng.standard_normal(4)
    full = N.conv3d(x, w, b)
    pts = [(0, 0, 0, 0), (1, 4, 3, 6), (0, 2, 1, 3), (1, 0, 2, 6), (0, 4, 0, 2)]
    got = N.conv3d_at(x, w, b, pts)
    for k, (bi, z, y, xx) in enumerate(pts):
        assert np.abs(got[k] - full[bi, z, y, xx]).max() < 1e-12


def test_conv_gradients_match_torch_autograd():
    x, w, b = rnd(2, 4, 5, 3, 3, seed=4), rnd(5, 27, 3, seed=5), rnd(5, seed=6)
    g = rnd(2, 4, 5, 3, 5, seed=7)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    Co, _, Ci = w.shape
    out = torch.nn.functional.conv3d(xt.permute(0, 4, 1, 2, 3),
                                     wt.reshape(Co, 3, 3, 3, Ci).permute(0, 4, 1, 2, 3), bt,
                                     padding=1).permute(0, 2, 3, 4, 1)
    (out * torch.tensor(g)).sum().backward()
    assert np.abs(N.conv3d_dgrad(g, w) - xt.grad.numpy()).max() < 1e-12
    gw, gb = N.conv3d_wgrad(x, g)
    assert np.abs(gw - wt.grad.numpy()).max() < 1e-11
    assert np.abs(gb - bt.grad.numpy()).max() < 1e-12


def test_conv_finite_differences():
    x, w = rnd(1, 3, 3, 3, 2, seed=8), rnd(2, 27, 2, seed=9)
    g = rnd(1, 3, 3, 3, 2, seed=10)
    f = lambda xx, ww: float((N.conv3d(xx, ww) * g).sum())
    h = 1e-6
    gx = N.conv3d_dgrad(g, w)
    gw, _ = N.conv3d_wgrad(x, g)
    for idx in [(0, 0, 0, 0, 0), (0, 1, 2, 0, 1), (0, 2, 2, 2, 0)]:
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        assert abs((f(xp, w) - f(xm, w)) / (2 * h) - gx[idx]) < 1e-7
    for idx in [(0, 0, 0), (1, 13, 1), (0, 26, 1)]:
        wp = w.copy(); wp[idx] += h
        wm = w.copy(); wm[idx] -= h
        assert abs((f(x, wp) - f(x, wm)) / (2 * h) - gw[idx]) < 1e-7


def test_pool_and_upsample_against_torch_and_adjoint():
    x = rnd(2, 4, 6, 4, 3, seed=11)
    xt = torch.tensor(x).permute(0, 4, 1, 2, 3)
    p = torch.nn.functional.avg_pool3d(xt, 2).permute(0, 2, 3, 4, 1).numpy()
    assert np.abs(N.pool2(x) - p).max() < 1e-15
    u = torch.nn.functional.interpolate(xt, scale_factor=2, mode="nearest").permute(0, 2, 3, 4, 1).numpy()
    assert np.abs(N.up2(x) - u).max() == 0
    y = rnd(2, 2, 3, 2, 3, seed=12)
    assert abs((N.pool2(x) * y).sum() - (x * N.pool2_bwd(y)).sum()) < 1e-12
    z = rnd(2, 8, 12, 8, 3, seed=13)
    assert abs((N.up2(x) * z).sum() - (x * N.up2_bwd(z)).sum()) < 1e-11


def test_silu_mse_adam():
    z = rnd(100, seed=14)
    assert np.abs(N.silu(z) - torch.nn.functional.silu(torch.tensor(z)).numpy()).max() < 1e-15
    zt = torch.tensor(z, requires_grad=True)
    ga = rnd(100, seed=15)
    (torch.nn.functional.silu(zt) * torch.tensor(ga)).sum().backward()
    assert np.abs(N.silu_bwd(z, ga) - zt.grad.numpy()).max() < 1e-14
    pred, tgt = rnd(10, 16, seed=16), rnd(10, 4, seed=17)
    loss, g = N.mse(pred, tgt, 4)
    pt = torch.tensor(pred, requires_grad=True)
    l2 = torch.nn.functional.mse_loss(pt[:, :4], torch.tensor(tgt))
    l2.backward()
    assert abs(loss - l2.item()) < 1e-14 and np.abs(g - pt.grad.numpy()).max() < 1e-15
    # Adam against torch.optim.AdamW (decoupled decay: w -= lr*wd*w first, same to 1st order)
    w0, gr = rnd(20, seed=18), rnd(20, seed=19)
    wt = torch.tensor(w0.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(20), np.zeros(20)
    for step in range(1, 4):
        wt.grad = torch.tensor(gr * step)
        opt.step()
        w, m, v = N.adam(w, gr * step, m, v, 1e-2, 0.9, 0.999, 1e-8, step, 0.0)
    assert np.abs(w - wt.detach().numpy()).max() < 1e-12


def test_bf16_round():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159])
    r = N.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0  # tie to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == -2.5 and abs(r[4] - 3.140625) < 1e-12
