"""FP64 CPU oracle of the surrogate network's kernels (numpy only).

TEST INFRASTRUCTURE ONLY: the GPU kernels of the U-Net (3x3x3 convolution
forward, data and weight gradients, 2x2x2 average pooling, nearest x2
upsampling, SiLU, squared error, Adam) are compared against these plain
definitions.  Layouts follow the library: activations channel-last
[B][D][H][W][C], weights [Co][27][Ci] with tap t = (kz*3 + ky)*3 + kx at
offset (kx-1, ky-1, kz-1), zero padding.
"""
from __future__ import annotations

import numpy as np


def taps():
    """(tap, dx, dy, dz) for the 27 taps."""
    return [(t, t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1) for t in range(27)]


def _shifted(x, dx, dy, dz):
    """s[b, z, y, x, c] = x[b, z+dz, y+dy, x+dx, c] with zeros outside."""
    B, D, H, W, C = x.shape
    p = np.zeros((B, D + 2, H + 2, W + 2, C), dtype=np.float64)
    p[:, 1:-1, 1:-1, 1:-1, :] = x
    return p[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]


def conv3d(x, w, b=None):
    """out[p, co] = b[co] + sum_{tap, ci} w[co, tap, ci] x[p + off(tap), ci]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros(x.shape[:4] + (w.shape[0],))
    for t, dx, dy, dz in taps():
        out += np.einsum("bzyxi,oi->bzyxo", _shifted(x, dx, dy, dz), w[:, t, :])
    if b is not None:
        out += np.asarray(b, np.float64)
    return out


def conv3d_at(x, w, b, points):
    """conv3d at the given output voxels only: out[k, co] for points[k] =
    (b, z, y, x), the same sum taken voxel by voxel (for tensors too large
    for the whole convolution)."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    B, D, H, W, _ = x.shape
    out = np.zeros((len(points), w.shape[0]))
    for k, (bi, z, y, xx) in enumerate(points):
        acc = np.zeros(w.shape[0]) if b is None else np.array(b, np.float64)
        for t, dx, dy, dz in taps():
            zz, yy, xs = z + dz, y + dy, xx + dx
            if 0 <= zz < D and 0 <= yy < H and 0 <= xs < W:
                acc = acc + w[:, t, :] @ x[bi, zz, yy, xs]
        out[k] = acc
    return out


def conv3d_dgrad(gout, w):
    """Gradient of sum(gout * conv3d(x, w)) with respect to x."""
    gout = np.asarray(gout, np.float64)
    w = np.asarray(w, np.float64)
    gin = np.zeros(gout.shape[:4] + (w.shape[2],))
    for t, dx, dy, dz in taps():
        # out[p] uses x[p + off]: the adjoint sends gout[p] back to p + off
        gin += np.einsum("bzyxo,oi->bzyxi", _shifted(gout, -dx, -dy, -dz), w[:, t, :])
    return gin


def conv3d_wgrad(x, gout):
    """Gradient with respect to w [Co][27][Ci] and the bias [Co]."""
    x = np.asarray(x, np.float64)
    gout = np.asarray(gout, np.float64)
    gw = np.zeros((gout.shape[4], 27, x.shape[4]))
    for t, dx, dy, dz in taps():
        gw[:, t, :] = np.einsum("bzyxo,bzyxi->oi", gout, _shifted(x, dx, dy, dz))
    return gw, gout.sum(axis=(0, 1, 2, 3))


def pool2(x):
    x = np.asarray(x, np.float64)
    B, D, H, W, C = x.shape
    return x.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4, 6))


def pool2_bwd(g):
    g = np.asarray(g, np.float64)
    return np.repeat(np.repeat(np.repeat(g, 2, 1), 2, 2), 2, 3) / 8.0


def up2(x):
    x = np.asarray(x, np.float64)
    return np.repeat(np.repeat(np.repeat(x, 2, 1), 2, 2), 2, 3)


def up2_bwd(g):
    g = np.asarray(g, np.float64)
    B, D, H, W, C = g.shape
    return g.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4, 6))


def silu(z):
    z = np.asarray(z, np.float64)
    return z / (1.0 + np.exp(-z))


def silu_bwd(z, ga):
    z = np.asarray(z, np.float64)
    s = 1.0 / (1.0 + np.exp(-z))
    return np.asarray(ga, np.float64) * s * (1.0 + z * (1.0 - s))


def mse(pred, target, K):
    """Loss over the first K channels and its gradient (zero in the rest)."""
    pred = np.asarray(pred, np.float64)
    target = np.asarray(target, np.float64)
    e = pred[..., :K] - target
    n = e.size
    g = np.zeros_like(pred)
    g[..., :K] = 2.0 * e / n
    return float((e * e).sum() / n), g


def adam(w, g, m, v, lr, b1, b2, eps, step, wd):
    """One bias-corrected Adam step with decoupled weight decay."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v


def bf16_round(a):
    """Round float64 values to the nearest BF16 (ties to even), as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
