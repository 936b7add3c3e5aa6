"""3-D convolutional U-Net surrogate: (log10 Ra, wall type) -> steady
u/u_c, v/u_c, w/u_c, theta on a 64^3 grid, used to warm-start the cavity.

Every arithmetic step runs in the library's HIP kernels (``lbmx_nn_*``):
this module only sequences them and holds device buffers, which PyTorch
allocates (memory only).  Weights are BF16 for the matrix cores with FP32
master copies, FP32 gradients and Adam state.

Architecture (channels per level; two 3x3x3 convolutions + SiLU per block):
  64^3: 16 -> 16 -> 16      (input: 7 features padded to 16)
  32^3: 16 -> 32 -> 32      (2x2x2 average pooling between levels)
  16^3: 32 -> 64 -> 64
   8^3: 64 -> 96 -> 96
  up (nearest x2) + skip concatenation: 96+64 -> 64 -> 64, 64+32 -> 32 -> 32,
  32+16 -> 16 -> 16; head 16 -> 16 (linear, FP32; the first 4 are the fields)
about 1.16 M parameters.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import lbmx

_vp = ctypes.c_void_p
_i32, _i64, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
_NN = None

NFEAT = 16       # padded input channels
NOUT = 4         # u, v, w, theta
LOG_RA_MID, LOG_RA_HALF = 4.5, 1.5  # log10 Ra in [3, 6] -> [-1, 1]


def nn():
    global _NN
    if _NN is None:
        L = lbmx.load()
        sig = {
            "lbmx_nn_conv3d_fwd": [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _vp],
            "lbmx_nn_conv3d_flip": [_vp, _vp, _i32, _i32, _vp],
            "lbmx_nn_conv3d_wgrad": [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp],
            "lbmx_nn_silu": [_vp, _vp, _i64, _vp],
            "lbmx_nn_silu_bwd": [_vp, _vp, _vp, _i64, _vp],
            "lbmx_nn_pool2": [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp],
            "lbmx_nn_up2": [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp],
            "lbmx_nn_concat": [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _vp],
            "lbmx_nn_mse": [_vp, _vp, _vp, _vp, _i32, _i64, _i32, _i32, _vp],
            "lbmx_nn_adam": [_vp, _vp, _vp, _vp, _vp, _i64, _f32, _f32, _f32, _f32, _i64, _f32, _vp],
            "lbmx_nn_to_bf16": [_vp, _vp, _i64, _vp],
            "lbmx_nn_make_input": [_vp, _vp, _i32, _i32, _vp],
            "lbmx_nn_add": [_vp, _vp, _vp, _i64, _vp],
            "lbmx_nn_layout": [_vp, _vp, _i32, _i64, _i32, _i32, _i32, _vp, _vp],
            "lbmx_nn_layout_flip": [_vp, _vp, _i32, _i32, _i32, _i32, _i32,
                                    ctypes.POINTER(ctypes.c_float), _vp, _vp],
            "lbmx_nn_conv3d_fwd_ep": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32,
                                      _i32, _i32, _i32, _vp],
            "lbmx_nn_upcat": [_vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp],
            "lbmx_nn_conv3d_fwd_upcat": [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32,
                                         _i32, _i32, _i32, _vp],
            "lbmx_nn_conv3d_wgrad_upcat": [_vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32,
                                           _i32, _i32, _i32, _vp],
            "lbmx_nn_conv3d_mse": [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _i32, _i32,
                                   _i32, _i32, _i32, _i32, _vp],
            "lbmx_nn_adam_flip": [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _f32, _f32, _f32, _f32, _i64,
                                  _f32, _i32, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  _vp],
            "lbmx_nn_pool2_bwd_gate": [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _vp],
            "lbmx_nn_up2_bwd_gate": [_vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _vp],
            "lbmx_nn_conv3d_flip_many": [_vp, _vp, _i32, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), _vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _NN = L
    return _NN


def P(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else _vp(t.data_ptr())


def call(name, *args):
    st = getattr(nn(), name)(*args)
    if st != 0:
        raise lbmx.LbmxError(st, lbmx.load().lbmx_last_error().decode())


def stream_ptr():
    import torch
    return _vp(torch.cuda.current_stream().cuda_stream)


class Conv:
    """3x3x3 convolution with bias: BF16 weights, FP32 master / grads / Adam."""

    def __init__(self, ci, co, rng, act=True):
        import torch

        self.ci, self.co, self.act = ci, co, act
        std = math.sqrt(2.0 / (27 * ci)) if act else math.sqrt(1.0 / (27 * ci))
        w0 = (rng.standard_normal((co, 27, ci)) * std).astype(np.float32)
        dev = "cuda"
        self.w = torch.tensor(w0, device=dev)                         # master FP32
        self.b = torch.zeros(co, dtype=torch.float32, device=dev)
        self.wb = torch.empty((co, 27, ci), dtype=torch.bfloat16, device=dev)
        self.wflip = torch.empty((ci, 27, co), dtype=torch.bfloat16, device=dev)
        self.gw = torch.zeros_like(self.w)
        self.gb = torch.zeros_like(self.b)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.sync_bf16()

    def nparams(self):
        return self.w.numel() + self.b.numel()

    def sync_bf16(self):
        call("lbmx_nn_to_bf16", P(self.w), P(self.wb), self.w.numel(), stream_ptr())
        call("lbmx_nn_conv3d_flip", P(self.wb), P(self.wflip), self.ci, self.co, stream_ptr())

    def adam(self, lr, step, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
        s = stream_ptr()
        call("lbmx_nn_adam", P(self.w), P(self.gw), P(self.mw), P(self.vw), P(self.wb),
             self.w.numel(), lr, b1, b2, eps, step, wd, s)
        call("lbmx_nn_adam", P(self.b), P(self.gb), P(self.mb), P(self.vb), None,
             self.b.numel(), lr, b1, b2, eps, step, 0.0, s)
        call("lbmx_nn_conv3d_flip", P(self.wb), P(self.wflip), self.ci, self.co, s)


class UNet:
    LEVELS = (16, 32, 64, 96)

    def __init__(self, seed=0, m=64):
        rng = np.random.default_rng(seed)
        c0, c1, c2, c3 = self.LEVELS
        self.m = m
        self.enc = [(Conv(NFEAT, c0, rng), Conv(c0, c0, rng)),
                    (Conv(c0, c1, rng), Conv(c1, c1, rng)),
                    (Conv(c1, c2, rng), Conv(c2, c2, rng)),
                    (Conv(c2, c3, rng), Conv(c3, c3, rng))]
        self.dec = [(Conv(c3 + c2, c2, rng), Conv(c2, c2, rng)),
                    (Conv(c2 + c1, c1, rng), Conv(c1, c1, rng)),
                    (Conv(c1 + c0, c0, rng), Conv(c0, c0, rng))]
        self.head = Conv(c0, 16, rng, act=False)
        self.step_count = 0
        self.scale = None  # per-output-channel target scale (device FP32 [4])
        self._flatten()

    def _flatten(self):
        """Put every layer's parameters, gradients, Adam moments and BF16 /
        flipped copies into flat buffers (the layers keep views), so that one
        Adam launch per kind (weights, biases) and one flip launch update the
        whole network."""
        import torch

        convs = self.convs()
        nw = [c.w.numel() for c in convs]
        nb = [c.b.numel() for c in convs]
        ow = np.concatenate([[0], np.cumsum(nw)[:-1]]).astype(np.int64)
        ob = np.concatenate([[0], np.cumsum(nb)[:-1]]).astype(np.int64)
        f32 = dict(dtype=torch.float32, device="cuda")
        bf = dict(dtype=torch.bfloat16, device="cuda")
        W, Bn = int(sum(nw)), int(sum(nb))
        self._fw, self._fgw = torch.empty(W, **f32), torch.zeros(W, **f32)
        self._fmw, self._fvw = torch.zeros(W, **f32), torch.zeros(W, **f32)
        self._fwb, self._fwflip = torch.empty(W, **bf), torch.empty(W, **bf)
        self._fb, self._fgb = torch.empty(Bn, **f32), torch.zeros(Bn, **f32)
        self._fmb, self._fvb = torch.zeros(Bn, **f32), torch.zeros(Bn, **f32)
        for c, o, n, q, m in zip(convs, ow, nw, ob, nb):
            o, n, q, m = int(o), int(n), int(q), int(m)
            self._fw[o:o + n].copy_(c.w.reshape(-1))
            self._fb[q:q + m].copy_(c.b)
            c.w = self._fw[o:o + n].view(c.co, 27, c.ci)
            c.gw = self._fgw[o:o + n].view(c.co, 27, c.ci)
            c.mw, c.vw = self._fmw[o:o + n].view(c.co, 27, c.ci), self._fvw[o:o + n].view(c.co, 27, c.ci)
            c.wb = self._fwb[o:o + n].view(c.co, 27, c.ci)
            c.wflip = self._fwflip[o:o + n].view(c.ci, 27, c.co)
            c.b, c.gb = self._fb[q:q + m], self._fgb[q:q + m]
            c.mb, c.vb = self._fmb[q:q + m], self._fvb[q:q + m]
        k = len(convs)
        self._flip_args = ((ctypes.c_int64 * k)(*ow.tolist()),
                           (ctypes.c_int32 * k)(*[c.ci for c in convs]),
                           (ctypes.c_int32 * k)(*[c.co for c in convs]))
        self._sync_all()

    def _sync_all(self):
        s = stream_ptr()
        call("lbmx_nn_to_bf16", P(self._fw), P(self._fwb), self._fw.numel(), s)
        call("lbmx_nn_conv3d_flip_many", P(self._fwb), P(self._fwflip), len(self.convs()),
             *self._flip_args, s)

    def convs(self):
        out = []
        for a, b in self.enc + self.dec:
            out += [a, b]
        return out + [self.head]

    def nparams(self):
        return sum(c.nparams() for c in self.convs())

    # ---- buffers -------------------------------------------------------------
    @staticmethod
    def _bf(*shape):
        import torch
        return torch.empty(shape, dtype=torch.bfloat16, device="cuda")

    # ---- forward -------------------------------------------------------------
    # fused (default): the convolution kernels also apply SiLU (forward) and
    # its derivative (data gradients), split concatenated gradients, and read
    # a decoder layer's upsampled-and-concatenated input in place; unfused:
    # the separate elementwise kernels (kept to check the fused path against).
    fused = True
    # when a list, forward() and backward() append every convolution's GPU
    # tensors (inputs, outputs, gradients) to it, for per-layer checks
    record = None

    def _conv(self, conv, x, B, r, cache, up=None):
        """conv + SiLU on a [B, r, r, r, ci] BF16 tensor x, or (fused) on the
        concatenation [up2(low) | skip] read in place, up = (low, skip, cu, cs);
        returns the activation."""
        s = stream_ptr()
        z = self._bf(B, r, r, r, conv.co)
        a = self._bf(B, r, r, r, conv.co)
        if up is not None:
            low, skip, cu, cs = up
            call("lbmx_nn_conv3d_fwd_upcat", P(low), P(skip), P(conv.wb), P(conv.b), P(z), P(a),
                 B, r, r, r, cu, cs, conv.co, s)
        elif self.fused:
            call("lbmx_nn_conv3d_fwd_ep", P(x), P(conv.wb), P(conv.b), P(z), P(a), None, None, 0,
                 B, r, r, r, conv.ci, conv.co, s)
        else:
            call("lbmx_nn_conv3d_fwd", P(x), P(conv.wb), P(conv.b), P(z), 0, B, r, r, r, conv.ci,
                 conv.co, s)
            call("lbmx_nn_silu", P(z), P(a), z.numel(), s)
        cache.append({"kind": "conv", "conv": conv, "x": x, "up": up, "z": z, "r": r})
        if self.record is not None:
            self.record.append({"pass": "fwd", "conv": conv, "x": x, "up": up, "z": z, "a": a,
                                "r": r})
        return a

    def forward(self, cond, B, train=False):
        """cond: device FP32 [B, 2] = (normalised log10 Ra, wall type).
        Returns FP32 predictions [B, m^3, 16] (channel-last)."""
        import torch

        s = stream_ptr()
        m = self.m
        cache, h = self._trunk(cond, B)
        pred = torch.empty((B, m ** 3, 16), dtype=torch.float32, device="cuda")
        call("lbmx_nn_conv3d_fwd", P(h), P(self.head.wb), P(self.head.b), P(pred), 1, B, m, m, m,
             self.head.ci, 16, s)
        self._cache = (cache, h, B) if train else None
        return pred

    def forward_loss(self, cond, B, target, partial, pred=None, K=NOUT):
        """Training forward whose head computes the squared-error loss in its
        epilogue (fused; the unfused network runs forward + mse_loss):
        target FP32 [B, m^3, K]; per-block sums of squared errors go to
        partial (device FP64 [1024]); pred (FP32 [B, m^3, 16]) receives the
        prediction if given.  Returns (BF16 gradient [B, m^3, 16] for
        backward(), element count)."""
        import torch

        m = self.m
        if not self.fused:
            p = self.forward(cond, B, train=True)
            if pred is not None:
                pred.copy_(p)
            return mse_loss(p, target, partial, K)
        cache, h = self._trunk(cond, B)
        grad = torch.empty((B, m ** 3, 16), dtype=torch.bfloat16, device="cuda")
        call("lbmx_nn_conv3d_mse", P(h), P(self.head.wb), P(self.head.b), P(target), K, P(grad),
             P(partial), partial.numel(), P(pred), B, m, m, m, self.head.ci, 16, stream_ptr())
        self._cache = (cache, h, B)
        return grad, B * m ** 3 * K

    def _trunk(self, cond, B):
        """Input construction, encoder and decoder; returns (layer cache, last
        activation [B, m, m, m, 16])."""
        s = stream_ptr()
        m = self.m
        cache = []
        x = self._bf(B, m, m, m, NFEAT)
        call("lbmx_nn_make_input", P(cond), P(x), B, m, s)
        skips = []
        r = m
        h = x
        for lvl, (ca, cb) in enumerate(self.enc):
            h = self._conv(ca, h, B, r, cache)
            h = self._conv(cb, h, B, r, cache)
            if lvl < len(self.enc) - 1:
                skips.append((h, r))
                p = self._bf(B, r // 2, r // 2, r // 2, cb.co)
                call("lbmx_nn_pool2", P(h), P(p), B, r, r, r, cb.co, 0, s)
                cache.append({"kind": "pool", "h": h, "r": r})
                h = p
                r //= 2
        for (ca, cb) in self.dec:
            sk, rs = skips.pop()
            cu, cs = h.shape[-1], sk.shape[-1]
            if self.fused:
                r *= 2
                cache.append({"kind": "upcat", "r": r, "cu": cu, "cs": cs})
                h = self._conv(ca, None, B, r, cache, up=(h, sk, cu, cs))
            else:
                cat = self._bf(B, 2 * r, 2 * r, 2 * r, cu + cs)
                u = self._bf(B, 2 * r, 2 * r, 2 * r, cu)
                call("lbmx_nn_up2", P(h), P(u), B, r, r, r, cu, 0, s)
                call("lbmx_nn_concat", P(u), P(sk), P(cat), B * (2 * r) ** 3, cu, cs, 0, s)
                r *= 2
                cache.append({"kind": "upcat", "r": r, "cu": cu, "cs": cs})
                h = self._conv(ca, cat, B, r, cache)
            h = self._conv(cb, h, B, r, cache)
        return cache, h

    # ---- backward ------------------------------------------------------------
    def backward(self, gpred):
        """gpred: BF16 [B, m^3, 16] gradient of the loss w.r.t. the predictions."""
        if self.fused:
            self._backward_fused(gpred)
        else:
            self._backward_unfused(gpred)
        self._cache = None

    def _backward_fused(self, gpred):
        """Walks the layers backwards carrying dL/dz of the next convolution
        to differentiate: every data gradient comes out of the convolution
        kernel already multiplied by the SiLU derivative of the layer before
        (or split into the upsampled and skip parts of a concatenated input),
        the pooling and upsampling gradients fold in the skip gradient and
        the SiLU derivative, and the first layer's data gradient (w.r.t. the
        network input) is not computed."""
        s = stream_ptr()
        cache, hlast, B = self._cache
        m = self.m
        call("lbmx_nn_conv3d_wgrad", P(hlast), P(gpred), P(self.head.gw), P(self.head.gb), B, m,
             m, m, self.head.ci, 16, s)
        last = cache[-1]
        g = self._bf(B, m, m, m, self.head.ci)
        call("lbmx_nn_conv3d_fwd_ep", P(gpred), P(self.head.wflip), None, P(g), None, P(last["z"]),
             None, 0, B, m, m, m, 16, self.head.ci, s)
        skip_grads = []
        for i in range(len(cache) - 1, -1, -1):
            it = cache[i]
            if it["kind"] == "conv":
                conv, x, r = it["conv"], it["x"], it["r"]
                if it["up"] is not None:
                    low, skip, cu, cs = it["up"]
                    call("lbmx_nn_conv3d_wgrad_upcat", P(low), P(skip), P(g), P(conv.gw),
                         P(conv.gb), B, r, r, r, cu, cs, conv.co, s)
                else:
                    call("lbmx_nn_conv3d_wgrad", P(x), P(g), P(conv.gw), P(conv.gb), B, r, r, r,
                         conv.ci, conv.co, s)
                rec = {"pass": "bwd", "conv": conv, "x": x, "up": it["up"], "gz": g, "r": r}
                prev = cache[i - 1] if i > 0 else None
                if prev is None:
                    rec["dgrad"] = None
                elif prev["kind"] == "conv":
                    gn = self._bf(B, r, r, r, conv.ci)
                    call("lbmx_nn_conv3d_fwd_ep", P(g), P(conv.wflip), None, P(gn), None,
                         P(prev["z"]), None, 0, B, r, r, r, conv.co, conv.ci, s)
                    rec["dgrad"], rec["gate"] = gn, prev["z"]
                    g = gn
                elif prev["kind"] == "pool":
                    gn = self._bf(B, r, r, r, conv.ci)
                    call("lbmx_nn_conv3d_fwd", P(g), P(conv.wflip), None, P(gn), 0, B, r, r, r,
                         conv.co, conv.ci, s)
                    rec["dgrad"] = gn
                    g = gn
                else:  # upcat: split the concatenated input's gradient
                    cu, cs = prev["cu"], prev["cs"]
                    gu = self._bf(B, r, r, r, cu)
                    gs = self._bf(B, r, r, r, cs)
                    call("lbmx_nn_conv3d_fwd_ep", P(g), P(conv.wflip), None, P(gu), None, None,
                         P(gs), cu, B, r, r, r, conv.co, conv.ci, s)
                    rec["dgrad"], rec["dgrad2"] = gu, gs
                    skip_grads.append(gs)
                    g = gu
                if self.record is not None:
                    self.record.append(rec)
            elif it["kind"] == "pool":
                h, r = it["h"], it["r"]
                before = cache[i - 1]  # the convolution whose activation was pooled
                gn = self._bf(B, r, r, r, h.shape[-1])
                call("lbmx_nn_pool2_bwd_gate", P(g), P(skip_grads.pop()), P(before["z"]), P(gn),
                     B, r, r, r, h.shape[-1], s)
                g = gn
            else:  # upcat
                r, cu = it["r"], it["cu"]
                before = cache[i - 1]  # the convolution whose activation was upsampled
                gn = self._bf(B, r // 2, r // 2, r // 2, cu)
                call("lbmx_nn_up2_bwd_gate", P(g), P(before["z"]), P(gn), B, r // 2, r // 2,
                     r // 2, cu, s)
                g = gn

    def _conv_bwd(self, conv, x, z, r, B, ga):
        s = stream_ptr()
        gz = self._bf(B, r, r, r, conv.co)
        call("lbmx_nn_silu_bwd", P(z), P(ga), P(gz), z.numel(), s)
        call("lbmx_nn_conv3d_wgrad", P(x), P(gz), P(conv.gw), P(conv.gb), B, r, r, r, conv.ci,
             conv.co, s)
        gx = self._bf(B, r, r, r, conv.ci)
        call("lbmx_nn_conv3d_fwd", P(gz), P(conv.wflip), None, P(gx), 0, B, r, r, r, conv.co,
             conv.ci, s)
        return gx

    def _backward_unfused(self, gpred):
        s = stream_ptr()
        cache, hlast, B = self._cache
        m = self.m
        call("lbmx_nn_conv3d_wgrad", P(hlast), P(gpred), P(self.head.gw), P(self.head.gb), B, m,
             m, m, self.head.ci, 16, s)
        g = self._bf(B, m, m, m, self.head.ci)
        call("lbmx_nn_conv3d_fwd", P(gpred), P(self.head.wflip), None, P(g), 0, B, m, m, m, 16,
             self.head.ci, s)
        skip_grads = []   # gradients reaching the skip tensors, deepest first
        for item in reversed(cache):
            if item["kind"] == "conv":
                g = self._conv_bwd(item["conv"], item["x"], item["z"], item["r"], B, g)
            elif item["kind"] == "upcat":
                r, cu, cs = item["r"], item["cu"], item["cs"]
                gu = self._bf(B, r, r, r, cu)
                gs = self._bf(B, r, r, r, cs)
                call("lbmx_nn_concat", P(gu), P(gs), P(g), B * r ** 3, cu, cs, 1, s)
                skip_grads.append(gs)
                g = self._bf(B, r // 2, r // 2, r // 2, cu)
                call("lbmx_nn_up2", P(gu), P(g), B, r // 2, r // 2, r // 2, cu, 1, s)
            else:  # pool
                h, r = item["h"], item["r"]
                gh = self._bf(B, r, r, r, h.shape[-1])
                call("lbmx_nn_pool2", P(g), P(gh), B, r, r, r, h.shape[-1], 1, s)
                gsk = skip_grads.pop()
                call("lbmx_nn_add", P(gh), P(gsk), P(gh), gh.numel(), s)
                g = gh

    def adam(self, lr, wd=0.0, b1=0.9, b2=0.999, eps=1e-8):
        """One Adam step on every layer (as Conv.adam per layer, in two
        launches over the flat buffers: the weights, with their BF16 and
        flipped BF16 copies, and the biases)."""
        self.step_count += 1
        s = stream_ptr()
        call("lbmx_nn_adam_flip", P(self._fw), P(self._fgw), P(self._fmw), P(self._fvw),
             P(self._fwb), P(self._fwflip), self._fw.numel(), lr, b1, b2, eps, self.step_count, wd,
             len(self.convs()), *self._flip_args, s)
        call("lbmx_nn_adam", P(self._fb), P(self._fgb), P(self._fmb), P(self._fvb), None,
             self._fb.numel(), lr, b1, b2, eps, self.step_count, 0.0, s)

    # ---- persistence -----------------------------------------------------------
    def state(self):
        d = {}
        for k, c in enumerate(self.convs()):
            d[f"w{k}"] = c.w.cpu().numpy()
            d[f"b{k}"] = c.b.cpu().numpy()
        if self.scale is not None:
            d["scale"] = self.scale.cpu().numpy()
        return d

    def load_state(self, d):
        import torch
        for k, c in enumerate(self.convs()):
            c.w.copy_(torch.tensor(d[f"w{k}"]))
            c.b.copy_(torch.tensor(d[f"b{k}"]))
        self._sync_all()
        if "scale" in d:
            self.scale = torch.tensor(np.asarray(d["scale"], np.float32), device="cuda")


def cond_tensor(log10_ra, wall_type):
    """Device FP32 [B, 2] conditioning: ((log10 Ra - 4.5)/1.5, wall type)."""
    import torch
    lr = (np.asarray(log10_ra, np.float64) - LOG_RA_MID) / LOG_RA_HALF
    c = np.stack([lr, np.asarray(wall_type, np.float64)], axis=1).astype(np.float32)
    return torch.tensor(c, device="cuda")


def mse_loss(pred, target_cl, partial, K=NOUT):
    """BF16 gradient of the squared error of pred [B, V, 16] (FP32) against
    target [B, V, K] (FP32); per-block partial sums go to `partial` (device
    FP64 [1024]).  Returns (gradient, element count)."""
    import torch
    nv = pred.shape[0] * pred.shape[1]
    grad = torch.empty(pred.shape, dtype=torch.bfloat16, device="cuda")
    call("lbmx_nn_mse", P(pred), P(target_cl), P(grad), P(partial), 1024, nv, pred.shape[2], K,
         stream_ptr())
    return grad, nv * K


# The cavity's symmetries (Sec. 2) acting on the fields (u, v, w, theta) of
# a node-centred m^3 grid [z][y][x]: (axis flips for lbmx_nn_layout_flip,
# per-channel signs).  The walls and gravity are symmetric under the
# spanwise mirror x -> H - x (u odd); the inversion about the centre
# exchanges the hot and cold walls (theta_h = -theta_c), reverses gravity's
# axis and maps each linear wall profile (Eqs. 9-10) to minus itself, so u
# and theta are odd under it.  Together with the identity and their product
# they form the group the training augmentation draws from.
SYMMETRIES = (
    (0, (1.0, 1.0, 1.0, 1.0)),      # identity
    (1, (-1.0, 1.0, 1.0, 1.0)),     # x mirror
    (7, (-1.0, -1.0, -1.0, -1.0)),  # inversion about the centre
    (6, (1.0, -1.0, -1.0, -1.0)),   # both
)


def transform_fields(f, g):
    """Symmetry g of SYMMETRIES applied to host fields [..., 4, m, m, m]
    (z, y, x): the reference for the device gather and the dataset check."""
    flip, signs = SYMMETRIES[g]
    out = np.asarray(f)
    for bit, ax in ((1, -1), (2, -2), (4, -3)):
        if flip & bit:
            out = np.flip(out, axis=ax)
    return out * np.array(signs).reshape((4, 1, 1, 1))


def field_asymmetry(fields):
    """max |T f - f| / max |f| over the set (fields [N, 4, m, m, m]) for each
    non-identity symmetry T: how far the steady fields already are
    symmetric (the augmentation adds information only where they are not)."""
    top = float(np.abs(fields).max()) or 1.0
    return {g: float(np.abs(transform_fields(fields, g) - fields).max()) / top
            for g in range(1, len(SYMMETRIES))}


def train(net, fields, log10_ra, wall_type, epochs=300, batch=4, lr=1e-3, seed=0, log=None,
          warmup=None, augment=True):
    """Fit the network to steady fields [N, 4, m, m, m] (channel-first FP32;
    velocities already divided by u_c).  Per-channel target scales are the
    fields' standard deviations; the learning rate rises linearly over
    `warmup` steps (default 5 % of the run, at least 10) and then follows a
    cosine decay.  With augment, every sample of every step is transformed by
    a symmetry drawn uniformly from SYMMETRIES while it is gathered into the
    target (lbmx_nn_layout_flip), the condition (Ra, wall type) unchanged."""
    import time

    import torch

    N = fields.shape[0]
    m = net.m
    V = m ** 3
    std = fields.reshape(N, NOUT, -1).std(axis=(0, 2)).astype(np.float32)
    std = np.maximum(std, 1e-3)
    net.scale = torch.tensor(std, device="cuda")
    inv = torch.tensor(1.0 / std, device="cuda")
    dev_fields = torch.tensor(np.ascontiguousarray(fields.reshape(N, NOUT, V), np.float32),
                              device="cuda")
    sample_bytes = NOUT * V * 4
    target = torch.empty((batch, V, NOUT), dtype=torch.float32, device="cuda")
    per_epoch = N // batch
    partials = torch.zeros((per_epoch, 1024), dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(seed)
    arng = np.random.default_rng(seed + 1)  # symmetry draws
    sym = [(flip, (ctypes.c_float * NOUT)(*signs)) for flip, signs in SYMMETRIES]
    nsteps = epochs * per_epoch
    if warmup is None:
        warmup = max(10, nsteps // 20)
    hist = []
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        order = rng.permutation(N)
        for k in range(per_epoch):
            idx = order[k * batch:(k + 1) * batch]
            for j, i in enumerate(idx):
                flip, signs = sym[int(arng.integers(len(sym)))] if augment else sym[0]
                call("lbmx_nn_layout_flip", _vp(dev_fields.data_ptr() + int(i) * sample_bytes),
                     _vp(target.data_ptr() + j * sample_bytes), 1, m, NOUT, NOUT, flip, signs,
                     P(inv), stream_ptr())
            cond = cond_tensor(log10_ra[idx], wall_type[idx])
            grad, cnt = net.forward_loss(cond, batch, target, partials[k])
            net.backward(grad)
            if step < warmup:
                lr_t = lr * (step + 1) / warmup
            else:
                lr_t = lr * 0.5 * (1 + math.cos(math.pi * (step - warmup) / max(nsteps - warmup, 1)))
            net.adam(lr_t)
            step += 1
        hist.append(float(partials.cpu().numpy().sum()) / (cnt * per_epoch))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep} loss {hist[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return {"loss": hist, "seconds": time.perf_counter() - t0, "steps": step}


def predict_fields(net, log10_ra, wall_type, u_c=1.0):
    """Predicted fields on the m^3 grid, device FP32 [4, m^3]: u, v, w
    multiplied by u_c (u_c = 1 gives u/u_c; the cavity's u_c gives lattice
    units) and theta."""
    import torch
    m = net.m
    cond = cond_tensor([log10_ra], [wall_type])
    pred = net.forward(cond, 1)
    sc = torch.tensor(net.scale.cpu().numpy() * np.array([u_c, u_c, u_c, 1.0], np.float32),
                      device="cuda")
    out = torch.empty((NOUT, m ** 3), dtype=torch.float32, device="cuda")
    call("lbmx_nn_layout", P(pred), P(out), 1, m ** 3, NOUT, 16, 0, P(sc), stream_ptr())
    torch.cuda.current_stream().synchronize()
    return out


def conv_layers(m=64):
    """(ci, co, resolution, upsampled input channels) of every convolution of
    the network, in forward order, the head last."""
    c0, c1, c2, c3 = UNet.LEVELS
    return [(NFEAT, c0, m, 0), (c0, c0, m, 0), (c0, c1, m // 2, 0), (c1, c1, m // 2, 0),
            (c1, c2, m // 4, 0), (c2, c2, m // 4, 0), (c2, c3, m // 8, 0), (c3, c3, m // 8, 0),
            (c3 + c2, c2, m // 4, c3), (c2, c2, m // 4, 0), (c2 + c1, c1, m // 2, c2),
            (c1, c1, m // 2, 0), (c1 + c0, c0, m, c1), (c0, c0, m, 0), (c0, 16, m, 0)]


def conv_floor(batch=4, m=64, hbm_bps=8e12, mfma_flops=2.5e15):
    """FLOPs of one training step's convolutions and the floor of their time:
    per launch (forward and weight gradient of every layer, data gradient of
    all but the first) the larger of its HBM time (BF16 activations read once
    and written once: the forward reads its input and writes z and SiLU(z),
    the weight gradient reads input and output gradient, the data gradient
    reads the output gradient and the gating pre-activation and writes the
    input gradient; the head reads its FP32 targets and writes its BF16 loss
    gradient) and its MFMA time at the dense BF16 peak.  Returns (flop,
    floor_s, hbm_only_s, mfma_only_s)."""
    flop_tot = floor = hbm = mf = 0.0
    layers = conv_layers(m)
    for k, (ci, co, r, cu) in enumerate(layers):
        v = batch * r ** 3
        fl = 2.0 * 27 * ci * co * v
        inb = 2.0 * (v // 8 * cu + v * (ci - cu))
        if k == len(layers) - 1:  # head: loss in the epilogue, no SiLU
            launches = [2.0 * v * ci + 4.0 * v * NOUT + 2.0 * v * co, inb + 2.0 * v * co,
                        2.0 * v * co + 4.0 * v * ci]
        else:
            launches = [inb + 4.0 * v * co, inb + 2.0 * v * co]
            if k > 0:
                launches.append(2.0 * v * co + 4.0 * v * ci)
        for b in launches:
            flop_tot += fl
            floor += max(b / hbm_bps, fl / mfma_flops)
            hbm += b / hbm_bps
            mf += fl / mfma_flops
    return flop_tot, floor, hbm, mf


def bench_step(batch=4, m=64, steps=20, warmup=3, fused=True):
    """Time one training step (forward, loss, backward, Adam) of the U-Net at
    `batch` x m^3 on synthetic targets (seeded smooth fields); returns the
    mean milliseconds per step (HIP events on torch's current stream)."""
    import torch

    net = UNet(seed=0, m=m)
    net.fused = fused
    V = m ** 3
    ax = (np.arange(m) + 0.5) / m
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    fields = np.stack([np.sin(np.pi * yy) * np.cos(np.pi * zz), np.cos(np.pi * xx) * yy,
                       np.sin(2 * np.pi * yy) * zz, 0.5 - yy], axis=-1).reshape(V, NOUT)
    target = torch.tensor(np.broadcast_to(fields, (batch, V, NOUT)).astype(np.float32),
                          device="cuda")
    cond = cond_tensor(np.linspace(3.5, 5.5, batch), (np.arange(batch) % 3) + 1)
    partial = torch.zeros(1024, dtype=torch.float64, device="cuda")

    def one():
        grad, _ = net.forward_loss(cond, batch, target, partial)
        net.backward(grad)
        net.adam(1e-4)

    for _ in range(warmup):
        one()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        one()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / steps


if __name__ == "__main__":
    import json
    import sys

    if "--bench-step" in sys.argv:
        only = "--fused-only" in sys.argv
        out = {"workload": "U-Net training step, batch 4, 64^3, BF16 MFMA",
               "fused_ms": round(bench_step(fused=True), 4)}
        if not only:
            out["unfused_ms"] = round(bench_step(fused=False), 4)
        print(json.dumps(out), flush=True)
