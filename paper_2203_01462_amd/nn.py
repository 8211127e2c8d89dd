"""Surrogate network on the library's BF16 matrix-core kernels (include/fdtd_nn.h).

A U-Net maps a design density (one 2D design box, side divisible by 8) to two
outputs: the objective F and the sensitivity map dF/drho of eq. (27).  Four
levels with 32-64-128-256 channels, two 3x3 convolutions + ReLU per level,
2x2 average pooling on the way down, nearest 2x upsampling and skip
concatenation on the way up, a 3x3 convolution to one channel for the
sensitivity head and global average pooling + a linear layer on the deepest
level for the scalar head.  Weights and activations are BF16, accumulation and
the gradients FP32, the optimizer Adam on FP32 master weights.

Every layer, its backward and the optimizer step run in the HIP library; this
module allocates the buffers (torch device tensors), lays out the parameters
in one flat array and calls the kernels in order on one stream.  Activations
are channel-major [C][N][H][W], so a skip concatenation is a pair of writes
into one buffer.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from .fdtd import FDTDError, load_library

CHANNELS = (32, 64, 128, 256)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(rc):
    if rc:
        raise FDTDError(rc, load_library().fdtd_nn_last_error().decode())


def _s(stream):
    return C.c_void_p(stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream)


def _u16(t):
    if t.dtype != torch.int16 and t.dtype != torch.uint16:
        raise TypeError("BF16 tensors are stored as int16 bit patterns")
    return t


# ---- single-kernel wrappers (device tensors; BF16 as int16 bit patterns) ----

def conv3x3(x, wt, bias, n, cin, cout, h, w, z=None, a=None, stream=None):
    _check(load_library().fdtd_nn_conv3x3(n, cin, cout, h, w, _p(_u16(x)), _p(_u16(wt)), _p(bias), _p(z), _p(a),
                                          _s(stream)))


def _u16n(t):
    return None if t is None else _u16(t)


def conv3x3_dgrad(dz, wt, wrot, dx, n, cin, cout, h, w, stream=None):
    """wt None: wrot already holds the turned weights (rot_weights)."""
    _check(load_library().fdtd_nn_conv3x3_dgrad(n, cin, cout, h, w, _p(_u16(dz)), _p(_u16n(wt)), _p(_u16(wrot)),
                                                _p(dx), _s(stream)))


def conv3x3_dgrad_relu(dz, wt, wrot, a, dza, n, cin, cout, h, w, stream=None):
    """The data gradient with the ReLU backward of the layer below fused in:
    dza = bf16(dx * (a > 0)), a the BF16 activation that is this layer's input."""
    _check(load_library().fdtd_nn_conv3x3_dgrad_relu(n, cin, cout, h, w, _p(_u16(dz)), _p(_u16n(wt)), _p(_u16(wrot)),
                                                     _p(_u16(a)), _p(_u16(dza)), _s(stream)))


def rot_weights(layers, w, wrot, stream=None):
    """Turned weights of every (cin, cout, offset) layer of the flat BF16
    array w into wrot at the same offsets, in one launch."""
    k = len(layers)
    cin = (C.c_int32 * k)(*[ci for ci, _, _ in layers])
    cout = (C.c_int32 * k)(*[co for _, co, _ in layers])
    off = (C.c_int64 * k)(*[o for _, _, o in layers])
    _check(load_library().fdtd_nn_rot_weights(k, cin, cout, off, _p(_u16(w)), _p(_u16(wrot)), _s(stream)))


def wgrad_work(n, cin, cout, h, w):
    return int(load_library().fdtd_nn_wgrad_work(n, cin, cout, h, w))


def conv3x3_wgrad(x, dz, dw, db, work, n, cin, cout, h, w, stream=None):
    _check(load_library().fdtd_nn_conv3x3_wgrad(n, cin, cout, h, w, _p(_u16(x)), _p(_u16(dz)), _p(dw), _p(db),
                                                _p(work), _s(stream)))


def conv3x3_wgrad_noalloc(x, dz, dw, db, n, cin, cout, h, w, stream=None):
    """conv3x3_wgrad with the partial sums in the library's static per-device
    scratch instead of a workspace (for callers that cannot allocate)."""
    _check(load_library().fdtd_nn_conv3x3_wgrad_noalloc(n, cin, cout, h, w, _p(_u16(x)), _p(_u16(dz)), _p(dw),
                                                        _p(db), _s(stream)))


def relu_bf16(z, a, stream=None):
    _check(load_library().fdtd_nn_relu_bf16(z.numel(), _p(z), _p(_u16(a)), _s(stream)))


def relu_bf16_backward(a, da, dz, stream=None):
    _check(load_library().fdtd_nn_relu_bf16_backward(a.numel(), _p(_u16(a)), _p(da), _p(_u16(dz)), _s(stream)))


def to_bf16(x, y=None, stream=None):
    y = torch.empty(x.shape, dtype=torch.int16, device=x.device) if y is None else y
    _check(load_library().fdtd_nn_to_bf16(x.numel(), _p(x), _p(_u16(y)), _s(stream)))
    return y


def from_bf16(x, y=None, stream=None):
    y = torch.empty(x.shape, dtype=torch.float32, device=x.device) if y is None else y
    _check(load_library().fdtd_nn_from_bf16(x.numel(), _p(_u16(x)), _p(y), _s(stream)))
    return y


def pool2(x, y, planes, h, w, stream=None):
    _check(load_library().fdtd_nn_pool2(planes, h, w, _p(_u16(x)), _p(_u16(y)), _s(stream)))


def pool2_backward(dy, dx, planes, h, w, stream=None):
    _check(load_library().fdtd_nn_pool2_backward(planes, h, w, _p(dy), _p(dx), _s(stream)))


def up2(x, y, planes, h, w, stream=None):
    _check(load_library().fdtd_nn_up2(planes, h, w, _p(_u16(x)), _p(_u16(y)), _s(stream)))


def up2_backward(dy, dx, planes, h, w, stream=None):
    _check(load_library().fdtd_nn_up2_backward(planes, h, w, _p(dy), _p(dx), _s(stream)))


def adam(p, m, v, g, pb, lr, t, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load_library().fdtd_nn_adam(p.numel(), _p(p), _p(m), _p(v), _p(g), _p(pb), float(lr), float(beta1),
                                       float(beta2), float(eps), int(t), _s(stream)))


def axpy(a, x, y, stream=None):
    _check(load_library().fdtd_nn_axpy(x.numel(), float(a), _p(x), _p(y), _s(stream)))


def gap_linear(a, wl, bl, out, n, c, hw, stream=None):
    _check(load_library().fdtd_nn_gap_linear(n, c, hw, _p(_u16(a)), _p(wl), _p(bl), _p(out), _s(stream)))


def gap_linear_backward(a, wl, dout, da, dwl, dbl, n, c, hw, stream=None):
    _check(load_library().fdtd_nn_gap_linear_backward(n, c, hw, _p(_u16(a)), _p(wl), _p(dout), _p(da), _p(dwl),
                                                      _p(dbl), _s(stream)))


def mse_work(count):
    return int(load_library().fdtd_nn_mse_work(count))


def mse(pred, target, scale, grad, work, out, stream=None):
    """out[0] (device FP64) = sum (pred - target)^2; grad = 2 scale (pred - target)."""
    _check(load_library().fdtd_nn_mse(pred.numel(), _p(pred), _p(target), float(scale), _p(grad), _p(work), _p(out),
                                      _s(stream)))


# ---- the U-Net ----

def layer_plan(channels=CHANNELS):
    """(cin, cout, level) of every 3x3 convolution in execution order.
    Encoder level l: (prev -> c_l, c_l -> c_l); decoder level l (from the
    bottom up): (c_{l+1} + c_l -> c_l, c_l -> c_l); head: c_0 -> 1."""
    plan, prev = [], 1
    for lvl, c in enumerate(channels):
        plan += [(prev, c, lvl), (c, c, lvl)]
        prev = c
    for lvl in range(len(channels) - 2, -1, -1):
        plan += [(channels[lvl + 1] + channels[lvl], channels[lvl], lvl), (channels[lvl], channels[lvl], lvl)]
    plan.append((channels[0], 1, 0))
    return plan


class UNet:
    """Parameters, Adam state and the activation/gradient buffers for one
    batch size and input side.  ``forward`` returns (F_hat [n], S_hat [n][side][side]);
    ``backward`` takes dL/dF_hat, dL/dS_hat and fills the flat gradient."""

    def __init__(self, side, batch, channels=CHANNELS, seed=0, device="cuda", stream=None):
        if side % (1 << (len(channels) - 1)):
            raise ValueError("side must be divisible by 2^(levels-1)")
        self.side, self.batch, self.ch = side, batch, tuple(channels)
        self.dev = torch.device(device)
        self.stream = stream
        self.plan = layer_plan(channels)
        # flat parameter layout: per conv w [cout][3][3][cin] (starting at a
        # multiple of 8 elements: 16-byte aligned BF16 rows) then b [cout];
        # then the linear head
        offs, o = [], 0
        for cin, cout, _ in self.plan:
            o = (o + 7) // 8 * 8
            offs.append((o, o + cout * cin * 9))
            o += cout * cin * 9 + cout
        self.lin_off = o
        o += channels[-1] + 1
        self.n_params = o
        self.offs = offs
        g = torch.Generator().manual_seed(seed)
        p = torch.zeros(o, dtype=torch.float32)
        for (cin, cout, _), (ow, ob) in zip(self.plan, offs):
            std = math.sqrt(2.0 / (cin * 9))  # He init for ReLU
            p[ow:ow + cout * cin * 9] = torch.randn(cout * cin * 9, generator=g) * std
        p[self.lin_off:self.lin_off + channels[-1]] = torch.randn(channels[-1], generator=g) / math.sqrt(channels[-1])
        # the sensitivity head starts small so early training is stable
        ow, ob = offs[-1]
        p[ow:ob] *= 0.1
        self.p = p.to(self.dev)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.zeros_like(self.p)
        self.pb = to_bf16(self.p, stream=self.stream)
        # every conv layer's turned weights for the data gradients, at the
        # layer's own offset; refreshed in one launch at the first backward
        # after the BF16 weights change
        self.wrot = torch.empty_like(self.pb)
        self._rot_ok = False
        self.t = 0
        self._alloc(batch)

    # parameter views
    def w(self, i):
        ow, ob = self.offs[i]
        return self.pb[ow:ob]

    def b(self, i):
        ow, ob = self.offs[i]
        return self.p[ob:ob + self.plan[i][1]]

    def wrot_of(self, i):
        ow, ob = self.offs[i]
        return self.wrot[ow:ob]

    def dw(self, i):
        ow, ob = self.offs[i]
        return self.g[ow:ob]

    def db(self, i):
        ow, ob = self.offs[i]
        return self.g[ob:ob + self.plan[i][1]]

    def _alloc(self, n):
        d, ch, s = self.dev, self.ch, self.side
        L = len(ch)
        sz = [s >> l for l in range(L)]
        bf = dict(dtype=torch.int16, device=d)
        f32 = dict(dtype=torch.float32, device=d)
        self.x0 = torch.empty(n * s * s, **bf)
        # encoder: first conv output e1[l]; second conv output lands in the
        # skip half of the decoder concat buffer cat[l] (or bottom[L-1])
        self.e1 = [torch.empty(ch[l] * n * sz[l] ** 2, **bf) for l in range(L)]
        self.cat = [torch.empty((ch[l + 1] + ch[l]) * n * sz[l] ** 2, **bf) for l in range(L - 1)]
        self.bottom = torch.empty(ch[-1] * n * sz[-1] ** 2, **bf)
        self.pooled = [torch.empty(ch[l] * n * sz[l + 1] ** 2, **bf) for l in range(L - 1)]
        self.d1 = [torch.empty(ch[l] * n * sz[l] ** 2, **bf) for l in range(L - 1)]
        self.d2 = [torch.empty(ch[l] * n * sz[l] ** 2, **bf) for l in range(L - 1)]
        self.S = torch.empty(n * s * s, **f32)
        self.F = torch.empty(n, **f32)
        # backward buffers: FP32 gradients of activations, BF16 gradients of pre-activations
        big = max(c * n * sz[l] ** 2 for l, c in enumerate(ch))
        self.ga = torch.empty(big, **f32)
        self.gb = torch.empty(big, **f32)
        # gradient of each decoder concat buffer; its skip half is consumed by the encoder pass
        self.gcat = [torch.empty((ch[l + 1] + ch[l]) * n * sz[l] ** 2, **f32) for l in range(L - 1)]
        self.gz = torch.empty(max(big, n * s * s), **bf)
        # BF16 pre-activation gradient written by a data gradient with the
        # ReLU backward of the layer below fused in
        self.gz2 = torch.empty(big, **bf)
        self.dF = torch.empty(n, **f32)
        self.dS = torch.empty(n * s * s, **f32)
        self.work = torch.empty(max(wgrad_work(n, ci, co, sz[l], sz[l]) for ci, co, l in self.plan), **f32)
        self.msew = torch.empty(max(mse_work(n * s * s), 1), dtype=torch.float64, device=d)
        self.loss = torch.zeros(2, dtype=torch.float64, device=d)
        self.n = n

    def _skip(self, l):
        """Skip half (second part) of cat[l], or the bottom buffer."""
        ch, n, sz = self.ch, self.n, self.side >> l
        if l == len(ch) - 1:
            return self.bottom
        return self.cat[l][ch[l + 1] * n * sz * sz:]

    def forward(self, rho):
        """rho: device FP32 [n][side][side] (n = the batch the net was built for)."""
        ch, n, s, st = self.ch, self.n, self.side, self.stream
        L = len(ch)
        if rho.numel() != n * s * s or rho.dtype != torch.float32 or not rho.is_cuda:
            raise ValueError(f"rho must be CUDA float32 with {n}x{s}x{s} values")
        to_bf16(rho.reshape(-1), self.x0, stream=st)
        x, li = self.x0, 0
        for l in range(L):
            sz = s >> l
            cin = 1 if l == 0 else ch[l - 1]
            conv3x3(x, self.w(li), self.b(li), n, cin, ch[l], sz, sz, a=self.e1[l], stream=st)
            conv3x3(self.e1[l], self.w(li + 1), self.b(li + 1), n, ch[l], ch[l], sz, sz, a=self._skip(l), stream=st)
            li += 2
            if l < L - 1:
                pool2(self._skip(l), self.pooled[l], ch[l] * n, sz, sz, stream=st)
                x = self.pooled[l]
        gap_linear(self.bottom, self.p[self.lin_off:self.lin_off + ch[-1]], self.p[self.lin_off + ch[-1]:],
                   self.F, n, ch[-1], (s >> (L - 1)) ** 2, stream=st)
        y = self.bottom
        for l in range(L - 2, -1, -1):
            sz = s >> l
            up2(y, self.cat[l][:ch[l + 1] * n * sz * sz], ch[l + 1] * n, sz // 2, sz // 2, stream=st)
            conv3x3(self.cat[l], self.w(li), self.b(li), n, ch[l + 1] + ch[l], ch[l], sz, sz, a=self.d1[l], stream=st)
            conv3x3(self.d1[l], self.w(li + 1), self.b(li + 1), n, ch[l], ch[l], sz, sz, a=self.d2[l], stream=st)
            li += 2
            y = self.d2[l]
        conv3x3(y, self.w(li), self.b(li), n, ch[0], 1, s, s, z=self.S, stream=st)
        return self.F, self.S.view(n, s, s)

    def _conv_back(self, li, x, a_out, ga, gx, h, gz=None, fuse=False):
        """Backward of conv li (input x, BF16 output a_out = relu(z), or the
        head when a_out is None) given the FP32 gradient ga of its output, or
        its BF16 pre-activation gradient gz when the layer above formed it.
        Writes the FP32 input gradient into gx unless gx is None; with fuse
        (x is the ReLU output of the layer below, whose backward comes next)
        writes that layer's BF16 pre-activation gradient into self.gz2 instead
        and returns it."""
        cin, cout, _ = self.plan[li]
        n, st = self.n, self.stream
        cnt = cout * n * h * h
        if gz is None:
            gz = self.gz[:cnt]
            if a_out is None:
                to_bf16(ga[:cnt], gz, stream=st)
            else:
                relu_bf16_backward(a_out, ga[:cnt], gz, stream=st)
        conv3x3_wgrad(x, gz, self.dw(li), self.db(li), self.work, n, cin, cout, h, h, stream=st)
        if fuse:
            out = self.gz2[:cin * n * h * h]
            conv3x3_dgrad_relu(gz, None, self.wrot_of(li), x, out, n, cin, cout, h, h, stream=st)
            return out
        if gx is not None:
            conv3x3_dgrad(gz, None, self.wrot_of(li), gx[:cin * n * h * h], n, cin, cout, h, h, stream=st)
        return None

    def backward(self, dF, dS):
        """dF: device FP32 [n] = dL/dF_hat; dS: device FP32 [n*side*side] = dL/dS_hat."""
        ch, n, s, st = self.ch, self.n, self.side, self.stream
        L = len(ch)
        li = len(self.plan) - 1
        ga, gb = self.ga, self.gb
        if not self._rot_ok:
            rot_weights([(ci, co, ow) for (ci, co, _), (ow, _) in zip(self.plan, self.offs)], self.pb, self.wrot,
                        stream=st)
            self._rot_ok = True
        # sensitivity head and decoder, top down
        self._conv_back(li, self.d2[0], None, dS, ga, s)
        for l in range(L - 1):
            sz = s >> l
            li -= 1
            gz = self._conv_back(li, self.d1[l], self.d2[l], ga, None, sz, fuse=True)
            li -= 1
            self._conv_back(li, self.cat[l], self.d1[l], None, self.gcat[l], sz, gz=gz)
            # up half of the concat gradient -> gradient of the level below's output
            up_cnt = ch[l + 1] * n * sz * sz
            up2_backward(self.gcat[l][:up_cnt], ga[:up_cnt // 4], ch[l + 1] * n, sz // 2, sz // 2, stream=st)
        # ga: gradient of the decoder input at the bottom (= the bottom activation)
        hb = s >> (L - 1)
        cnt = ch[-1] * n * hb * hb
        lo = self.lin_off
        gap_linear_backward(self.bottom, self.p[lo:lo + ch[-1]], dF, gb[:cnt], self.g[lo:lo + ch[-1]],
                            self.g[lo + ch[-1]:lo + ch[-1] + 1], n, ch[-1], hb * hb, stream=st)
        axpy(1.0, gb[:cnt], ga[:cnt], stream=st)
        # encoder, bottom up
        for l in range(L - 1, -1, -1):
            sz = s >> l
            li = 2 * l + 1
            if l < L - 1:
                # ga holds the gradient of pooled[l]; expand it and add the skip gradient
                pool2_backward(ga[:ch[l] * n * (sz // 2) ** 2], gb[:ch[l] * n * sz * sz], ch[l] * n, sz, sz,
                               stream=st)
                up_cnt = ch[l + 1] * n * sz * sz
                axpy(1.0, self.gcat[l][up_cnt:], gb[:ch[l] * n * sz * sz], stream=st)
                ga, gb = gb, ga
            gz = self._conv_back(li, self.e1[l], self._skip(l), ga, None, sz, fuse=True)
            x = self.x0 if l == 0 else self.pooled[l - 1]
            self._conv_back(li - 1, x, self.e1[l], None, None if l == 0 else ga, sz, gz=gz)

    def loss_grad(self, F_t, S_t, wF=1.0, wS=1.0):
        """L = wF mean (F_hat - F_t)^2 + wS mean (S_hat - S_t)^2 on the last
        forward; fills dF, dS and the device pair self.loss = (sum sq F, sum sq S)."""
        n, s, st = self.n, self.side, self.stream
        mse(self.F, F_t, wF / n, self.dF, self.msew, self.loss[0:1], stream=st)
        mse(self.S, S_t.reshape(-1), wS / (n * s * s), self.dS, self.msew, self.loss[1:2], stream=st)
        return self.dF, self.dS

    def step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        adam(self.p, self.m, self.v, self.g, self.pb, lr, self.t, beta1, beta2, eps, stream=self.stream)
        self._rot_ok = False

    def state(self):
        return {"p": self.p.detach().cpu(), "channels": self.ch, "side": self.side}

    def load(self, p):
        self.p.copy_(p.to(self.dev))
        to_bf16(self.p, self.pb, stream=self.stream)
        self._rot_ok = False

