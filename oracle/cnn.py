"""FP64 oracle of the learned segment proposer (test infrastructure only).

The network scores the four children of a quadtree box from the box's 32 x 32
coarse DAS energy image (normalised by its maximum):

    conv3x3(1 -> 32, stride 1) -> ReLU
    3 x [conv3x3(32 -> 32, stride 2) -> ReLU]              32x32 -> 16 -> 8 -> 4
    child c = bx + 2 by: mean over the 2 x 2 cells of quadrant (bx, by)  -> 32 features
    shared linear 32 -> 1 per child                        -> 4 logits -> softmax

All convolutions use zero padding 1.  Training minimises the mean cross-entropy
against the child that contains the full-resolution DMAS maximum.

Written plainly: every convolution is the sum over the nine kernel offsets of a
channel contraction on a shifted, strided view; the backward pass is derived by
hand from the same sums.  The GPU stores weights and activations in BF16 and
accumulates in FP32; ``bf16_round`` lets the tests feed this oracle the same
rounded values.
"""
from __future__ import annotations

import dataclasses

import numpy as np

CH = 32
IN = 32
STRIDES = (1, 2, 2, 2)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    r = ((u + rounding) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


@dataclasses.dataclass
class Params:
    w: list      # 4 conv weights [Cout, Cin, 3, 3]
    b: list      # 4 conv biases [Cout]
    wl: np.ndarray   # readout weight [32]
    bl: float        # readout bias

    def flat(self) -> np.ndarray:
        return np.concatenate([x.ravel() for x in self.w] + [x.ravel() for x in self.b] + [self.wl, [self.bl]])

    @staticmethod
    def shapes():
        ws = [(CH, 1, 3, 3)] + [(CH, CH, 3, 3)] * 3
        return ws, [(CH,)] * 4

    @classmethod
    def from_flat(cls, v: np.ndarray) -> "Params":
        v = np.asarray(v, dtype=np.float64)
        ws, bs = cls.shapes()
        out_w, out_b, k = [], [], 0
        for s in ws:
            n = int(np.prod(s))
            out_w.append(v[k:k + n].reshape(s))
            k += n
        for s in bs:
            out_b.append(v[k:k + s[0]].copy())
            k += s[0]
        wl = v[k:k + CH].copy()
        bl = float(v[k + CH])
        return cls(out_w, out_b, wl, bl)

    @classmethod
    def init(cls, seed: int) -> "Params":
        """He-normal convolutions, zero biases, small readout (the GPU initialiser draws the same numbers
        when given this array)."""
        rng = np.random.default_rng(seed)
        ws, _ = cls.shapes()
        w = [rng.standard_normal(s) * np.sqrt(2.0 / (s[1] * 9)) for s in ws]
        b = [np.zeros(CH) for _ in range(4)]
        wl = rng.standard_normal(CH) * np.sqrt(1.0 / CH)
        return cls(w, b, wl, 0.0)


N_PARAMS = sum(int(np.prod(s)) for s in Params.shapes()[0]) + 4 * CH + CH + 1


def conv_forward(x, w, b, stride):
    """x [N, Cin, H, W], w [Cout, Cin, 3, 3] -> [N, Cout, H/stride, W/stride], zero padding 1."""
    n, cin, h, wd = x.shape
    ho, wo = (h + 2 - 3) // stride + 1, (wd + 2 - 3) // stride + 1
    xp = np.zeros((n, cin, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((n, w.shape[0], ho, wo)) + b[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            view = xp[:, :, ky:ky + stride * (ho - 1) + 1:stride, kx:kx + stride * (wo - 1) + 1:stride]
            out += np.einsum("nchw,oc->nohw", view, w[:, :, ky, kx])
    return out


def conv_backward(x, w, stride, dout):
    """Gradients of conv_forward with respect to x, w, b, given dout."""
    n, cin, h, wd = x.shape
    ho, wo = dout.shape[2], dout.shape[3]
    xp = np.zeros((n, cin, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(None), slice(ky, ky + stride * (ho - 1) + 1, stride),
                  slice(kx, kx + stride * (wo - 1) + 1, stride))
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dout, xp[sl])
            dxp[sl] += np.einsum("nohw,oc->nchw", dout, w[:, :, ky, kx])
    db = dout.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:-1, 1:-1], dw, db


def quadrant_pool(a):
    """a [N, C, 4, 4] -> [N, 4, C]: child c = bx + 2 by averages rows 2by..2by+1, cols 2bx..2bx+1."""
    out = np.zeros((a.shape[0], 4, a.shape[1]))
    for c in range(4):
        bx, by = c & 1, c >> 1
        out[:, c, :] = a[:, :, 2 * by:2 * by + 2, 2 * bx:2 * bx + 2].mean(axis=(2, 3))
    return out


def forward(p: Params, x, act_round=None):
    """x [N, 32, 32] -> (logits [N, 4], cache).  act_round (e.g. bf16_round) is applied to every
    stored activation, as the GPU stores BF16 activations."""
    r = act_round or (lambda v: v)
    a = [r(np.asarray(x, dtype=np.float64)[:, None, :, :])]
    pre = []
    for i in range(4):
        z = conv_forward(a[-1], p.w[i], p.b[i], STRIDES[i])
        pre.append(z)
        a.append(r(np.maximum(z, 0.0)))
    feat = quadrant_pool(a[-1])                  # [N, 4, C]
    logits = feat @ p.wl + p.bl                  # [N, 4]
    return logits, (a, pre, feat)


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(p: Params, x, labels, act_round=None):
    """Mean cross-entropy and its gradient (as a flat vector in Params.flat order)."""
    logits, (a, pre, feat) = forward(p, x, act_round)
    n = logits.shape[0]
    prob = softmax(logits)
    labels = np.asarray(labels, dtype=np.int64)
    loss = float(-np.mean(np.log(prob[np.arange(n), labels])))
    dlog = prob.copy()
    dlog[np.arange(n), labels] -= 1.0
    dlog /= n                                    # [N, 4]
    dwl = np.einsum("nc,nck->k", dlog, feat)
    dbl = float(dlog.sum())
    dfeat = dlog[:, :, None] * p.wl[None, None, :]   # [N, 4, C]
    da = np.zeros_like(a[-1])
    for c in range(4):
        bx, by = c & 1, c >> 1
        da[:, :, 2 * by:2 * by + 2, 2 * bx:2 * bx + 2] += dfeat[:, c, :, None, None] / 4.0
    dw, db = [None] * 4, [None] * 4
    for i in reversed(range(4)):
        dz = da * (pre[i] > 0)
        dx, dw[i], db[i] = conv_backward(a[i], p.w[i], STRIDES[i], dz)
        da = dx
    g = Params(dw, db, dwl, dbl)
    return loss, g.flat(), prob


def macs_per_sample() -> int:
    m, h, cin = 0, IN, 1
    for s in STRIDES:
        ho = h // s
        m += ho * ho * CH * cin * 9
        h, cin = ho, CH
    return m


# ----------------------------------------------------------------------------------
# Adam (Kingma & Ba 2015) on FP32 master weights, the update the GPU applies
# ----------------------------------------------------------------------------------

def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
