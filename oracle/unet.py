"""FP64 reference of the warm-start U-Net: forward, loss and backward.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network is not in the thesis: it is the learned warm start for the
robust inversion of Chapter 4 (a predicted initial Radon model m0 and
initial residual weights w0 for the IRLS outer loop).  This module is its
plain definition, written out with numpy in FP64, and the gradient by hand
(reverse-mode, layer by layer), so the GPU kernels can be checked against it.

Architecture (channels c = base * (1, 2, 4, 8), four levels):

    enc1a: 3x3 conv  Cin -> c1, ReLU          enc1b: c1 -> c1, ReLU
    enc2a: 2x2 mean pool, 3x3 c1 -> c2, ReLU  enc2b: c2 -> c2, ReLU
    enc3a: pool, c2 -> c3, ReLU               enc3b: c3 -> c3, ReLU
    bota:  pool, c3 -> c4, ReLU               botb:  c4 -> c4, ReLU
    dec3a: [nearest 2x upsample(botb), enc3b] c4+c3 -> c3, ReLU;  dec3b: c3 -> c3
    dec2a: [up(dec3b), enc2b] c3+c2 -> c2, ReLU;                   dec2b: c2 -> c2
    dec1a: [up(dec2b), enc1b] c2+c1 -> c1, ReLU;                   dec1b: c1 -> c1
    head_m: 1x1 conv c1 -> P (linear)          -> y_m (predicted model / scale)
    head_w: 1x1 conv c1 -> 1, logistic sigmoid -> y_w (predicted weights)

3x3 convolutions are cross-correlations with zero padding and a bias.
Loss:  mean (y_m - t_m)^2 + lam_w mean (y_w - t_w)^2.

Parameters live in one flat vector, conv by conv in the order above: weight
[co][ci][3][3] (1x1 heads: [co][ci]) then bias [co].
"""
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np


@dataclass(frozen=True)
class UNetSpec:
    cin: int = 1
    pout: int = 32
    base: int = 16

    def convs(self) -> List[Tuple[str, int, int, int]]:
        """(name, c_in, c_out, kernel size) in parameter order."""
        c1, c2, c3, c4 = (self.base * f for f in (1, 2, 4, 8))
        return [
            ("enc1a", self.cin, c1, 3), ("enc1b", c1, c1, 3),
            ("enc2a", c1, c2, 3), ("enc2b", c2, c2, 3),
            ("enc3a", c2, c3, 3), ("enc3b", c3, c3, 3),
            ("bota", c3, c4, 3), ("botb", c4, c4, 3),
            ("dec3a", c4 + c3, c3, 3), ("dec3b", c3, c3, 3),
            ("dec2a", c3 + c2, c2, 3), ("dec2b", c2, c2, 3),
            ("dec1a", c2 + c1, c1, 3), ("dec1b", c1, c1, 3),
            ("head_m", c1, self.pout, 1), ("head_w", c1, 1, 1),
        ]

    def n_params(self) -> int:
        return sum(co * ci * k * k + co for _, ci, co, k in self.convs())


def unpack(spec: UNetSpec, theta: np.ndarray) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
    out, o = {}, 0
    for name, ci, co, k in spec.convs():
        nw = co * ci * k * k
        w = theta[o:o + nw].reshape(co, ci, k, k)
        b = theta[o + nw:o + nw + co]
        out[name] = (w, b)
        o += nw + co
    assert o == theta.size
    return out


def pack(spec: UNetSpec, grads: Dict[str, Tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    return np.concatenate([np.concatenate([grads[n][0].ravel(), grads[n][1].ravel()])
                           for n, _, _, _ in spec.convs()])


def init_params(spec: UNetSpec, rng) -> np.ndarray:
    """He-normal weights (fan-in), zero biases."""
    parts = []
    for _, ci, co, k in spec.convs():
        parts.append(rng.standard_normal(co * ci * k * k) * np.sqrt(2.0 / (ci * k * k)))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


# ------------------------------------------------------------------ layers
# Tensors are [B][C][H][W].

def conv3(x, w, b):
    """Cross-correlation with a 3x3 kernel, zero padding 1, plus bias."""
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    y = np.zeros((B, w.shape[0], H, W))
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oc,bchw->bohw", w[:, :, dy, dx], xp[:, :, dy:dy + H, dx:dx + W])
    return y + b[None, :, None, None]


def conv3_backward(x, w, gy):
    """Gradients of conv3 w.r.t. its input, weight and bias, given dL/dy."""
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            gw[:, :, dy, dx] = np.einsum("bohw,bchw->oc", gy, xp[:, :, dy:dy + H, dx:dx + W])
            gxp[:, :, dy:dy + H, dx:dx + W] += np.einsum("oc,bohw->bchw", w[:, :, dy, dx], gy)
    return gxp[:, :, 1:H + 1, 1:W + 1], gw, gy.sum(axis=(0, 2, 3))


def conv1(x, w, b):
    return np.einsum("oc,bchw->bohw", w[:, :, 0, 0], x) + b[None, :, None, None]


def conv1_backward(x, w, gy):
    gx = np.einsum("oc,bohw->bchw", w[:, :, 0, 0], gy)
    gw = np.einsum("bohw,bchw->oc", gy, x)[:, :, None, None]
    return gx, gw, gy.sum(axis=(0, 2, 3))


def pool2(x):
    B, C, H, W = x.shape
    return x.reshape(B, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def pool2_backward(gy):
    return np.repeat(np.repeat(gy, 2, axis=2), 2, axis=3) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def up2_backward(gy):
    B, C, H, W = gy.shape
    return gy.reshape(B, C, H // 2, 2, W // 2, 2).sum(axis=(3, 5))


def relu(z):
    return np.maximum(z, 0.0)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


# ------------------------------------------------------------------ network
_ENC = [("enc1a", "enc1b", None), ("enc2a", "enc2b", "pool"), ("enc3a", "enc3b", "pool"), ("bota", "botb", "pool")]
_DEC = [("dec3a", "dec3b", "enc3b"), ("dec2a", "dec2b", "enc2b"), ("dec1a", "dec1b", "enc1b")]


def forward(spec: UNetSpec, theta: np.ndarray, x: np.ndarray):
    """x [B][cin][H][W] (H, W divisible by 8) -> (y_m [B][P][H][W], y_w [B][H][W], cache)."""
    p = unpack(spec, theta)
    a = {}          # post-ReLU activations
    inp = {}        # the input each conv saw
    h = x
    for ca, cb, mode in _ENC:
        if mode == "pool":
            h = pool2(h)
        inp[ca] = h
        a[ca] = relu(conv3(h, *p[ca]))
        inp[cb] = a[ca]
        a[cb] = relu(conv3(a[ca], *p[cb]))
        h = a[cb]
    for ca, cb, skip in _DEC:
        h = np.concatenate([up2(h), a[skip]], axis=1)
        inp[ca] = h
        a[ca] = relu(conv3(h, *p[ca]))
        inp[cb] = a[ca]
        a[cb] = relu(conv3(a[ca], *p[cb]))
        h = a[cb]
    y_m = conv1(h, *p["head_m"])
    y_w = sigmoid(conv1(h, *p["head_w"]))[:, 0]
    return y_m, y_w, (p, a, inp)


def loss(y_m, y_w, t_m, t_w, lam_w=1.0):
    return float(np.mean((y_m - t_m) ** 2) + lam_w * np.mean((y_w - t_w) ** 2))


def loss_and_grad(spec: UNetSpec, theta, x, t_m, t_w, lam_w=1.0):
    """Loss and its gradient w.r.t. the flat parameter vector."""
    y_m, y_w, (p, a, inp) = forward(spec, theta, x)
    L = loss(y_m, y_w, t_m, t_w, lam_w)
    g = {}
    gy_m = 2.0 * (y_m - t_m) / y_m.size
    gy_w = 2.0 * lam_w * (y_w - t_w) / y_w.size
    gz_w = (gy_w * y_w * (1.0 - y_w))[:, None]
    h = a["dec1b"]
    gh_m, gwm, gbm = conv1_backward(h, p["head_m"][0], gy_m)
    gh_w, gww, gbw = conv1_backward(h, p["head_w"][0], gz_w)
    g["head_m"] = (gwm, gbm)
    g["head_w"] = (gww, gbw)
    ga = {k: np.zeros_like(v) for k, v in a.items()}
    ga["dec1b"] += gh_m + gh_w

    def conv_back(name):
        gz = ga[name] * (a[name] > 0)
        gx, gw_, gb_ = conv3_backward(inp[name], p[name][0], gz)
        g[name] = (gw_, gb_)
        return gx

    for ca, cb, skip in reversed(_DEC):
        gx = conv_back(cb)
        ga[ca] += gx
        gx = conv_back(ca)
        cu = gx.shape[1] - a[skip].shape[1]
        ga[skip] += gx[:, cu:]
        below = {"enc3b": "botb", "enc2b": "dec3b", "enc1b": "dec2b"}[skip]
        ga[below] += up2_backward(gx[:, :cu])
    for i in reversed(range(len(_ENC))):
        ca, cb, mode = _ENC[i]
        gx = conv_back(cb)
        ga[ca] += gx
        gx = conv_back(ca)
        if mode == "pool":
            ga[_ENC[i - 1][1]] += pool2_backward(gx)
    return L, pack(spec, g)


def adamw_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One AdamW update (decoupled weight decay), step counted from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    theta = theta * (1 - lr * weight_decay) - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v
