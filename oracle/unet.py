"""FP64 reference of the warm-start U-Net: forward, loss and backward.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network is not in the thesis: it is the learned warm start for the
robust inversion of Chapter 4 (a predicted initial Radon model m0 and
initial residual weights w0 for the IRLS outer loop).  This module is its
plain definition, written out with numpy in FP64, and the gradient by hand
(reverse-mode, layer by layer), so the GPU kernels can be checked against it.

Architecture (channels c = base * (1, 2, 4, 8, 8), four 2x down-samplings):

    enc1a: 3x3 conv  Cin -> c1, ReLU          enc1b: c1 -> c1, ReLU
    enc2a: 2x2 mean pool, 3x3 c1 -> c2, ReLU  enc2b: c2 -> c2, ReLU
    enc3a: pool, c2 -> c3, ReLU               enc3b: c3 -> c3, ReLU
    enc4a: pool, c3 -> c4, ReLU               enc4b: c4 -> c4, ReLU
    bota:  pool, c4 -> c5, ReLU               botb:  c5 -> c5, ReLU
    dec4a: [nearest 2x upsample(botb), enc4b] c5+c4 -> c4, ReLU;  dec4b: c4 -> c4
    dec3a: [up(dec4b), enc3b] c4+c3 -> c3, ReLU;                   dec3b: c3 -> c3
    dec2a: [up(dec3b), enc2b] c3+c2 -> c2, ReLU;                   dec2b: c2 -> c2
    dec1a: [up(dec2b), enc1b] c2+c1 -> c1, ReLU;                   dec1b: c1 -> c1
    head_m: 1x1 conv c1 -> P (linear)          -> y_m (predicted model / scale)
    head_w: 1x1 conv c1 -> 1, logistic sigmoid -> y_w (predicted weights)

With base 16 and P = 32 this is 1,225,345 parameters.  H and W must be
multiples of 16.

3x3 convolutions are cross-correlations with zero padding and a bias.
Loss:  mean (y_m - t_m)^2 + lam_w mean (y_w - t_w)^2.

Precision model (optional, ``bf16=True``): the arithmetic stays FP64, but the
operands of every 3x3 convolution are rounded to bfloat16 (round to nearest,
ties to even) where a BF16 matrix-core implementation would hold them: the
network input, the 3x3 weights, every 3x3 conv output after bias and ReLU,
every 2x2 mean pool output, and in the backward pass the ReLU-masked output
gradient that feeds the input- and weight-gradient products.  Biases, the 1x1
heads, the loss and the bias gradients stay unrounded.  Comparing the exact
and the rounded network on the CPU measures what BF16 operands alone cost;
comparing a BF16 implementation with the rounded network leaves only its
accumulation.  With ``acc32=True`` as well, the 3x3 products are summed in
FP32 (numpy's order): the distance between that and the FP64-summed rounded
network is the floor any FP32-accumulating BF16 implementation sits at, since
a different summation flips some BF16 roundings of the activations and the
flips propagate.

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
        c1, c2, c3, c4, c5 = (self.base * f for f in (1, 2, 4, 8, 8))
        return [
            ("enc1a", self.cin, c1, 3), ("enc1b", c1, c1, 3),
            ("enc2a", c1, c2, 3), ("enc2b", c2, c2, 3),
            ("enc3a", c2, c3, 3), ("enc3b", c3, c3, 3),
            ("enc4a", c3, c4, 3), ("enc4b", c4, c4, 3),
            ("bota", c4, c5, 3), ("botb", c5, c5, 3),
            ("dec4a", c5 + c4, c4, 3), ("dec4b", c4, c4, 3),
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

def conv3(x, w, b, acc=np.float64):
    """Cross-correlation with a 3x3 kernel, zero padding 1, plus bias; the
    products summed in `acc` (FP64 unless the precision model asks for FP32)."""
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1))).astype(acc)
    w = w.astype(acc)
    y = np.zeros((B, w.shape[0], H, W), acc)
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oc,bchw->bohw", w[:, :, dy, dx], xp[:, :, dy:dy + H, dx:dx + W])
    return (y + b[None, :, None, None].astype(acc)).astype(np.float64)


def conv3_backward(x, w, gy, acc=np.float64):
    """Gradients of conv3 w.r.t. its input, weight and bias, given dL/dy
    (products summed in `acc`)."""
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1))).astype(acc)
    w, gy = w.astype(acc), gy.astype(acc)
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            gw[:, :, dy, dx] = np.einsum("bohw,bchw->oc", gy, xp[:, :, dy:dy + H, dx:dx + W])
            gxp[:, :, dy:dy + H, dx:dx + W] += np.einsum("oc,bohw->bchw", w[:, :, dy, dx], gy)
    f = np.float64
    return gxp[:, :, 1:H + 1, 1:W + 1].astype(f), gw.astype(f), gy.sum(axis=(0, 2, 3)).astype(f)


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


def bf16_round(a):
    """Round to the nearest bfloat16 value, ties to even.  bfloat16 keeps 8
    significant bits (7 stored, 1 implicit) and FP32's exponent range, so a
    normal value with frexp exponent E (a = f 2^E, 0.5 <= |f| < 1) is
    rounded to a multiple of 2^(E - 8).  Values below FP32's normal range
    (|a| < 2^-126) round on the subnormal grid 2^-133."""
    a = np.asarray(a, dtype=np.float64)
    _, e = np.frexp(a)
    q = np.ldexp(1.0, np.maximum(e, -125) - 8)
    return np.round(a / q) * q


def _ident(a):
    return a


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


# ------------------------------------------------------------------ network
_ENC = [("enc1a", "enc1b", None), ("enc2a", "enc2b", "pool"), ("enc3a", "enc3b", "pool"),
        ("enc4a", "enc4b", "pool"), ("bota", "botb", "pool")]
_DEC = [("dec4a", "dec4b", "enc4b"), ("dec3a", "dec3b", "enc3b"), ("dec2a", "dec2b", "enc2b"),
        ("dec1a", "dec1b", "enc1b")]


def forward(spec: UNetSpec, theta: np.ndarray, x: np.ndarray, bf16: bool = False, acc32: bool = False):
    """x [B][cin][H][W] (H, W divisible by 16) -> (y_m [B][P][H][W], y_w [B][H][W], cache).
    bf16 / acc32: round the convolution operands / sum their products in
    FP32, as the precision model above states."""
    rd = bf16_round if bf16 else _ident
    acc = np.float32 if acc32 else np.float64
    p = unpack(spec, theta)
    if bf16:
        p = {k: ((rd(w), b) if w.shape[-1] == 3 else (w, b)) for k, (w, b) in p.items()}
    a = {}          # post-ReLU activations
    inp = {}        # the input each conv saw

    def conv_relu(name, h):
        inp[name] = h
        a[name] = rd(relu(conv3(h, *p[name], acc=acc)))
        return a[name]

    h = rd(x)
    for ca, cb, mode in _ENC:
        if mode == "pool":
            h = rd(pool2(h))
        h = conv_relu(cb, conv_relu(ca, h))
    for ca, cb, skip in _DEC:
        h = np.concatenate([up2(h), a[skip]], axis=1)
        h = conv_relu(cb, conv_relu(ca, h))
    y_m = conv1(h, *p["head_m"])
    y_w = sigmoid(conv1(h, *p["head_w"]))[:, 0]
    return y_m, y_w, (p, a, inp)


def loss(y_m, y_w, t_m, t_w, lam_w=1.0):
    return float(np.mean((y_m - t_m) ** 2) + lam_w * np.mean((y_w - t_w) ** 2))


def loss_and_grad(spec: UNetSpec, theta, x, t_m, t_w, lam_w=1.0, bf16: bool = False, acc32: bool = False):
    """Loss and its gradient w.r.t. the flat parameter vector (bf16, acc32:
    the precision model above; the weights the products use are the rounded
    ones, the gradient is still taken for the unrounded parameters)."""
    rd = bf16_round if bf16 else _ident
    acc = np.float32 if acc32 else np.float64
    y_m, y_w, (p, a, inp) = forward(spec, theta, x, bf16, acc32)
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
        gx, gw_, _ = conv3_backward(inp[name], p[name][0], rd(gz), acc=acc)
        g[name] = (gw_, gz.sum(axis=(0, 2, 3)))
        return gx

    for ca, cb, skip in reversed(_DEC):
        gx = conv_back(cb)
        ga[ca] += gx
        gx = conv_back(ca)
        cu = gx.shape[1] - a[skip].shape[1]
        ga[skip] += gx[:, cu:]
        below = {"enc4b": "botb", "enc3b": "dec4b", "enc2b": "dec3b", "enc1b": "dec2b"}[skip]
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
