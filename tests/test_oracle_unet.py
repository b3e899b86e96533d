"""Pins of the FP64 warm-start U-Net reference (oracle/unet.py).

* the 3x3 convolution equals scipy's 2-D cross-correlation summed over
  input channels (library routine);
* pooling / upsampling backward passes are the transposes of their forward
  passes (dot-product test);
* the hand-written gradient of the whole network equals central finite
  differences of the loss (brute force) on a tiny network;
* the AdamW step reproduces its closed form on a one-parameter problem.
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet as U


def test_conv3_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 6, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = U.conv3(x, w, b)
    ref = np.zeros_like(y)
    for bi in range(2):
        for o in range(4):
            ref[bi, o] = b[o] + sum(correlate2d(x[bi, c], w[o, c], mode="same") for c in range(3))
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_pool_and_upsample_backward_are_transposes():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 8, 12))
    y = rng.standard_normal((2, 3, 4, 6))
    assert np.isclose(np.sum(U.pool2(x) * y), np.sum(x * U.pool2_backward(y)), rtol=1e-13)
    assert np.isclose(np.sum(U.up2(y) * x), np.sum(y * U.up2_backward(x)), rtol=1e-13)


def test_conv_backward_is_transpose():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 3, 5, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    gy = rng.standard_normal((1, 4, 5, 7))
    gx, gw, gb = U.conv3_backward(x, w, gy)
    lin = U.conv3(x, w, np.zeros(4))
    assert np.isclose(np.sum(lin * gy), np.sum(x * gx), rtol=1e-12)
    assert np.isclose(np.sum(lin * gy), np.sum(w * gw), rtol=1e-12)


def test_network_gradient_matches_finite_differences():
    spec = U.UNetSpec(cin=1, pout=3, base=2)
    rng = np.random.default_rng(3)
    theta = U.init_params(spec, rng) + 0.05 * rng.standard_normal(spec.n_params())
    x = rng.standard_normal((2, 1, 16, 16))
    t_m = rng.standard_normal((2, 3, 16, 16))
    t_w = rng.uniform(0.1, 1.0, (2, 16, 16))
    L, g = U.loss_and_grad(spec, theta, x, t_m, t_w, lam_w=0.7)
    assert g.shape == theta.shape
    idx = rng.choice(theta.size, 60, replace=False)
    # every conv's bias and a few weights of each
    o = 0
    for _, ci, co, k in spec.convs():
        idx = np.append(idx, [o, o + co * ci * k * k])
        o += co * ci * k * k + co
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        yp = U.forward(spec, tp, x)
        ym = U.forward(spec, tm, x)
        fd = (U.loss(yp[0], yp[1], t_m, t_w, 0.7) - U.loss(ym[0], ym[1], t_m, t_w, 0.7)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_param_count_and_layout():
    spec = U.UNetSpec(cin=1, pout=32, base=16)
    n = spec.n_params()
    assert n == sum(co * ci * k * k + co for _, ci, co, k in spec.convs())
    theta = np.arange(n, dtype=np.float64)
    assert np.array_equal(U.pack(spec, U.unpack(spec, theta)), theta)
    assert U.unpack(spec, theta)["enc1a"][0].shape == (16, 1, 3, 3)
    assert U.unpack(spec, theta)["dec3a"][0].shape == (64, 192, 3, 3)
    assert U.unpack(spec, theta)["dec4a"][0].shape == (128, 256, 3, 3)
    assert U.unpack(spec, theta)["botb"][0].shape == (128, 128, 3, 3)
    assert n == 1_225_345


def test_bf16_round_matches_torch_bfloat16():
    """The precision model's rounding against torch's FP32 -> bfloat16
    conversion (round to nearest, ties to even) on the CPU: random values
    over many binades, exact ties, values already on the grid, subnormals."""
    import torch
    rng = np.random.default_rng(5)
    v = rng.standard_normal(20000) * np.exp2(rng.integers(-40, 40, 20000))
    grid = rng.integers(-2**15, 2**15, 4000).astype(np.int64)
    on = np.ldexp(128.0 + (np.abs(grid) % 128), rng.integers(-20, 20, 4000)) * np.sign(grid + 0.5)
    ties = on + np.ldexp(1.0, np.frexp(on)[1] - 9) * np.sign(on)      # half an ulp above a grid value
    sub = rng.standard_normal(2000) * 2.0 ** -130
    for a in (v, on, ties, sub):
        a32 = a.astype(np.float32)
        ref = torch.from_numpy(a32).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(U.bf16_round(a32.astype(np.float64)), ref)
    assert np.array_equal(U.bf16_round(on), on)
    # a tie goes to the even neighbour: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert U.bf16_round(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert U.bf16_round(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6


def test_bf16_precision_model_is_a_small_perturbation():
    """Rounding the operands moves the outputs by a BF16-sized amount (a
    few units of 2^-9 relative), never zero and never O(1)."""
    spec = U.UNetSpec(cin=1, pout=3, base=4)
    rng = np.random.default_rng(8)
    theta = U.init_params(spec, rng) + 0.05 * rng.standard_normal(spec.n_params())
    x = rng.standard_normal((1, 1, 32, 48))
    y0, w0, _ = U.forward(spec, theta, x)
    y1, w1, _ = U.forward(spec, theta, x, bf16=True)
    e = np.linalg.norm(y1 - y0) / np.linalg.norm(y0)
    assert 2.0 ** -12 < e < 2.0 ** -4
    t_m = rng.standard_normal(y0.shape)
    t_w = rng.uniform(0.1, 1.0, w0.shape)
    L0, g0 = U.loss_and_grad(spec, theta, x, t_m, t_w)
    L1, g1 = U.loss_and_grad(spec, theta, x, t_m, t_w, bf16=True)
    eg = np.linalg.norm(g1 - g0) / np.linalg.norm(g0)
    assert 2.0 ** -12 < eg < 2.0 ** -3


def test_adamw_closed_form():
    th, g = np.array([2.0]), np.array([0.5])
    th1, m, v = U.adamw_step(th, g, np.zeros(1), np.zeros(1), 1, lr=0.1, weight_decay=0.01)
    # first step: mhat = g, vhat = g^2, update = g / (|g| + eps)
    assert np.isclose(th1[0], 2.0 * (1 - 0.1 * 0.01) - 0.1 * 0.5 / (0.5 + 1e-8), rtol=1e-14)
