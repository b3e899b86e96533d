"""GPU parity of the warm-start U-Net kernels against the FP64 reference
(oracle/unet.py), through the C ABI (unet_forward, unet_loss_grad,
unet_train_step).

The GPU runs BF16 weights and activations with FP32 accumulation, so the bar
is BF16-level: relative L2 <= 3e-2 on outputs and per-layer gradients.
Shapes cover several conv tiles (4 x 32 outputs) with ragged edges at every
level (H = 24 -> 3 rows at the bottom, W = 200 -> 25 columns).
"""
import numpy as np
import pytest

from oracle import unet as U
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available()
    return A


def _setup(A, B, H, W, P, base, seed):
    import torch
    spec = U.UNetSpec(cin=1, pout=P, base=base)
    rng = np.random.default_rng(seed)
    theta = U.init_params(spec, rng)
    theta += 0.05 * rng.standard_normal(theta.size)   # nonzero biases
    theta = theta.astype(np.float32).astype(np.float64)
    x = rng.standard_normal((B, 1, H, W)).astype(np.float32).astype(np.float64)
    net = A.UNet(P, base=base)
    assert net.n_params == spec.n_params()
    net.set_params(theta)
    xt = torch.tensor(x[:, 0], dtype=torch.float32, device="cuda")
    return spec, rng, theta, x, net, xt


@pytest.mark.parametrize("shape", [(2, 16, 64, 4, 16), (1, 24, 200, 8, 16), (1, 16, 32, 3, 8)])
def test_forward_matches_reference(A, shape):
    B, H, W, P, base = shape
    print(f"[gpu] unet forward B={B} H={H} W={W} P={P} base={base}", flush=True)
    spec, rng, theta, x, net, xt = _setup(A, B, H, W, P, base, 10)
    y_m, y_w = net.forward(xt)
    r_m, r_w, _ = U.forward(spec, theta, x)
    e_m = rel_l2(y_m.cpu().numpy(), r_m)
    e_w = rel_l2(y_w.cpu().numpy(), r_w)
    e_wmax = float(np.max(np.abs(y_w.cpu().numpy() - r_w)))
    print(f"  y_m rel-L2 {e_m:.2e}  y_w rel-L2 {e_w:.2e} max abs {e_wmax:.2e}", flush=True)
    assert e_m <= 3e-2
    assert e_w <= 3e-2
    # one output through 14 BF16-rounded layers: ~ a few BF16 ulps of the
    # logit, times the sigmoid's slope (<= 1/4)
    assert e_wmax <= 5e-2


@pytest.mark.parametrize("shape", [(2, 16, 64, 4, 16), (1, 24, 200, 8, 16)])
def test_gradient_matches_reference(A, shape):
    import torch
    B, H, W, P, base = shape
    print(f"[gpu] unet gradient B={B} H={H} W={W} P={P}", flush=True)
    spec, rng, theta, x, net, xt = _setup(A, B, H, W, P, base, 11)
    t_m = rng.standard_normal((B, P, H, W)).astype(np.float32).astype(np.float64) * 0.5
    t_w = rng.uniform(0.05, 1.0, (B, H, W)).astype(np.float32).astype(np.float64)
    loss, g = net.loss_grad(xt, torch.tensor(t_m, dtype=torch.float32, device="cuda"),
                            torch.tensor(t_w, dtype=torch.float32, device="cuda"), lam_w=0.5)
    L_ref, g_ref = U.loss_and_grad(spec, theta, x, t_m, t_w, lam_w=0.5)
    g = g.cpu().numpy()
    print(f"  loss gpu {loss:.6f} ref {L_ref:.6f}", flush=True)
    assert abs(loss - L_ref) <= 1e-2 * abs(L_ref)
    o = 0
    for name, ci, co, k in spec.convs():
        nw = co * ci * k * k
        ew = rel_l2(g[o:o + nw], g_ref[o:o + nw])
        eb = rel_l2(g[o + nw:o + nw + co], g_ref[o + nw:o + nw + co])
        print(f"  {name}: dW {ew:.2e} db {eb:.2e}", flush=True)
        # the backward pass rounds the masked output gradient to BF16 at
        # every layer (the matrix-core operand), so the error grows with the
        # depth from the loss: ~1e-2 next to the heads, ~3e-2 at the bottom
        assert ew <= 5e-2 and eb <= 5e-2, name
        o += nw + co
    e_all = rel_l2(g, g_ref)
    print(f"  whole gradient rel-L2 {e_all:.2e}", flush=True)
    assert e_all <= 3e-2


def test_train_step_is_adamw_on_the_gradient(A):
    import torch
    B, H, W, P = 1, 16, 64, 4
    spec, rng, theta, x, net, xt = _setup(A, B, H, W, P, 16, 12)
    t_m = torch.tensor(rng.standard_normal((B, P, H, W)), dtype=torch.float32, device="cuda")
    t_w = torch.tensor(rng.uniform(0.1, 1, (B, H, W)), dtype=torch.float32, device="cuda")
    _, g = net.loss_grad(xt, t_m, t_w)
    tp = A.TrainParams(lr=1e-3, weight_decay=0.01)
    net.train_step(xt, t_m, t_w, tp)
    th1 = net.get_params().astype(np.float64)
    ref, _, _ = U.adamw_step(theta, g.cpu().numpy().astype(np.float64), np.zeros_like(theta),
                             np.zeros_like(theta), 1, lr=1e-3, weight_decay=0.01)
    np.testing.assert_allclose(th1, ref, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss(A):
    import torch
    B, H, W, P = 2, 32, 128, 4
    spec, rng, theta, x, net, xt = _setup(A, B, H, W, P, 16, 13)
    # a learnable target: smooth functions of the input
    xs = x[:, 0]
    t_m = torch.tensor(np.stack([np.stack([np.roll(xs[b], s, axis=1) * 0.3 for s in range(P)]) for b in range(B)]),
                       dtype=torch.float32, device="cuda")
    t_w = torch.tensor(1.0 / (1.0 + np.abs(xs)), dtype=torch.float32, device="cuda")
    tp = A.TrainParams(lr=2e-3)
    losses = [net.train_step(xt, t_m, t_w, tp) for _ in range(60)]
    print(f"[gpu] unet training loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0]


def test_rejects_bad_shapes(A):
    import torch
    net = A.UNet(4, base=16)
    with pytest.raises(A.AshrtError):
        net.forward(torch.zeros((1, 12, 64), device="cuda"))
    with pytest.raises(A.AshrtError):
        A.UNet(200, base=16)
