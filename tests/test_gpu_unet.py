"""GPU parity of the warm-start U-Net kernels against the FP64 reference
(oracle/unet.py), through the C ABI (unet_forward, unet_loss_grad,
unet_train_step).

The GPU runs BF16 weights and activations with FP32 accumulation.  Both bars
are derived from the reference on the CPU, for the same inputs:

* against the reference under its BF16 operand precision model (the same
  operands rounded at the same places, FP64 sums) what is left is FP32
  accumulation, whose different rounding flips some BF16 roundings of the
  activations, and a flipped rounding is a whole BF16 unit that cascades
  through the next layers.  The floor for that is the distance between the
  rounded reference summed in FP32 (numpy's order) and in FP64: a second,
  independent summation.  The bar is twice the floor (2.5 times for the
  gradients, whose reductions the GPU splits into more partial sums) plus a
  small absolute term (the sigmoid's fast exponential);
* against the exact reference the bar is what BF16 operands alone cost (the
  distance between the exact and the rounded reference) times 1.5, plus the
  first bar.

Shapes cover several conv tiles (4 x 32 outputs) with ragged edges at every
level (W = 208 -> 13 columns at the bottom level), and the production
gather's shape (256 x 1024, P = 32, 1.2M parameters) against stored values.
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


def _tight(floor, slack=5e-4, factor=2.0):
    """Bar against the BF16-operand reference from the FP32-accumulation floor."""
    return factor * floor + slack


def _derived(cost, tight):
    """Bar against the exact reference from the BF16-operand cost."""
    return 1.5 * cost + tight


@pytest.mark.parametrize("shape", [(2, 16, 64, 4, 16), (1, 32, 208, 8, 16), (1, 16, 32, 3, 8)])
def test_forward_matches_reference(A, shape):
    B, H, W, P, base = shape
    print(f"[gpu] unet forward B={B} H={H} W={W} P={P} base={base}", flush=True)
    spec, rng, theta, x, net, xt = _setup(A, B, H, W, P, base, 10)
    y_m, y_w = net.forward(xt)
    y_m, y_w = y_m.cpu().numpy(), y_w.cpu().numpy()
    r_m, r_w, _ = U.forward(spec, theta, x)
    b_m, b_w, _ = U.forward(spec, theta, x, bf16=True)
    f_m, f_w, _ = U.forward(spec, theta, x, bf16=True, acc32=True)
    t_m, t_w = rel_l2(y_m, b_m), rel_l2(y_w, b_w)
    t_wmax = float(np.max(np.abs(y_w - b_w)))
    fl_m, fl_w, fl_wmax = rel_l2(f_m, b_m), rel_l2(f_w, b_w), float(np.max(np.abs(f_w - b_w)))
    e_m, e_w = rel_l2(y_m, r_m), rel_l2(y_w, r_w)
    c_m, c_w = rel_l2(b_m, r_m), rel_l2(b_w, r_w)
    print(f"  vs BF16-operand reference: y_m {t_m:.2e} y_w {t_w:.2e} max abs {t_wmax:.2e} "
          f"(FP32 floor {fl_m:.2e} {fl_w:.2e} {fl_wmax:.2e})", flush=True)
    print(f"  vs exact: y_m {e_m:.2e} y_w {e_w:.2e} (BF16 operand cost {c_m:.2e} {c_w:.2e})", flush=True)
    assert t_m <= _tight(fl_m) and t_w <= _tight(fl_w)
    assert t_wmax <= _tight(fl_wmax, 1e-3)
    assert e_m <= _derived(c_m, _tight(fl_m)) and e_w <= _derived(c_w, _tight(fl_w))


@pytest.mark.parametrize("shape", [(2, 16, 64, 4, 16), (1, 32, 208, 8, 16)])
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
    L_bf, g_bf = U.loss_and_grad(spec, theta, x, t_m, t_w, lam_w=0.5, bf16=True)
    L_32, g_32 = U.loss_and_grad(spec, theta, x, t_m, t_w, lam_w=0.5, bf16=True, acc32=True)
    g = g.cpu().numpy()
    print(f"  loss gpu {loss:.6f} BF16-operand ref {L_bf:.6f} (FP32-summed {L_32:.6f}) exact {L_ref:.6f}",
          flush=True)
    tight_L = 2.5 * abs(L_32 - L_bf) + 1e-4 * abs(L_bf)
    assert abs(loss - L_bf) <= tight_L
    assert abs(loss - L_ref) <= 1.5 * abs(L_bf - L_ref) + tight_L
    o = 0
    for name, ci, co, k in spec.convs():
        # one layer's weight and bias gradient together (head_w's bias alone
        # is one cancelling sum, too small a sample for a relative bar)
        sl = slice(o, o + co * ci * k * k + co)
        t, f = rel_l2(g[sl], g_bf[sl]), rel_l2(g_32[sl], g_bf[sl])
        e, c = rel_l2(g[sl], g_ref[sl]), rel_l2(g_bf[sl], g_ref[sl])
        print(f"  {name}: vs BF16-operand ref {t:.2e} (FP32 floor {f:.2e}) | vs exact {e:.2e} "
              f"(BF16 operand cost {c:.2e})", flush=True)
        bar = _tight(f, 1e-3, 2.5)
        assert t <= bar, name
        assert e <= _derived(c, bar), name
        o += co * ci * k * k + co
    t_all, e_all = rel_l2(g, g_bf), rel_l2(g, g_ref)
    f_all, c_all = rel_l2(g_32, g_bf), rel_l2(g_bf, g_ref)
    print(f"  whole gradient: vs BF16-operand ref {t_all:.2e} (floor {f_all:.2e}) vs exact {e_all:.2e} "
          f"(cost {c_all:.2e})", flush=True)
    assert t_all <= _tight(f_all, 5e-4, 2.5)
    assert e_all <= _derived(c_all, _tight(f_all, 5e-4, 2.5))


def test_forward_production_shape_matches_stored_reference(A):
    """256 x 1024 gather, P = 32, base 16 (1,225,345 parameters): sampled
    outputs against the stored exact and BF16-operand references."""
    import json
    import os
    import torch
    from tests.golden.make_unet_values import inputs
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_unet_samples.json")))
    spec, theta, x = inputs()
    B, _, H, W = x.shape
    P = spec.pout
    assert (H, W, P, spec.n_params()) == (ref["H"], ref["W"], ref["pout"], ref["n_params"])
    print(f"[gpu] unet forward production shape H={H} W={W} P={P} params={spec.n_params()}", flush=True)
    net = A.UNet(P, base=spec.base)
    net.set_params(theta)
    y_m, y_w = net.forward(torch.tensor(x[:, 0], dtype=torch.float32, device="cuda"))
    y_m, y_w = y_m.cpu().numpy().astype(np.float64), y_w.cpu().numpy().astype(np.float64)
    mi, wi = np.array(ref["y_m_index"]), np.array(ref["y_w_index"])
    sm, sw = y_m.ravel()[mi], y_w.ravel()[wi]
    t_m = rel_l2(sm, ref["bf16_y_m_value"])
    t_w = rel_l2(sw, ref["bf16_y_w_value"])
    e_m = rel_l2(sm, ref["exact_y_m_value"])
    e_w = rel_l2(sw, ref["exact_y_w_value"])
    nm = abs(np.linalg.norm(y_m) / ref["bf16_y_m_norm"] - 1)
    print(f"  samples vs BF16-operand ref: y_m {t_m:.2e} y_w {t_w:.2e}; norm {nm:.2e}", flush=True)
    print(f"  samples vs exact: y_m {e_m:.2e} y_w {e_w:.2e} (BF16 operand cost {ref['bf16_cost_y_m']:.2e} "
          f"{ref['bf16_cost_y_w']:.2e})", flush=True)
    tm_bar, tw_bar = _tight(ref["acc32_floor_y_m"]), _tight(ref["acc32_floor_y_w"])
    print(f"  bars: {tm_bar:.2e} {tw_bar:.2e} (FP32 floor {ref['acc32_floor_y_m']:.2e} "
          f"{ref['acc32_floor_y_w']:.2e})", flush=True)
    assert t_m <= tm_bar and t_w <= tw_bar and nm <= tm_bar
    assert e_m <= _derived(ref["bf16_cost_y_m"], tm_bar)
    assert e_w <= _derived(ref["bf16_cost_y_w"], tw_bar)


def test_batch_matches_single_samples(A):
    """A batch and its samples one at a time take different launch shapes:
    at 8 x 64 x 256 several convolutions split their channel chunks over
    workgroups (fewer than 512 workgroups) in different ways for B = 8 and
    B = 1, and the weight gradients split their pixels differently.  The
    batch forward must equal the single-sample forwards, and the batch
    gradient (the loss is a mean over samples) the mean of the single-sample
    gradients, to the FP32-accumulation floor of the production-shape
    reference: two FP32 summation orders of the same BF16-operand network
    differ by up to that much, where a wrong split or route is O(1)."""
    import json
    import os
    import torch
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_unet_samples.json")))
    bar = ref["acc32_floor_y_m"]
    B, H, W, P = 8, 64, 256, 8
    spec, rng, theta, x, net, xt = _setup(A, B, H, W, P, 16, 14)
    t_m = torch.tensor(0.3 * rng.standard_normal((B, P, H, W)), dtype=torch.float32, device="cuda")
    t_w = torch.tensor(rng.uniform(0.1, 1, (B, H, W)), dtype=torch.float32, device="cuda")
    y_m, y_w = net.forward(xt)
    y_m, y_w = y_m.clone(), y_w.clone()
    _, g = net.loss_grad(xt, t_m, t_w)
    g = g.clone()
    g_mean = torch.zeros_like(g)
    e_m = e_w = 0.0
    for i in range(B):
        a, b = net.forward(xt[i:i + 1].contiguous())
        e_m = max(e_m, rel_l2(a[0].cpu().numpy(), y_m[i].cpu().numpy()))
        e_w = max(e_w, rel_l2(b[0].cpu().numpy(), y_w[i].cpu().numpy()))
        _, gi = net.loss_grad(xt[i:i + 1].contiguous(), t_m[i:i + 1].contiguous(), t_w[i:i + 1].contiguous())
        g_mean += gi
    g_mean /= B
    e_g = rel_l2(g_mean.cpu().numpy(), g.cpu().numpy())
    print(f"[gpu] unet batch vs single: y_m {e_m:.2e} y_w {e_w:.2e} gradient {e_g:.2e} (bar {bar:.2e})", flush=True)
    assert e_m <= bar and e_w <= bar and e_g <= bar


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
    with pytest.raises(A.AshrtError):     # a multiple of 8 but not of 16
        net.forward(torch.zeros((1, 24, 64), device="cuda"))
    with pytest.raises(A.AshrtError):
        A.UNet(200, base=16)
