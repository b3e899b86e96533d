"""The learned warm start against the plain method on the same GPU.

Training labels come from the plain zero-start GPU solve of seeded
synthetic gathers (the small receiver-gather law: 256 samples x 64 traces,
8 velocities, 5 x 10 IRLS-CG); the U-Net is trained by the library's own
kernels.  On held-out gathers, each method's outer-iteration count to reach
the plain method's final separated-signal SNR (minus 0.05 dB) is measured;
the warm start must need fewer on average and must reach the target on
every gather.
"""
import numpy as np
import pytest

from synth import make_gather, workload

pytestmark = pytest.mark.gpu


def test_learned_warm_start_reaches_plain_snr_sooner():
    import torch
    import paper_1711_10214_amd as A
    from paper_1711_10214_amd import warmstart as WS
    assert torch.cuda.is_available()
    w = workload("crg-256x64-nv8")
    train = [make_gather(w, seed=1_000_000 + i).d_blend.astype(np.float32) for i in range(192)]
    held = [make_gather(w, seed=2_000_000 + i) for i in range(16)]
    plan = A.Plan(w.nt, w.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    prm = A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)
    print("[gpu] warm start: labelling 192 gathers", flush=True)
    lab = WS.make_labels(plan, train, prm)
    net = A.UNet(w.npanel, base=16)
    net.init_params(seed=0)
    print("[gpu] warm start: training", flush=True)
    ws = WS.train(net, lab, epochs=16, batch=8, tp=A.TrainParams(lr=1e-3), seed=0)
    k_plain, k_warm, starts = [], [], []
    for i, g in enumerate(held):
        d = torch.tensor(g.d_blend.astype(np.float32), device="cuda")
        _, d_rec, _ = plan.robust_invert(d, prm, want_report=False)
        target = WS.q_db(g.d_clean, d_rec.cpu().numpy())
        kp, _, _, _ = WS.outer_to_target(plan, d, g.d_clean, target, prm)
        kw, qw, _, start = WS.outer_to_target(plan, d, g.d_clean, target, prm, ws=ws)
        print(f"  held-out {i}: target {target:.2f} dB plain {kp} warm {kw} ({start}, {qw:.2f} dB)", flush=True)
        assert kp is not None and kw is not None
        k_plain.append(kp)
        k_warm.append(kw)
        starts.append(start)
    print(f"  mean outer iterations to target: plain {np.mean(k_plain):.2f} warm {np.mean(k_warm):.2f}; "
          f"model starts {starts.count('model+weights')}/{len(starts)}", flush=True)
    assert np.mean(k_warm) < np.mean(k_plain)


def test_warm_start_vector_calls_match_numpy():
    """ashrt_vec_stats (FP64 sums of |a - alpha b|^p, <a, b>, <b, b>),
    ashrt_weight_target and ashrt_vec_scale against numpy in FP64."""
    import torch
    from paper_1711_10214_amd import warmstart as WS
    rng = np.random.default_rng(4)
    a = rng.standard_normal(300_001).astype(np.float32)
    b = rng.standard_normal(300_001).astype(np.float32)
    ta, tb = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    for p, alpha in ((1, 0.7), (2, -1.3), (2, 0.0)):
        s0, s1, s2 = WS.vec_stats(ta, tb, alpha, p)
        r = a64 - np.float64(alpha) * b64
        want0 = np.sum(np.abs(r)) if p == 1 else np.sum(r * r)
        assert abs(s0 / want0 - 1) < 1e-12
        assert abs(s1 - np.dot(a64, b64)) < 1e-9 * np.sum(np.abs(a64 * b64))
        assert abs(s2 / np.dot(b64, b64) - 1) < 1e-12
    s0, s1, s2 = WS.vec_stats(ta, None, 0.0, 2)
    assert abs(s0 / np.dot(a64, a64) - 1) < 1e-12 and s1 == 0.0 and s2 == 0.0
    w = WS.weight_target(ta, tb, 0.25).cpu().numpy()
    want = np.sqrt(0.25 / np.maximum(np.abs(a64 - b64), 0.25))
    assert np.max(np.abs(w - want)) < 1e-6
    y = WS.vec_scale(ta, -2.5).cpu().numpy()
    np.testing.assert_array_equal(y, (np.float32(-2.5) * a))
