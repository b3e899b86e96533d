"""Learned warm start for the robust inversion (thesis Chapter 4's IRLS loop).

A U-Net (``unet.UNet``, HIP kernels) maps a blended receiver gather to an
initial Radon model m0 and initial residual weights w0.  Its training labels
come from the method itself: the plain zero-start GPU solve gives m*, and its
final residual r = d - L m* with clip eps gives the weights
w* = sqrt(eps / max(|r|, eps)), the l1 IRLS residual weight scaled into (0, 1]
(a global scale of W_r does not change the weighted least-squares problem).

Network input and targets are scaled by the gather's RMS s: x = d / s,
t_m = m* / s; the prediction is used as m0 = s y_m, w0 = y_w.  Before a
warm-started solve the prediction is checked against the zero start: if
L m0 does not fit the data better than m = 0 (l_p misfit), the solve falls
back to a zero start (keeping the predicted weights).
"""
import sys
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from .ashrt import Params, Plan
from .unet import TrainParams, UNet


def gather_scale(d: torch.Tensor) -> float:
    s = float(torch.sqrt(torch.mean(d.double() * d.double())))
    return s if s > 0 else 1.0


def weight_target(d: torch.Tensor, d_rec: torch.Tensor, eps: float) -> torch.Tensor:
    """sqrt(eps / max(|d - d_rec|, eps)): the final l1 residual weights in (0, 1]."""
    r = (d - d_rec).abs()
    e = max(float(eps), 1e-30)
    return torch.sqrt(e / torch.clamp(r, min=e))


@dataclass
class Labels:
    x: torch.Tensor        # [N][H][W]   d / s
    t_m: torch.Tensor      # [N][P][H][W] m* / s
    t_w: torch.Tensor      # [N][H][W]
    scale: np.ndarray      # [N]


def make_labels(plan: Plan, gathers: List[np.ndarray], params: Params) -> Labels:
    """Plain zero-start GPU solves of every gather; returns the training set."""
    dev = plan.device
    N = len(gathers)
    H, W = gathers[0].shape
    x = torch.empty((N, H, W), dtype=torch.float32, device=dev)
    t_m = torch.empty((N, plan.npanel, H, W), dtype=torch.float32, device=dev)
    t_w = torch.empty((N, H, W), dtype=torch.float32, device=dev)
    scale = np.zeros(N)
    for i, g in enumerate(gathers):
        d = torch.tensor(g, dtype=torch.float32, device=dev)
        m, d_rec, rep = plan.robust_invert(d, params)
        s = gather_scale(d)
        scale[i] = s
        x[i] = d / s
        t_m[i] = m / s
        eps = rep["eps_r"][-1] if params.p == 1 else float((d - d_rec).abs().median())
        t_w[i] = weight_target(d, d_rec, eps)
    return Labels(x, t_m, t_w, scale)


def train(net: UNet, lab: Labels, epochs: int, batch: int, tp: TrainParams, seed: int = 0,
          log_every: int = 0) -> List[float]:
    """Shuffled mini-batch AdamW training; returns the per-step losses."""
    rng = np.random.default_rng(seed)
    N = lab.x.shape[0]
    losses = []
    step = 0
    for ep in range(epochs):
        order = rng.permutation(N)
        for b0 in range(0, N - batch + 1, batch):
            idx = torch.as_tensor(order[b0:b0 + batch], device=lab.x.device)
            xb = lab.x.index_select(0, idx).contiguous()
            mb = lab.t_m.index_select(0, idx).contiguous()
            wb = lab.t_w.index_select(0, idx).contiguous()
            want = log_every > 0 and step % log_every == 0
            loss = net.train_step(xb, mb, wb, tp, want_loss=want)
            if want:
                losses.append(loss)
                print(f"[warmstart] epoch {ep} step {step} loss {loss:.5f}", file=sys.stderr, flush=True)
            step += 1
    return losses


def predict(net: UNet, d: torch.Tensor):
    """(m0, w0) for one gather d [nx][nt]."""
    s = gather_scale(d)
    y_m, y_w = net.forward((d / s)[None].contiguous())
    return y_m[0] * s, y_w[0]


def lp_misfit(plan: Plan, d: torch.Tensor, m: torch.Tensor, p: int) -> float:
    r = d - plan.forward(m)
    return float(r.abs().sum()) if p == 1 else float((r * r).sum())


def warm_solve(plan: Plan, net: UNet, d: torch.Tensor, params: Params, use_weights: bool = True):
    """Warm-started robust solve.  The predicted model is kept only if L m0
    fits the data better than m = 0 (l_p misfit); otherwise the solve starts
    from zero, with the predicted weights if use_weights.  Returns
    (m, d_rec, report, start) with start "model+weights", "weights" or
    "plain"."""
    m0, w0 = predict(net, d)
    zero = float(d.abs().sum()) if params.p == 1 else float((d * d).sum())
    w = w0.contiguous() if use_weights else None
    if lp_misfit(plan, d, m0, params.p) < zero:
        m, d_rec, rep = plan.robust_invert(d, params, m0=m0, w0=w)
        return m, d_rec, rep, "model+weights" if use_weights else "model"
    if use_weights:
        m, d_rec, rep = plan.robust_invert(d, params, w0=w)
        return m, d_rec, rep, "weights"
    m, d_rec, rep = plan.robust_invert(d, params)
    return m, d_rec, rep, "plain"


def q_db(clean: np.ndarray, est: np.ndarray) -> float:
    """Separation quality 10 log10(|clean|^2 / |clean - est|^2) (thesis
    Chapter 4, equation ch4_Qr)."""
    c = np.asarray(clean, np.float64)
    e = np.asarray(est, np.float64)
    return float(10.0 * np.log10(np.sum(c * c) / np.sum((c - e) ** 2)))


def outer_to_target(plan: Plan, d: torch.Tensor, clean: np.ndarray, target_db: float, params: Params,
                    net: Optional[UNet] = None, max_outer: Optional[int] = None, slack_db: float = 0.05,
                    use_weights: bool = True):
    """Smallest outer-iteration count whose separated gather reaches
    target_db - slack_db, for the plain (net None) or warm-started solve.
    Returns (k or None, Q_R at k, wall seconds of that solve including the
    network's inference, start kind)."""
    import time
    kmax = max_outer or params.n_outer
    q, dt, start = float("nan"), 0.0, "plain"
    for k in range(1, kmax + 1):
        prm = Params(**{**params.__dict__, "n_outer": k})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if net is None:
            _, d_rec, _ = plan.robust_invert(d, prm, want_report=False)
        else:
            _, d_rec, _, start = warm_solve(plan, net, d, prm, use_weights=use_weights)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        q = q_db(clean, d_rec.cpu().numpy())
        if q >= target_db - slack_db:
            return k, q, dt, start
    return None, q, dt, start
