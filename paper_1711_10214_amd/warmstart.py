"""Learned warm start for the robust inversion (thesis Chapter 4's IRLS loop).

A U-Net (``unet.UNet``, HIP kernels) maps a blended receiver gather to an
initial Radon model m0 and initial residual weights w0.  Its training labels
come from the method itself: the plain zero-start GPU solve gives m*, and its
final residual r = d - L m* with clip eps gives the weights
w* = sqrt(eps / max(|r|, eps)), the l1 IRLS residual weight scaled into (0, 1]
(a global scale of W_r does not change the weighted least-squares problem).

Scales: the network sees x = d / s with s the gather's RMS; its model head
is trained on k m* / s, k a constant that brings the model labels to unit
RMS over the training set (without it the model head's loss is a small
fraction of the total and the head learns little); m0 = s y_m / k.

Before a warm-started solve the prediction is checked against the zero
start: m0 is first scaled by the least-squares step length along it,
alpha = <d, L m0> / |L m0|^2 (alpha >= 0), and alpha m0 replaces the zero
start only if it fits the data better than m = 0 in the l_p misfit;
otherwise the solve starts from zero with the predicted weights.  The
predicted weights only shape outer iteration 1: every later iteration
recomputes W_r from its own residual, so the solve still runs to the l1
fixed point of plain IRLS-CG.

Every step on the data runs in the library (ashrt_vec_stats,
ashrt_weight_target, ashrt_vec_scale, the operator and the solver); this
module only sequences the calls and reads back scalars.
"""
import ctypes as C
import sys
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Iterable, List, Optional

import numpy as np
import torch

from . import _lib as L
from .ashrt import Params, Plan
from .unet import TrainParams, UNet


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream(t):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def vec_stats(a: torch.Tensor, b: Optional[torch.Tensor] = None, alpha: float = 1.0, p: int = 2):
    """(sum |a - alpha b|^p, <a, b>, <b, b>) in FP64 by the library (b None: zeros)."""
    out = torch.empty(3, dtype=torch.float64, device=a.device)
    L.check(L.lib().ashrt_vec_stats(_ptr(a), _ptr(b), a.numel(), float(alpha), int(p), _ptr(out), _stream(a)),
            "ashrt_vec_stats")
    v = out.cpu().numpy()
    return float(v[0]), float(v[1]), float(v[2])


def vec_scale(x: torch.Tensor, s: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    y = torch.empty_like(x) if out is None else out
    L.check(L.lib().ashrt_vec_scale(_ptr(x), x.numel(), float(s), _ptr(y), _stream(x)), "ashrt_vec_scale")
    return y


def gather_scale(d: torch.Tensor) -> float:
    """RMS of the gather (1 for an all-zero gather)."""
    ss, _, _ = vec_stats(d, None, 0.0, 2)
    s = float(np.sqrt(ss / max(d.numel(), 1)))
    return s if s > 0 else 1.0


def weight_target(d: torch.Tensor, d_rec: torch.Tensor, eps: float, out: Optional[torch.Tensor] = None):
    """sqrt(eps / max(|d - d_rec|, eps)): the final l1 residual weights in (0, 1]."""
    w = torch.empty_like(d) if out is None else out
    L.check(L.lib().ashrt_weight_target(_ptr(d), _ptr(d_rec), d.numel(), max(float(eps), 1e-30), _ptr(w),
                                        _stream(d)), "ashrt_weight_target")
    return w


@dataclass
class Labels:
    x: torch.Tensor        # [N][H][W]   d / s
    t_m: torch.Tensor      # [N][P][H][W] m* / s (times the model-label scale when used for training)
    t_w: torch.Tensor      # [N][H][W]
    scale: np.ndarray      # [N]


def label_one(plan: Plan, d: torch.Tensor, params: Params, x_out, tm_out, tw_out) -> float:
    """Plain zero-start solve of one gather; writes its network input and
    labels into the given slots and returns the gather scale s."""
    m, d_rec, rep = plan.robust_invert(d, params)
    s = gather_scale(d)
    vec_scale(d, 1.0 / s, x_out)
    vec_scale(m, 1.0 / s, tm_out)
    if params.p == 1:
        eps = rep["eps_r"][-1]
    else:   # the l2 solve has no clip: use the residual's RMS
        ss, _, _ = vec_stats(d, d_rec, 1.0, 2)
        eps = float(np.sqrt(ss / max(d.numel(), 1)))
    weight_target(d, d_rec, eps, tw_out)
    return s


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
        scale[i] = label_one(plan, d, params, x[i], t_m[i], t_w[i])
    return Labels(x, t_m, t_w, scale)


def model_label_scale(t_m: torch.Tensor) -> float:
    """k with RMS(k t_m) = 1 over the given labels."""
    ss, _, _ = vec_stats(t_m, None, 0.0, 2)
    rms = float(np.sqrt(ss / max(t_m.numel(), 1)))
    return 1.0 / rms if rms > 0 else 1.0


@dataclass
class WarmStart:
    """A trained network with the model-label scale it was trained with."""
    net: UNet
    m_scale: float = 1.0
    stats: dict = field(default_factory=dict)


def _train_steps(net: UNet, x, t_m, t_w, n_valid: int, steps: int, batch: int, tp: TrainParams, k: float, rng,
                 losses: list, log_every: int, step0: int):
    """steps AdamW steps on random mini-batches of the first n_valid buffer slots."""
    dev = x.device
    mb = torch.empty((batch,) + tuple(t_m.shape[1:]), dtype=torch.float32, device=dev)
    for s_ in range(steps):
        idx = torch.as_tensor(rng.choice(n_valid, size=batch, replace=False), device=dev)
        xb = x.index_select(0, idx).contiguous()
        vec_scale(t_m.index_select(0, idx).contiguous(), k, mb)
        wb = t_w.index_select(0, idx).contiguous()
        step = step0 + s_
        want = log_every > 0 and step % log_every == 0
        loss = net.train_step(xb, mb, wb, tp, want_loss=want)
        if want:
            losses.append(loss)
            print(f"[warmstart] step {step} loss {loss:.5f}", file=sys.stderr, flush=True)
    return step0 + steps


def train(net: UNet, lab: Labels, epochs: int, batch: int, tp: TrainParams, seed: int = 0,
          log_every: int = 0, m_scale: Optional[float] = None) -> WarmStart:
    """Shuffled mini-batch AdamW training on resident labels; returns the
    warm start (network and model-label scale)."""
    rng = np.random.default_rng(seed)
    N = lab.x.shape[0]
    k = model_label_scale(lab.t_m) if m_scale is None else m_scale
    losses: List[float] = []
    step = 0
    for _ in range(epochs):
        step = _train_steps(net, lab.x, lab.t_m, lab.t_w, N, N // batch, batch, tp, k, rng, losses, log_every,
                            step)
    return WarmStart(net, k, {"losses": losses, "steps": step})


def train_streaming(plan: Plan, net: UNet, gathers: Iterable[np.ndarray], n_total: int, params: Params,
                    tp: TrainParams, buffer: int = 512, chunk: int = 128, passes: float = 3.0, batch: int = 4,
                    seed: int = 0, log_every: int = 0) -> WarmStart:
    """Rolling generate -> label -> train: gathers arrive from an iterator
    (drawn on host workers while the GPU works), are labelled by the plain
    solve in chunks into a resident ring buffer of `buffer` gathers (the
    oldest labels are overwritten), and after each chunk the network takes
    passes * chunk / batch steps on mini-batches drawn from the buffer, so
    every label is used about `passes` times in expectation however large
    n_total is.  The model-label scale comes from the first chunk."""
    import time
    dev = plan.device
    rng = np.random.default_rng(seed)
    it = iter(gathers)
    first = next(it)
    H, W = first.shape
    x = torch.empty((buffer, H, W), dtype=torch.float32, device=dev)
    t_m = torch.empty((buffer, plan.npanel, H, W), dtype=torch.float32, device=dev)
    t_w = torch.empty((buffer, H, W), dtype=torch.float32, device=dev)
    pending = deque([first])
    losses: List[float] = []
    k = None
    filled = 0
    head = 0
    done = 0
    step = 0
    t_label = t_train = 0.0
    while done < n_total:
        n = min(chunk, n_total - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            g = pending.popleft() if pending else next(it)
            d = torch.tensor(g, dtype=torch.float32, device=dev)
            label_one(plan, d, params, x[head], t_m[head], t_w[head])
            head = (head + 1) % buffer
            filled = min(filled + 1, buffer)
        torch.cuda.synchronize()
        t_label += time.perf_counter() - t0
        done += n
        if k is None:
            k = model_label_scale(t_m[:filled])
        t0 = time.perf_counter()
        steps = max(1, int(round(passes * n / batch)))
        step = _train_steps(net, x, t_m, t_w, filled, steps, batch, tp, k, rng, losses, log_every, step)
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t0
        print(f"[warmstart] labelled {done}/{n_total} gathers, {step} training steps", file=sys.stderr, flush=True)
    return WarmStart(net, k, {"losses": losses, "steps": step, "label_s": t_label, "train_s": t_train,
                              "gathers": n_total, "buffer": buffer})


def predict(ws: WarmStart, d: torch.Tensor):
    """(m0, w0) for one gather d [nx][nt]."""
    s = gather_scale(d)
    x = vec_scale(d, 1.0 / s)[None].contiguous()
    y_m, y_w = ws.net.forward(x)
    return vec_scale(y_m[0], s / ws.m_scale), y_w[0]


def lp_misfit(plan: Plan, d: torch.Tensor, m: torch.Tensor, p: int) -> float:
    y = plan.forward(m)
    return vec_stats(d, y, 1.0, p)[0]


def warm_solve(plan: Plan, ws: WarmStart, d: torch.Tensor, params: Params, use_weights: bool = True,
               use_model: bool = True):
    """Warm-started robust solve.  The predicted model, scaled by its
    least-squares step length, is kept only if it fits the data better than
    m = 0 in the l_p misfit; otherwise the solve starts from zero, with the
    predicted weights if use_weights.  use_model False skips the model
    (weights only: an ablation).  Returns (m, d_rec, report, start) with
    start "model+weights" ("model"), "weights" or "plain"."""
    m0, w0 = predict(ws, d)
    w = w0.contiguous() if use_weights else None
    alpha, fit, zero = 0.0, 0.0, 0.0
    if use_model:
        y = plan.forward(m0)
        _, dy, yy = vec_stats(d, y, 1.0, params.p)
        alpha = max(dy / yy, 0.0) if yy > 0 else 0.0
        fit = vec_stats(d, y, alpha, params.p)[0]
        zero = vec_stats(d, None, 0.0, params.p)[0]
    if alpha > 0 and fit < zero:
        vec_scale(m0, alpha, m0)
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
                    ws: Optional[WarmStart] = None, max_outer: Optional[int] = None, slack_db: float = 0.05,
                    use_weights: bool = True):
    """Smallest outer-iteration count whose separated gather reaches
    target_db - slack_db, for the plain (ws None) or warm-started solve.
    Returns (k or None, Q_R at k, wall seconds of that solve including the
    network's inference and the start check, start kind)."""
    import time
    kmax = max_outer or params.n_outer
    q, dt, start = float("nan"), 0.0, "plain"
    for k in range(1, kmax + 1):
        prm = Params(**{**params.__dict__, "n_outer": k})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if ws is None:
            _, d_rec, _ = plan.robust_invert(d, prm, want_report=False)
        else:
            _, d_rec, _, start = warm_solve(plan, ws, d, prm, use_weights=use_weights)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        q = q_db(clean, d_rec.cpu().numpy())
        if q >= target_db - slack_db:
            return k, q, dt, start
    return None, q, dt, start
