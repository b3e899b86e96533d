"""FP64 oracle of the robust Radon inversion: IRLS outer loop, CGLS inner loop.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Thesis Chapter 4, "Robust Radon transform":

* cost J = ||d - L m||_p^p + mu ||m||_q^q (equation ch4_cost_fn);
* a p-norm as a weighted 2-norm, [W_x]_ii = |x_i|^{(p-2)/2}, with the weights
  clipped below eps_r (residual) and eps_m (model);
* eps_r = b_r * MAD(r) / 0.6745 with b_r = 1.345 (equation ch4_epcilon_r),
  MAD the median absolute deviation (the printed formula drops the absolute
  value; the standard definition median(|r - median(r)|) it cites is used);
* eps_m = b_m * max|m| / 100;
* change of variables u = W_m m (equation equ:11), mu = 0 and the number of
  CG iterations as the regulariser; an inner CG loop on the weighted system
  and an outer loop that updates the weights; stop when the misfit change is
  below a tolerance (0.01 in the thesis) or at the iteration limit.

Readings (where the thesis is silent):

* "|x_i| > eps" in the clipped weights, i.e. W = max(|x|, eps)^{(p-2)/2};
* eps_r is floored at eps_floor_rel * max|d_live| so it cannot collapse to 0;
* outer iteration 1 is unweighted (W_r = 1 on live samples, W_m = 1) unless
  an initial weight w0 is given, in which case W_r = w0;
* each CGLS run starts from the current model (u0 = W_m m) with fresh
  search directions;
* the "misfit" whose relative change is tested is sum_live |r_i|^p;
* the sampling mask S multiplies the residual (interpolation, Chapter 6).
"""
from dataclasses import dataclass

import numpy as np

from .stolt import Geometry, forward, adjoint

B_R = 1.345          # Holland & Welsch tuning constant (Chapter 4)
MAD_TO_SIGMA = 0.6745
EPS_M_DIVISOR = 100.0
TOLERANCE = 0.01


@dataclass
class IrlsParams:
    p: int = 1
    q: int = 2
    n_outer: int = 10
    n_inner: int = 20
    b_r: float = B_R
    b_m: float = 1.0
    tol: float = 0.0
    eps_floor_rel: float = 1e-6
    freeze_eps: bool = False


def mad(x):
    """Median absolute deviation about the median (numpy median: even n -> mean of middles)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    return float(np.median(np.abs(x - np.median(x))))


def eps_r(r_live, b_r=B_R, floor=0.0):
    return max(b_r * mad(r_live) / MAD_TO_SIGMA, floor)


def huber(r, eps):
    """Huber objective sum rho_eps(r_i); rho = r^2/(2 eps) for |r| <= eps, |r| - eps/2 beyond."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    return float(np.sum(np.where(a <= eps, a * a / (2.0 * eps), a - 0.5 * eps)))


def _clip_weight(x, eps, power):
    """max(|x|, eps)^((power-2)/2); power 2 gives ones."""
    if power == 2:
        return np.ones_like(x)
    if eps <= 0:
        return np.ones_like(x)
    return np.maximum(np.abs(x), eps) ** ((power - 2) / 2.0)


def cgls(A, AT, b, u0, n_iter):
    """Conjugate gradients on the normal equations (CGLS) from the start u0.

    Returns (u, iterations run).  Stops early if the gradient or the
    step-length denominator is exactly zero.
    """
    u = u0.copy()
    s = b - A(u)
    g = AT(s)
    pdir = g.copy()
    gamma = float(np.vdot(g, g).real)
    it = 0
    for _ in range(n_iter):
        if gamma == 0.0:
            break
        qv = A(pdir)
        delta = float(np.vdot(qv, qv).real)
        if delta == 0.0:
            break
        alpha = gamma / delta
        u = u + alpha * pdir
        s = s - alpha * qv
        g = AT(s)
        gamma_new = float(np.vdot(g, g).real)
        pdir = g + (gamma_new / gamma) * pdir
        gamma = gamma_new
        it += 1
    return u, it


def robust_invert(g: Geometry, d, params: IrlsParams, mask=None, m0=None, w0=None,
                  Lop=None, LTop=None):
    """IRLS with CGLS inner solves.  Returns (m, d_rec, report).

    ``report`` holds, per completed outer iteration k (after its CGLS):
    ``misfit`` = sum_live |r_k|^p with r_k = S(d - L m_k); ``eps_r`` = the
    residual clip computed from r_k (or the frozen one; 0 when p = 2);
    ``huber`` = the Huber objective of r_k at that eps_r (for p = 2 the
    least-squares objective sum r^2 / 2); ``inner`` = CG iterations run.
    ``Lop``/``LTop`` override the operator pair (for tests on explicit matrices).
    """
    d = np.asarray(d, dtype=np.float64)
    nx, nt = d.shape
    live = np.ones(nx, bool) if mask is None else (np.asarray(mask) != 0)
    S = live.astype(np.float64)[:, None] * np.ones((1, nt))
    Lf = Lop if Lop is not None else (lambda m: forward(g, m))
    LTf = LTop if LTop is not None else (lambda x: adjoint(g, x))
    mshape = (g.npanel, g.nx, g.nt) if Lop is None else np.shape(LTf(np.zeros_like(d)))
    m = np.zeros(mshape) if m0 is None else np.asarray(m0, dtype=np.float64).copy()
    dmax = float(np.max(np.abs(d[live]))) if live.any() else 0.0
    floor = params.eps_floor_rel * dmax

    rep = {"misfit": [], "eps_r": [], "huber": [], "inner": [], "eps_m": []}
    Lm = Lf(m)
    r = S * (d - Lm)
    eps_frozen = None
    for k in range(1, params.n_outer + 1):
        # weights for this outer iteration
        if k == 1:
            Wr = S.copy() if w0 is None else S * np.asarray(w0, np.float64)
            Wm = np.ones_like(m)
        else:
            e = rep["eps_r"][-1]
            Wr = S * _clip_weight(r, e, params.p)
            if params.q == 1:
                em = params.b_m * float(np.max(np.abs(m))) / EPS_M_DIVISOR
                rep["eps_m"].append(em)
                Wm = _clip_weight(m, em, params.q)
            else:
                Wm = np.ones_like(m)
        Wm_inv = 1.0 / Wm

        def A(u):
            return Wr * (S * Lf(Wm_inv * u))

        def AT(x):
            return Wm_inv * LTf(S * (Wr * x))

        b = Wr * (S * d)
        u, it = cgls(A, AT, b, Wm * m, params.n_inner)
        m = Wm_inv * u
        Lm = Lf(m)
        r = S * (d - Lm)
        r_live = r[live]
        rep["misfit"].append(float(np.sum(np.abs(r_live) ** params.p)))
        if params.p == 2:
            # no residual clip is needed; report the least-squares objective
            e = 0.0
            obj = 0.5 * float(np.sum(r_live * r_live))
        else:
            if params.freeze_eps and eps_frozen is not None:
                e = eps_frozen
            else:
                e = eps_r(r_live, params.b_r, floor)
                if params.freeze_eps:
                    eps_frozen = e
            obj = huber(r_live, e) if e > 0 else float(np.sum(np.abs(r_live)))
        rep["eps_r"].append(e)
        rep["huber"].append(obj)
        rep["inner"].append(it)
        if params.tol > 0 and k >= 2:
            prev = rep["misfit"][-2]
            if prev > 0 and abs(rep["misfit"][-1] - prev) / prev < params.tol:
                break
    rep["outer_done"] = len(rep["misfit"])
    return m, Lm, rep
