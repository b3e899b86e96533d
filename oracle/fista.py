"""FP64 oracle of the l2-l1 sparse inversion by FISTA (thesis Chapter 6,
section "Sparse inversion", equation cost_fn with p = 2, q = 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Minimises J(m) = ||d - S L m||_2^2 + mu ||m||_1:

* the largest eigenvalue of L' S L by the power (Rayleigh) method from the
  all-ones model, n_power iterations, lambda = ||L' S L x|| with ||x|| = 1;
* Lipschitz constant of grad ||d - S L m||^2 = 2 L' S (S L m - d):
  Lf = 2 * lambda * lip_safety (the power method approaches lambda from
  below; the safety factor keeps the step within 1/Lf);
* mu given, or mu = mu_rel * max|2 L' S d| (the smallest mu for which m = 0
  is optimal, scaled by mu_rel);
* FISTA (Beck and Teboulle): m_k = soft(y_k + (2/Lf) L' S (d - L y_k), mu/Lf),
  t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, y_{k+1} = m_k + ((t_k - 1)/t_{k+1})
  (m_k - m_{k-1}), from y_1 = m_0, t_1 = 1.

Readings (the thesis names the algorithm and the power method only): the
all-ones start vector, the safety factor 1.05, the mu_rel rule.
"""
from dataclasses import dataclass

import numpy as np

from . import stolt


@dataclass
class FistaParams:
    n_iter: int = 50
    n_power: int = 20
    mu: float = 0.0          # > 0: used as is
    mu_rel: float = 0.05     # otherwise mu = mu_rel * max|2 L' S d|
    lip_safety: float = 1.05


def soft(v, tau):
    return np.sign(v) * np.maximum(np.abs(v) - tau, 0.0)


def power_lambda(g, mask, n_power):
    """Largest eigenvalue of L' S L by the power method from the all-ones model."""
    x = np.ones((g.npanel, g.nx, g.nt))
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(n_power):
        z = stolt.adjoint(g, stolt.forward(g, x, mask), mask)
        lam = float(np.linalg.norm(z))
        if lam == 0.0:
            break
        x = z / lam
    return lam


def fista(g, d, prm: FistaParams, mask=None, m0=None, Lop=None, LTop=None):
    """Returns (m, L m, report).  Lop / LTop override the operator pair (tests)."""
    fwd = Lop or (lambda m: stolt.forward(g, m, mask))
    adj = LTop or (lambda r: stolt.adjoint(g, r, mask))
    d = np.asarray(d, np.float64)
    if mask is not None:
        d = d * np.asarray(mask)[:, None]
    if Lop is None:
        lam = power_lambda(g, mask, prm.n_power)
    else:
        x = np.ones_like(adj(d))
        x /= np.linalg.norm(x)
        lam = 0.0
        for _ in range(prm.n_power):
            z = adj(fwd(x))
            lam = float(np.linalg.norm(z))
            if lam == 0.0:
                break
            x = z / lam
    lf = 2.0 * lam * prm.lip_safety
    mu = prm.mu if prm.mu > 0 else prm.mu_rel * float(np.max(np.abs(2.0 * adj(d))))
    m = np.zeros_like(adj(d)) if m0 is None else np.asarray(m0, np.float64).copy()
    y = m.copy()
    t = 1.0
    for _ in range(prm.n_iter):
        if lf == 0.0:
            break
        m_new = soft(y + (2.0 / lf) * adj(d - fwd(y)), mu / lf)
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        y = m_new + ((t - 1.0) / t_new) * (m_new - m)
        m, t = m_new, t_new
    r = d - fwd(m)
    misfit = float(np.sum(r * r))
    l1 = float(np.sum(np.abs(m)))
    rep = {"lipschitz": lf, "mu": mu, "misfit": misfit, "l1": l1, "objective": misfit + mu * l1,
           "iters": prm.n_iter}
    Lm = stolt.forward(g, m, None) if Lop is None else fwd(m)
    return m, Lm, rep
