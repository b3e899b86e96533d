"""The CG recurrence the GPU solver runs for q = 1, checked on the CPU.

The thesis' inner solve is CGLS on A = W_r S L W_m^-1 in the variable
u = W_m m (Chapter 4, the reweighted system).  The GPU keeps the same
recurrence in model space: m = W_m^-1 u, pdir' = W_m^-1 pdir and
g' = W_m^-1 g, so the forward applies W_r S L to pdir' with no model weight
and the adjoint applies W_m^-2, with gamma = |W_m^-1 L' S W_r s|^2.  This test
runs both forms in FP64 on a small explicit system and requires the iterates
to agree (m_k = W_m^-1 u_k) together with the step scalars."""
import numpy as np
import pytest


def _system(seed, nd=40, nm=25):
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((nd, nm))
    S = np.diag((rng.uniform(size=nd) > 0.2).astype(float))     # sampling
    Wr = np.diag(rng.uniform(0.3, 2.0, nd))                      # residual weights
    winv = rng.uniform(0.2, 3.0, nm)                              # W_m^-1 (diagonal)
    d = rng.standard_normal(nd)
    m0 = rng.standard_normal(nm) * 0.1
    return L, S, Wr, winv, d, m0


def _cgls_u(L, S, Wr, winv, d, m0, n):
    """Textbook CGLS on A = W_r S L W_m^-1 from u0 = W_m m0."""
    A = Wr @ S @ L @ np.diag(winv)
    u = m0 / winv
    s = Wr @ S @ (d - L @ m0)
    g = A.T @ s
    p = g.copy()
    gam = g @ g
    out = []
    for _ in range(n):
        q = A @ p
        alpha = gam / (q @ q)
        u = u + alpha * p
        s = s - alpha * q
        g = A.T @ s
        gnew = g @ g
        p = g + (gnew / gam) * p
        gam = gnew
        out.append((winv * u, alpha, gam))
    return out


def _cgls_model_space(L, S, Wr, winv, d, m0, n):
    """The same recurrence with m, pdir' = W_m^-1 pdir and g' = W_m^-1 g."""
    m = m0.copy()
    s = Wr @ S @ (d - L @ m0)
    y = L.T @ (S @ (Wr @ s))
    gp = winv * winv * y                 # g' = W_m^-2 L' S W_r s
    gam = np.sum((winv * y) ** 2)        # |g|^2 = |W_m^-1 L' S W_r s|^2
    pp = gp.copy()
    out = []
    for _ in range(n):
        q = Wr @ (S @ (L @ pp))          # forward without a model weight
        alpha = gam / (q @ q)
        m = m + alpha * pp
        s = s - alpha * q
        y = L.T @ (S @ (Wr @ s))
        gp = winv * winv * y
        gnew = np.sum((winv * y) ** 2)
        pp = gp + (gnew / gam) * pp
        gam = gnew
        out.append((m.copy(), alpha, gam))
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_model_space_recurrence_equals_u_space_cgls(seed):
    L, S, Wr, winv, d, m0 = _system(seed)
    a = _cgls_u(L, S, Wr, winv, d, m0, 12)
    b = _cgls_model_space(L, S, Wr, winv, d, m0, 12)
    for (mu, al_u, g_u), (mm, al_m, g_m) in zip(a, b):
        np.testing.assert_allclose(mm, mu, rtol=1e-9, atol=1e-12)
        assert abs(al_m / al_u - 1) < 1e-9
        assert abs(g_m / g_u - 1) < 1e-9


def test_model_space_recurrence_reaches_the_weighted_least_squares_solution():
    """After nm iterations CGLS has (up to rounding) the minimiser of
    |W_r S (d - L m)|^2 over m = W_m^-1 u, i.e. the normal equations hold."""
    L, S, Wr, winv, d, m0 = _system(5, nd=30, nm=12)
    m = _cgls_model_space(L, S, Wr, winv, d, m0, 40)[-1][0]
    r = Wr @ S @ (d - L @ m)
    grad = np.diag(winv) @ L.T @ S @ Wr @ r
    assert np.linalg.norm(grad) < 1e-8 * np.linalg.norm(np.diag(winv) @ L.T @ S @ Wr @ Wr @ S @ d)
