"""Pins of the FISTA oracle (oracle/fista.py) on an explicit tiny Stolt
operator (built column by column from the oracle's forward):

* the power-method eigenvalue against LAPACK's eigvalsh of L' S L;
* the FISTA minimiser's objective against scikit-learn's coordinate-descent
  Lasso on the same explicit matrix (independent algorithm and library);
* soft thresholding against its closed form at a few points.
"""
import numpy as np
import pytest

import oracle
from oracle import fista as F

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def _explicit(g, mask):
    n = g.npanel * g.nx * g.nt
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(oracle.forward(g, e.reshape(g.npanel, g.nx, g.nt), mask).ravel())
    return np.stack(cols, axis=1)


@pytest.fixture(scope="module")
def tiny():
    g = oracle.geometry(24, 8, 0.004, 12.5, [1500.0, 2600.0], fmax=120.0)
    mask = np.array([1, 1, 0, 1, 1, 1, 0, 1], np.uint8)
    return g, mask, _explicit(g, mask)


def test_soft_threshold():
    v = np.array([-3.0, -0.5, 0.0, 0.2, 2.0])
    assert np.allclose(F.soft(v, 1.0), [-2.0, 0.0, 0.0, 0.0, 1.0])


def test_power_method_matches_eigvalsh(tiny):
    g, mask, A = tiny
    lam = F.power_lambda(g, mask, 3000)  # clustered top eigenvalues: slow convergence
    ev = np.linalg.eigvalsh(A.T @ A)[-1]
    assert abs(lam - ev) <= 1e-6 * ev


def test_fista_reaches_the_lasso_optimum(tiny):
    from sklearn.linear_model import Lasso
    g, mask, A = tiny
    rng = np.random.default_rng(3)
    mt = np.zeros(A.shape[1])
    mt[rng.choice(A.shape[1], 12, replace=False)] = rng.standard_normal(12)
    d = (A @ mt + 0.01 * rng.standard_normal(A.shape[0])).reshape(g.nx, g.nt)
    prm = F.FistaParams(n_iter=3000, n_power=300, mu_rel=0.05)
    m, _, rep = F.fista(g, d, prm, mask=mask)
    # sklearn: (1 / (2 n)) ||y - X w||^2 + alpha ||w||_1  ==  J / (2 n) with alpha = mu / (2 n)
    n = A.shape[0]
    y = (d * mask[:, None]).ravel()
    las = Lasso(alpha=rep["mu"] / (2 * n), fit_intercept=False, max_iter=200000, tol=1e-12)
    las.fit(A, y)
    w = las.coef_
    j_ref = float(np.sum((y - A @ w) ** 2) + rep["mu"] * np.sum(np.abs(w)))
    assert rep["objective"] <= j_ref * (1 + 1e-6)
    assert abs(rep["objective"] - j_ref) <= 1e-5 * j_ref
