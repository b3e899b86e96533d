"""Pins of the FP64 oracle's robust inversion (thesis Chapter 4).

Fixed against: the constants the thesis prints (tests/golden/), the normal
distribution (MAD / 0.6745 estimates sigma), Krylov-subspace least squares
computed by dense linear algebra (CGLS), the majorize-minimize property of
IRLS on the Huber objective (monotone decrease with a frozen clip), the
convex optimum found by an independent optimiser (scipy L-BFGS), and the
thesis' qualitative claim that the l1 misfit beats l2 under blending
interference (Chapter 4 conclusions).
"""
import os

import numpy as np
import pytest
import scipy.optimize

import oracle
from oracle import irls as I
from synth import workload, make_gather

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_pairs(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


def test_constants_match_thesis():
    c = _read_pairs("irls_constants.txt")
    assert I.B_R == c["b_r"]
    assert I.MAD_TO_SIGMA == c["mad_to_sigma"]
    assert I.EPS_M_DIVISOR == c["eps_m_divisor"]
    assert I.TOLERANCE == c["tolerance"]
    assert I.IrlsParams().b_r == c["b_r"]


def test_quality_metric_worked_examples():
    with open(os.path.join(GOLD, "quality_example.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    for row in rows:
        a, b, q = row.split(";")
        do = np.array([float(v) for v in a.split()])
        dr = np.array([float(v) for v in b.split()])
        assert oracle.q_db(do, dr) == pytest.approx(float(q), abs=1e-12)


def test_mad_estimates_sigma():
    rng = np.random.default_rng(11)
    for sigma in (0.3, 2.0):
        x = rng.normal(1.7, sigma, 1_000_000)
        assert abs(I.mad(x) / I.MAD_TO_SIGMA - sigma) < 0.01 * sigma


def test_mad_even_count_and_absolute_value():
    # median of [1,2,3,10] = 2.5; |x - 2.5| = [1.5, .5, .5, 7.5] -> median 1.0
    assert I.mad([1.0, 2.0, 3.0, 10.0]) == 1.0
    # the absolute value matters: without it the deviations' median would be 0
    assert I.mad([-5.0, -1.0, 0.0, 1.0, 5.0]) == 1.0


def test_huber_pieces():
    eps = 2.0
    assert I.huber([1.0], eps) == pytest.approx(0.25)       # r^2 / (2 eps)
    assert I.huber([5.0], eps) == pytest.approx(4.0)        # |r| - eps / 2
    assert I.huber([2.0], eps) == pytest.approx(1.0)        # continuous at |r| = eps


def _krylov_ls(A, b, k):
    """argmin_{x in K_k(A'A, A'b)} ||b - A x|| by dense linear algebra."""
    v = A.T @ b
    basis = []
    for _ in range(k):
        for q in basis:           # Gram-Schmidt, twice
            v = v - (q @ v) * q
        for q in basis:
            v = v - (q @ v) * q
        nrm = np.linalg.norm(v)
        if nrm < 1e-14:
            break
        q = v / nrm
        basis.append(q)
        v = A.T @ (A @ q)
    Q = np.array(basis).T
    c, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    return Q @ c


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_cgls_equals_krylov_least_squares_random(k):
    rng = np.random.default_rng(12)
    A = rng.standard_normal((30, 12))
    b = rng.standard_normal(30)
    x, it = I.cgls(lambda u: A @ u, lambda r: A.T @ r, b, np.zeros(12), k)
    np.testing.assert_allclose(x, _krylov_ls(A, b, k), rtol=1e-9, atol=1e-10)


def test_cgls_on_explicit_stolt_operator():
    # a tiny Stolt operator written out column by column
    g = oracle.geometry(12, 6, 0.004, 12.5, [1500.0, 3000.0], fmax=90.0)
    n = g.npanel * g.nx * g.nt
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(oracle.forward(g, e.reshape(g.npanel, g.nx, g.nt)).ravel())
    Lmat = np.array(cols).T
    rng = np.random.default_rng(13)
    d = rng.standard_normal(g.nx * g.nt)
    for k in (1, 3, 6):
        x, _ = I.cgls(lambda u: oracle.forward(g, u.reshape(g.npanel, g.nx, g.nt)).ravel(),
                      lambda r: oracle.adjoint(g, r.reshape(g.nx, g.nt)).ravel(),
                      d, np.zeros(n), k)
        np.testing.assert_allclose(x, _krylov_ls(Lmat, d, k), rtol=1e-8, atol=1e-9)
    # the residual norm decreases monotonically along the iterations
    res = []
    for k in range(1, 15):
        x, _ = I.cgls(lambda u: Lmat @ u, lambda r: Lmat.T @ r, d, np.zeros(n), k)
        res.append(np.linalg.norm(d - Lmat @ x))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:]))


def _explicit_problem(seed, m=60, n=25, n_out=8):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    x_true = rng.standard_normal(n)
    d = A @ x_true + 0.05 * rng.standard_normal(m)
    idx = rng.choice(m, n_out, replace=False)
    d[idx] += rng.choice([-1, 1], n_out) * rng.uniform(5, 20, n_out)
    return A, d


def test_irls_huber_objective_is_monotone_with_frozen_clip():
    A, d = _explicit_problem(14)
    prm = I.IrlsParams(p=1, q=2, n_outer=12, n_inner=3, freeze_eps=True)
    d2 = d.reshape(1, -1)
    _, _, rep = I.robust_invert(None, d2, prm,
                                Lop=lambda u: (A @ u.ravel()).reshape(1, -1),
                                LTop=lambda r: A.T @ r.ravel())
    h = rep["huber"]
    assert len(set(rep["eps_r"])) == 1
    for a, b in zip(h, h[1:]):
        assert b <= a * (1 + 1e-12)
    assert h[-1] < h[0]


def test_irls_reaches_convex_huber_optimum():
    A, d = _explicit_problem(15)
    prm = I.IrlsParams(p=1, q=2, n_outer=300, n_inner=25, freeze_eps=True)
    d2 = d.reshape(1, -1)
    x, _, rep = I.robust_invert(None, d2, prm,
                                Lop=lambda u: (A @ u.ravel()).reshape(1, -1),
                                LTop=lambda r: A.T @ r.ravel())
    eps = rep["eps_r"][0]

    def f(z):
        r = d - A @ z
        a = np.abs(r)
        val = np.sum(np.where(a <= eps, a * a / (2 * eps), a - eps / 2))
        psi = np.where(a <= eps, r / eps, np.sign(r))
        return val, -A.T @ psi

    res = scipy.optimize.minimize(f, np.zeros(A.shape[1]), jac=True, method="L-BFGS-B",
                                  options={"maxiter": 10000, "gtol": 1e-13, "ftol": 1e-15})
    assert rep["huber"][-1] == pytest.approx(res.fun, rel=1e-6)


def test_least_squares_case_matches_normal_equations():
    # p = q = 2 with enough CG iterations is plain least squares
    A, d = _explicit_problem(16, n_out=0)
    prm = I.IrlsParams(p=2, q=2, n_outer=1, n_inner=25)
    x, _, rep = I.robust_invert(None, d.reshape(1, -1), prm,
                                Lop=lambda u: (A @ u.ravel()).reshape(1, -1),
                                LTop=lambda r: A.T @ r.ravel())
    np.testing.assert_allclose(x.ravel(), np.linalg.lstsq(A, d, rcond=None)[0], rtol=1e-7, atol=1e-9)
    assert rep["eps_r"] == [0.0]


def test_tolerance_stops_early():
    A, d = _explicit_problem(17)
    prm = I.IrlsParams(p=1, q=2, n_outer=50, n_inner=25, tol=0.01)
    _, _, rep = I.robust_invert(None, d.reshape(1, -1), prm,
                                Lop=lambda u: (A @ u.ravel()).reshape(1, -1),
                                LTop=lambda r: A.T @ r.ravel())
    assert rep["outer_done"] < 50
    m = rep["misfit"]
    assert abs(m[-1] - m[-2]) / m[-2] < 0.01


def test_dead_traces_do_not_influence_solution():
    w = workload("crg-256x64-nv8", nt=64, nx=24, vel=(1500.0, 2500.0), tau0=(0, 0),
                 n_outer=2, n_inner=3)
    gth = make_gather(w)
    g = oracle.geometry(gth.nt, gth.nx, w.dt, w.dx, w.vel, fmax=w.fmax)
    mask = np.ones(gth.nx, np.uint8)
    mask[[3, 7, 11]] = 0
    prm = I.IrlsParams(p=1, q=1, n_outer=2, n_inner=3)
    d1 = gth.d_blend.copy()
    d2 = d1.copy()
    d2[[3, 7, 11]] = 123.0
    m1, _, _ = I.robust_invert(g, d1, prm, mask=mask)
    m2, _, _ = I.robust_invert(g, d2, prm, mask=mask)
    np.testing.assert_allclose(m1, m2, atol=1e-12)


@pytest.mark.slow
def test_l1_misfit_beats_l2_on_blended_small_gather():
    # Chapter 4 conclusions: the robust (p = 1) misfit removes blending noise
    # better than least squares; directional check on the small workload.
    w = workload("crg-256x64-nv8")
    gth = make_gather(w)
    g = oracle.geometry(gth.nt, gth.nx, w.dt, w.dx, w.vel, fmax=w.fmax)
    q_pd = oracle.q_db(gth.d_clean, gth.d_blend)
    out = {}
    for p in (1, 2):
        prm = I.IrlsParams(p=p, q=2, n_outer=w.n_outer, n_inner=w.n_inner)
        _, drec, _ = I.robust_invert(g, gth.d_blend, prm)
        out[p] = oracle.q_db(gth.d_clean, drec)
    assert out[1] > out[2]
    assert out[1] > q_pd
