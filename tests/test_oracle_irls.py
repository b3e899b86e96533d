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


# --------------------------------------------------------------------------
# Pins of the model-weight branch (q = 1) and of the initial weight w0.
#
# Chapter 4's reweighted system: CG on A = W_r S L W_m^-1 in u = W_m m,
# with eps_m = b_m max|m| / 100 and W_m = max(|m|, eps_m)^((q-2)/2).  Run to
# convergence, CGLS from a start u0 returns u0 + A^+ (b - A u0), so each
# outer step has a closed form that fixes where every weight goes:
#
# * underdetermined, consistent L (more model than data samples): the data
#   are fitted exactly and the step is the smallest change of m in the
#   W_m-norm,  m_k = m_{k-1} + D L'(L D L')^-1 (d - L m_{k-1}),
#   D = W_m^-2 = diag(max(|m_{k-1}|, eps_m)) for q = 1 -- independent of W_r;
# * overdetermined, full column rank L: m_k is the weighted least-squares
#   solution argmin |W_r S (d - L m)|, whatever W_m is (a change of
#   variables does not move the minimiser).
#
# Each mistake in the branch changes one of these: eps_m taken from u = W_m m
# instead of m, a wrong divisor, W_m and W_m^-1 swapped, a start other than
# u0 = W_m m, a residual weight other than w0 in outer iteration 1.


def _explicit_ops(L):
    # data laid out as nd traces of one sample, so the trace mask selects samples
    return (lambda u: (L @ np.ravel(u)).reshape(-1, 1)), (lambda r: L.T @ np.ravel(r))


def _run_explicit(L, d, prm, m0=None, w0=None, mask=None):
    Lop, LTop = _explicit_ops(L)
    return I.robust_invert(None, d.reshape(-1, 1), prm, m0=m0,
                           w0=None if w0 is None else w0.reshape(-1, 1),
                           mask=mask, Lop=Lop, LTop=LTop)


def test_eps_m_hand_example():
    # L = identity: one CG step from m0 = 0 reproduces d exactly (alpha = 1),
    # so outer iteration 2 sees m = d and eps_m = b_m * max|d| / 100 by hand
    d = np.array([3.0, -200.0, 0.5, 1.0])
    for b_m, want in ((1.0, 2.0), (3.0, 6.0)):
        prm = I.IrlsParams(p=2, q=1, n_outer=2, n_inner=1, b_m=b_m)
        m, _, rep = _run_explicit(np.eye(4), d, prm)
        assert rep["eps_m"] == [pytest.approx(want, rel=1e-15)]
        np.testing.assert_allclose(m, d, rtol=1e-15)   # zero residual: no further step


def _underdetermined(seed, nd=12, nm=30, rank=None):
    rng = np.random.default_rng(seed)
    if rank is None:
        L = rng.standard_normal((nd, nm))
    else:   # rank-deficient: no exact fit, and a null space in model space
        L = rng.standard_normal((nd, rank)) @ rng.standard_normal((rank, nm)) / np.sqrt(rank)
    d = rng.standard_normal(nd)
    d[3] += 25.0                                   # an outlier sample (p = 1 reweights it)
    m0 = rng.standard_normal(nm) * 0.3
    return L, d, m0


@pytest.mark.parametrize("b_m", [1.0, 10.0])
def test_q1_converged_steps_are_weighted_pseudo_inverse_steps(b_m):
    # rank-deficient L: every outer step leaves a residual (so the weights of
    # the next one act) and keeps the start's null-space component, so the
    # converged step m_k = m_{k-1} + W_m^-1 (W_r S L W_m^-1)^+ W_r S r_{k-1}
    # depends on eps_r, eps_m, the placement of both weights and u0 = W_m m
    rank = 8
    L, d, m0 = _underdetermined(21, nd=14, nm=30, rank=rank)
    nd, nm = L.shape
    live = np.ones(nd, bool)
    live[[6, 11]] = False
    S = live.astype(float)
    n_outer = 4
    prm = I.IrlsParams(p=1, q=1, n_outer=n_outer, n_inner=4 * rank, b_m=b_m)
    ms = [_run_explicit(L, d, I.IrlsParams(**{**prm.__dict__, "n_outer": k}), m0=m0,
                        mask=live.astype(np.uint8))[0].ravel()
          for k in range(1, n_outer + 1)]
    dmax = np.max(np.abs(d[live]))
    ref, alt = [m0], [m0]
    clipped = 0
    for k in range(1, n_outer + 1):
        for seq, weighted in ((ref, True), (alt, False)):
            mp = seq[-1]
            r = S * (d - L @ mp)
            if k == 1:
                wr, wm = S.copy(), np.ones(nm)
            else:
                rl = r[live]
                e = max(prm.b_r * np.median(np.abs(rl - np.median(rl))) / 0.6745,
                        prm.eps_floor_rel * dmax)
                wr = S / np.sqrt(np.maximum(np.abs(r), e))
                em = b_m * np.max(np.abs(mp)) / 100.0
                wm = 1.0 / np.sqrt(np.maximum(np.abs(mp), em)) if weighted else np.ones(nm)
                if weighted:
                    clipped += int(np.sum(np.abs(mp) < em))
            A = wr[:, None] * L / wm[None, :]
            seq.append(mp + (np.linalg.pinv(A, rcond=1e-10) @ (wr * r)) / wm)
    for k in range(n_outer):
        np.testing.assert_allclose(ms[k], ref[k + 1], rtol=1e-7, atol=1e-9)
    if b_m > 1.0:
        assert clipped > 0        # the clip eps_m took part
    # the model weights matter here: the same steps with W_m = 1 end elsewhere
    assert np.linalg.norm(ms[-1] - alt[-1]) > 1e-3 * np.linalg.norm(alt[-1])


def test_q1_eps_m_follows_the_model_not_u():
    # the stored eps_m of outer iteration k is b_m max|m_{k-1}| / 100 with
    # m_{k-1} the model the oracle returned after k-1 iterations
    L, d, m0 = _underdetermined(22)
    b_m = 4.0
    prm = I.IrlsParams(p=1, q=1, n_outer=4, n_inner=5, b_m=b_m)
    _, _, rep = _run_explicit(L, d, prm, m0=m0)
    for k in range(2, 5):
        mk, _, _ = _run_explicit(L, d, I.IrlsParams(**{**prm.__dict__, "n_outer": k - 1}), m0=m0)
        assert rep["eps_m"][k - 2] == pytest.approx(b_m * np.max(np.abs(mk)) / 100.0, rel=1e-13)


def _overdetermined(seed, nd=40, nm=10):
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((nd, nm))
    d = L @ rng.standard_normal(nm) + 0.05 * rng.standard_normal(nd)
    idx = rng.choice(nd, 6, replace=False)
    d[idx] += rng.choice([-1, 1], 6) * rng.uniform(5, 20, 6)
    return L, d


@pytest.mark.parametrize("q", [2, 1])
def test_converged_steps_are_weighted_least_squares(q):
    L, d = _overdetermined(23)
    nd, nm = L.shape
    live = np.ones(nd, bool)
    live[[5, 17, 30]] = False
    n_outer = 4
    prm = I.IrlsParams(p=1, q=q, n_outer=n_outer, n_inner=4 * nm)
    dmax = np.max(np.abs(d[live]))
    m = np.zeros(nm)
    for k in range(1, n_outer + 1):
        if k == 1:
            w = live.astype(float)
        else:
            r = (d - L @ m)[live]
            mad = np.median(np.abs(r - np.median(r)))
            e = max(prm.b_r * mad / 0.6745, prm.eps_floor_rel * dmax)
            w = np.zeros(nd)
            w[live] = 1.0 / np.sqrt(np.maximum(np.abs(r), e))
        m = np.linalg.lstsq(w[:, None] * L, w * d, rcond=None)[0]
        got = _run_explicit(L, d, I.IrlsParams(**{**prm.__dict__, "n_outer": k}),
                            mask=live.astype(np.uint8))[0].ravel()
        np.testing.assert_allclose(got, m, rtol=1e-8, atol=1e-10)


def test_w0_weights_the_first_outer_iteration():
    L, d = _overdetermined(24)
    nd, nm = L.shape
    w0 = np.random.default_rng(25).uniform(0.05, 1.0, nd)
    prm = I.IrlsParams(p=1, q=2, n_outer=1, n_inner=4 * nm)
    got = _run_explicit(L, d, prm, w0=w0)[0].ravel()
    want = np.linalg.lstsq(w0[:, None] * L, w0 * d, rcond=None)[0]
    np.testing.assert_allclose(got, want, rtol=1e-8, atol=1e-10)
    # W_r = w0, not w0^2 or sqrt(w0): those minimisers differ here
    for alt in (w0 ** 2, np.sqrt(w0)):
        other = np.linalg.lstsq(alt[:, None] * L, alt * d, rcond=None)[0]
        assert np.linalg.norm(other - want) > 1e-4 * np.linalg.norm(want)


def _krylov_ls_from(A, b, u0, k):
    """u0 + argmin over K_k(A'A, A'(b - A u0)) of |b - A u| (dense)."""
    return u0 + _krylov_ls(A, b - A @ u0, k)


def test_q1_partial_cg_equals_krylov_least_squares_on_the_weighted_system():
    # outer iteration 2 with three CG steps: the oracle's model equals the
    # Krylov-subspace least-squares solution of the explicitly assembled
    # W_r S L W_m^-1 system started at u0 = W_m m1
    L, d, m0 = _underdetermined(26, nd=20, nm=16)     # overdetermined-ish: no exact fit
    nd, nm = L.shape
    live = np.ones(nd, bool)
    live[[2, 9]] = False
    S = live.astype(float)
    b_m, k_in = 20.0, 3
    prm1 = I.IrlsParams(p=1, q=1, n_outer=1, n_inner=k_in, b_m=b_m)
    prm2 = I.IrlsParams(p=1, q=1, n_outer=2, n_inner=k_in, b_m=b_m)
    m1 = _run_explicit(L, d, prm1, m0=m0, mask=live.astype(np.uint8))[0].ravel()
    m2, _, rep = _run_explicit(L, d, prm2, m0=m0, mask=live.astype(np.uint8))
    # outer 1 (unweighted) against Krylov from m0
    A1 = S[:, None] * L
    np.testing.assert_allclose(m1, _krylov_ls_from(A1, S * d, m0, k_in), rtol=1e-9, atol=1e-11)
    # outer 2: weights from m1 and its residual
    r = (S * (d - L @ m1))[live]
    e = max(prm2.b_r * np.median(np.abs(r - np.median(r))) / 0.6745,
            prm2.eps_floor_rel * np.max(np.abs(d[live])))
    wr = np.zeros(nd)
    wr[live] = np.maximum(np.abs(r), e) ** -0.5
    em = b_m * np.max(np.abs(m1)) / 100.0
    wm = np.maximum(np.abs(m1), em) ** -0.5
    assert np.sum(np.abs(m1) < em) > 0
    A2 = (wr * S)[:, None] * L / wm[None, :]
    u2 = _krylov_ls_from(A2, wr * S * d, wm * m1, k_in)
    np.testing.assert_allclose(m2.ravel(), u2 / wm, rtol=1e-9, atol=1e-11)
    assert rep["eps_m"] == [pytest.approx(em, rel=1e-14)]
