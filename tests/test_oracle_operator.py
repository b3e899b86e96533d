"""Pins of the FP64 oracle's Stolt (A)ASHRT operator pair.

Each test fixes part of the oracle against something other than itself:
brute-force DFT sums, the dot-product identity, closed-form special cases
(v = 0, kx = 0), the dispersion relation of Chapter 5, the change-of-variables
factor C = w_tau / w of equation ch5_Stolt_adj, symmetries, and a brute-force
time-domain hyperbola summation (Chapter 3 table / Chapter 6 equations) for
the kinematics.  The Stolt amplitudes differ from the time-domain operator by
design, so only kinematics are compared there.
"""
import math

import numpy as np
import pytest
import scipy.signal

import oracle
from oracle import stolt as S
from oracle import timedomain as TD


def _rng(s):
    return np.random.default_rng(s)


# ---------------------------------------------------------------- sizes, kernel
def test_fft_len_rule():
    # smallest 2^a or 3*2^a >= 2n
    cases = {1: 2, 3: 6, 5: 12, 64: 128, 96: 192, 100: 256, 160: 384, 256: 512,
             320: 768, 1024: 2048, 1536: 3072, 2048: 4096}
    for n, want in cases.items():
        assert S.fft_len(n) == want, (n, S.fft_len(n), want)


def test_band_edges():
    g = oracle.geometry(1024, 256, 0.004, 12.5, [2000.0], fmax=100.0)
    assert (g.ntp, g.nxp) == (2048, 512)
    # 100 Hz * 2048 * 0.004 s = 819.2 bins -> 819; DC is never mapped
    assert S.band(g) == (1, 819)
    # 10 Hz * 128 * 0.004 s = 5.12 bins -> first mapped bin 6; fmax <= 0: up to Nyquist - 1
    g2 = oracle.geometry(64, 16, 0.004, 12.5, [2000.0], fmin=10.0, fmax=0.0)
    assert S.band(g2) == (6, 63)


def test_hann_sinc_values():
    R = 4
    assert S.hann_sinc(0.0, R) == pytest.approx(1.0, abs=0)
    for n in range(1, 8):
        assert abs(S.hann_sinc(float(n), R)) < 1e-15
        assert abs(S.hann_sinc(float(-n), R)) < 1e-15
    x = np.linspace(-5, 5, 1001)
    h = S.hann_sinc(x, R)
    assert np.all(h[np.abs(x) >= R] == 0)
    np.testing.assert_allclose(h, h[::-1], atol=1e-15)
    # near-partition of unity of the windowed sinc over the 2R taps
    for dlt in np.linspace(0, 1, 11, endpoint=False):
        s = sum(S.hann_sinc(dlt - t, R) for t in range(-R + 1, R + 1))
        assert abs(s - 1.0) < 0.02


# ---------------------------------------------------------------- FFT conventions
def _dft_matrix(n, sign):
    k = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / n)


def test_F_and_Finv_match_bruteforce_dft():
    rng = _rng(1)
    g = oracle.geometry(6, 5, 0.004, 10.0, [1000.0], ntp=12, nxp=10)
    x = rng.standard_normal((5, 6))
    pad = np.zeros((10, 12))
    pad[:5, :6] = x
    Ft = _dft_matrix(12, -1)[: 12 // 2 + 1]      # rows j = 0..ntp/2, e^{-i}
    Fx = _dft_matrix(10, -1)
    want = Fx @ (pad @ Ft.T)
    np.testing.assert_allclose(S._F(g, x), want, atol=1e-12)
    # inverse: ifft along x first, then the Hermitian-extended inverse along t
    Y = rng.standard_normal((10, 7)) + 1j * rng.standard_normal((10, 7))
    Y[:, 0] = 0
    Y[:, 6] = 0
    Z = (_dft_matrix(10, +1) @ Y) / 10
    full = np.zeros((10, 12), complex)
    full[:, :7] = Z
    full[:, 7:] = np.conj(Z[:, 1:6][:, ::-1])
    want_inv = np.real(full @ _dft_matrix(12, +1).T / 12)[:5, :6]
    np.testing.assert_allclose(S._Finv(g, Y), want_inv, atol=1e-12)


def _bruteforce_forward(g, m):
    """O(N^2) direct-sum evaluation of L on a tiny gather, scalar loops only."""
    P = g.npanel
    nx, nt, ntp, nxp, H, R = g.nx, g.nt, g.ntp, g.nxp, g.H, g.R
    jlo, jhi = S.band(g)
    # model spectra by direct sums
    M = np.zeros((P, nxp, H), complex)
    for p in range(P):
        for l in range(nxp):
            for k in range(H):
                acc = 0j
                for x in range(nx):
                    for t in range(nt):
                        acc += m[p, x, t] * complex(math.cos(-2 * math.pi * (l * x / nxp + k * t / ntp)),
                                                    math.sin(-2 * math.pi * (l * x / nxp + k * t / ntp)))
                M[p, l, k] = acc
    D = np.zeros((nxp, H), complex)
    for p in range(P):
        for l in range(nxp):
            ls = l if l < nxp // 2 else l - nxp
            a = g.vel[p] * abs(ls) * ntp * g.dt / (nxp * g.dx)
            for j in range(jlo, jhi + 1):
                if j < a:
                    continue
                u = math.sqrt(j * j - a * a)
                k0 = math.floor(u)
                acc = 0j
                for k in range(k0 - R + 1, k0 + R + 1):
                    if 1 <= k <= ntp // 2 - 1:
                        x_ = u - k
                        w = (1.0 if x_ == 0 else math.sin(math.pi * x_) / (math.pi * x_)) * \
                            (0.5 + 0.5 * math.cos(math.pi * x_ / R))
                        acc += w * M[p, l, k]
                ph = -2 * math.pi * ((j * int(g.tau0[p])) % ntp) / ntp
                W = 1.0 if g.wavelet is None else g.wavelet[j]
                D[l, j] += W * g.scale[p] * complex(math.cos(ph), math.sin(ph)) * acc
    # inverse: d(t,x) = (2/(ntp nxp)) Re sum_{l, j interior} D e^{+i(...)}
    d = np.zeros((nx, nt))
    for x in range(nx):
        for t in range(nt):
            acc = 0j
            for l in range(nxp):
                for j in range(1, ntp // 2):
                    acc += D[l, j] * complex(math.cos(2 * math.pi * (l * x / nxp + j * t / ntp)),
                                             math.sin(2 * math.pi * (l * x / nxp + j * t / ntp)))
            d[x, t] = 2.0 * acc.real / (ntp * nxp)
    return d


def test_forward_matches_direct_sum():
    rng = _rng(2)
    g = oracle.geometry(7, 5, 0.004, 10.0, [0.0, 1200.0, 2600.0], tau0=[0, 2, 5],
                        scale=[1.0, 0.5, 2.0], ntp=16, nxp=10, fmin=40.0, fmax=220.0,
                        wavelet=np.linspace(0.5, 1.5, 9))
    m = rng.standard_normal((3, 5, 7))
    np.testing.assert_allclose(oracle.forward(g, m), _bruteforce_forward(g, m), atol=1e-11)


# ---------------------------------------------------------------- adjointness
@pytest.mark.parametrize("case", ["plain", "ramp_mask_wavelet", "no_pad", "radix3"])
def test_dot_product(case):
    rng = _rng(3)
    kw = dict(nt=40, nx=12, dt=0.004, dx=12.5, vel=[1400.0, 2100.0, 3900.0])
    if case == "ramp_mask_wavelet":
        kw.update(tau0=[0, 3, 11], scale=[1.0, 0.3, 2.0], fmin=5.0, fmax=90.0)
    if case == "no_pad":
        kw.update(ntp=40, nxp=12)
    if case == "radix3":
        kw.update(nt=48, nx=24, ntp=96, nxp=48)
    g = oracle.geometry(**kw)
    if case == "ramp_mask_wavelet":
        g.wavelet = rng.uniform(0.2, 1.0, g.H)
    mask = None
    if case == "ramp_mask_wavelet":
        mask = (rng.uniform(size=g.nx) > 0.4).astype(np.uint8)
    m = rng.standard_normal((g.npanel, g.nx, g.nt))
    d = rng.standard_normal((g.nx, g.nt))
    Lm = oracle.forward(g, m, mask)
    LTd = oracle.adjoint(g, d, mask)
    lhs = float(np.sum(Lm * d))
    rhs = float(np.sum(m * LTd))
    assert abs(lhs - rhs) / (np.linalg.norm(Lm) * np.linalg.norm(d)) < 1e-12


# ---------------------------------------------------------------- special cases
def _bandpass_fft2(g, x):
    """Reference band-pass: full complex 2-D FFT, keep |freq bin| in the band."""
    jlo, jhi = S.band(g)
    pad = np.zeros((g.nxp, g.ntp))
    pad[: g.nx, : g.nt] = x
    X = np.fft.fft2(pad)
    j = np.arange(g.ntp)
    jj = np.minimum(j, g.ntp - j)
    keep = (jj >= jlo) & (jj <= jhi)
    return np.real(np.fft.ifft2(X * keep[None, :]))[: g.nx, : g.nt]


def test_zero_velocity_is_band_pass():
    rng = _rng(4)
    g = oracle.geometry(50, 14, 0.004, 12.5, [0.0], fmin=8.0, fmax=70.0)
    m = rng.standard_normal((1, 14, 50))
    np.testing.assert_allclose(oracle.forward(g, m), _bandpass_fft2(g, m[0]), atol=1e-12)


@pytest.mark.parametrize("v", [1400.0, 2500.0, 4000.0])
def test_constant_in_x_passes_any_velocity(v):
    rng = _rng(5)
    g = oracle.geometry(60, 16, 0.004, 12.5, [v], nxp=16, fmax=80.0)
    trace = rng.standard_normal(60)
    m = np.tile(trace, (16, 1))[None]
    np.testing.assert_allclose(oracle.forward(g, m), _bandpass_fft2(g, m[0]), atol=1e-11)


def test_dispersion_relation_single_mode():
    # one 2-D Fourier mode (l0, k0) of the model lands at w = sqrt(w_tau^2 + (v kx)^2)
    nt, nx, dt, dx, v = 64, 32, 0.004, 10.0, 2300.0
    g = oracle.geometry(nt, nx, dt, dx, [v], ntp=nt, nxp=nx)
    for (l0, k0) in [(5, 12), (3, 20), (9, 4), (0, 17)]:
        X, T = np.meshgrid(np.arange(nx), np.arange(nt), indexing="ij")
        m = np.cos(2 * np.pi * (l0 * X / nx + k0 * T / nt))[None]
        D = np.fft.fft(np.fft.rfft(oracle.forward(g, m), axis=1), axis=0)
        a = v * l0 * nt * dt / (nx * dx)          # v kx / dw in bins
        j_exact = math.sqrt(k0 * k0 + a * a)
        other = np.delete(np.abs(D), l0, axis=0)
        assert other.max() < 1e-9 * np.abs(D).max()
        jstar = int(np.argmax(np.abs(D[l0])))
        assert abs(jstar - j_exact) < 1.0, (l0, k0, jstar, j_exact)
        # support limited to data bins whose model coordinate is within R of k0
        nz = np.nonzero(np.abs(D[l0]) > 1e-9 * np.abs(D).max())[0]
        for j in nz:
            assert abs(math.sqrt(j * j - a * a) - k0) < g.R


def test_adjoint_reproduces_change_of_variables_factor():
    # adjoint of a flat data spectrum: sum_j h(u_j - k) ~ dj/du = w_tau / w (equation ch5_Stolt_adj)
    g = oracle.geometry(512, 64, 0.004, 12.5, [2000.0], fmax=0.0)
    B = S.stolt_matrix(g, 0)
    H = g.H
    col = np.asarray(B.sum(axis=0)).ravel().reshape(g.nxp, H)
    a = S.apex_shift_bins(g, 0)
    checked = 0
    for l in [1, 5, 9, 13]:
        for k in range(40, 300, 37):
            w_over_wt = math.sqrt(k * k + a[l] ** 2) / k
            if w_over_wt > 1.2:
                continue
            assert abs(col[l, k] - 1.0 / w_over_wt) < 0.035 * (1.0 / w_over_wt)
            checked += 1
    assert checked > 10


def test_translation_and_mirror():
    rng = _rng(6)
    g = oracle.geometry(40, 16, 0.004, 12.5, [1600.0, 3000.0], nxp=16)
    m = rng.standard_normal((2, 16, 40))
    d = oracle.forward(g, m)
    np.testing.assert_allclose(oracle.forward(g, np.roll(m, 5, axis=1)), np.roll(d, 5, axis=0), atol=1e-11)
    mir = lambda a, ax: np.roll(np.flip(a, axis=ax), 1, axis=ax)  # x -> -x (mod nx)
    np.testing.assert_allclose(oracle.forward(g, mir(m, 1)), mir(d, 0), atol=1e-11)


# ---------------------------------------------------------------- kinematics vs brute force
def _envelope_peaks(d):
    env = np.abs(scipy.signal.hilbert(d, axis=1))
    return np.argmax(env, axis=1)


@pytest.mark.parametrize("n0", [0, 10])
def test_forward_kinematics_match_time_domain(n0):
    nt, nx, dt, dx, v = 128, 48, 0.004, 10.0, 2000.0
    g = oracle.geometry(nt, nx, dt, dx, [v], tau0=[n0], fmax=60.0)
    m = np.zeros((1, nx, nt))
    tau_i, xa = 50, 24
    m[0, xa, tau_i] = 1.0
    d = oracle.forward(g, m)
    d_td = TD.forward(m, dt, dx, [v], tau0=[n0])
    pk = _envelope_peaks(d)
    pk_td = _envelope_peaks(d_td)
    for x in range(8, 40):
        t_true = n0 + math.sqrt((tau_i * dt) ** 2 + ((x - xa) * dx) ** 2 / v ** 2) / dt
        assert abs(pk[x] - t_true) <= 1.0, (x, pk[x], t_true)
        assert abs(pk_td[x] - t_true) <= 1.0
    # the Stolt and time-domain responses are alike in shape, not in amplitude
    env = np.abs(scipy.signal.hilbert(d, axis=1))[8:40]
    env_td = np.abs(scipy.signal.hilbert(TD.forward(m, dt, dx, [v], tau0=[n0]), axis=1))[8:40]
    cc = np.sum(env * env_td) / np.sqrt(np.sum(env ** 2) * np.sum(env_td ** 2))
    assert cc > 0.5


def test_adjoint_focuses_hyperbola_at_true_parameters():
    from synth import render_events
    nt, nx, dt, dx = 128, 48, 0.004, 10.0
    vels = [1500.0, 2000.0, 2500.0]
    g = oracle.geometry(nt, nx, dt, dx, vels, fmax=80.0)
    tau, xa, v = 0.2, 24 * dx, 2000.0
    d = render_events(nt, nx, dt, dx, [(tau, v, xa, 0.0, 1.0)])
    m = oracle.adjoint(g, d)
    env = np.abs(scipy.signal.hilbert(m, axis=2))
    p, x, t = np.unravel_index(np.argmax(env), env.shape)
    assert p == 1
    assert abs(x - 24) <= 1
    assert abs(t - tau / dt) <= 1
    # the time-domain adjoint focuses at the same place
    m_td = TD.adjoint(d, dt, dx, vels)
    env_td = np.abs(scipy.signal.hilbert(m_td, axis=2))
    p2, x2, t2 = np.unravel_index(np.argmax(env_td), env_td.shape)
    assert (p2, abs(x2 - 24) <= 1, abs(t2 - tau / dt) <= 1) == (1, True, True)


def test_time_domain_pair_is_adjoint():
    rng = _rng(7)
    m = rng.standard_normal((2, 9, 20))
    d = rng.standard_normal((9, 20))
    vel = [1500.0, 2500.0]
    a = np.sum(TD.forward(m, 0.004, 10.0, vel, tau0=[0, 3]) * d)
    b = np.sum(m * TD.adjoint(d, 0.004, 10.0, vel, tau0=[0, 3]))
    assert abs(a - b) < 1e-10 * abs(a)


def test_wavelet_weight_is_zero_phase_filter_and_scale_is_linear():
    rng = _rng(8)
    nt, nx = 64, 12
    g0 = oracle.geometry(nt, nx, 0.004, 12.5, [1800.0, 2600.0], ntp=nt, fmax=90.0)
    W = np.exp(-((np.arange(nt // 2 + 1) - 10.0) / 8.0) ** 2)
    gw = oracle.geometry(nt, nx, 0.004, 12.5, [1800.0, 2600.0], ntp=nt, fmax=90.0, wavelet=W)
    gs = oracle.geometry(nt, nx, 0.004, 12.5, [1800.0, 2600.0], ntp=nt, fmax=90.0, scale=[2.0, 2.0])
    m = rng.standard_normal((2, nx, nt))
    d0 = oracle.forward(g0, m)
    filt = np.fft.irfft(W[None, :] * np.fft.rfft(d0, axis=1), n=nt, axis=1)
    np.testing.assert_allclose(oracle.forward(gw, m), filt, atol=1e-12)
    np.testing.assert_allclose(oracle.forward(gs, m), 2.0 * d0, atol=1e-12)


# ---------------------------------------------------------------- irregular traces
def _irr_geom(xpos=None, nxp=0):
    return oracle.geometry(48, 16, 0.004, 12.5, [1600.0, 2500.0], fmax=100.0, xpos=xpos, nxp=nxp)


def test_nudft_at_regular_positions_is_the_dft_without_nyquist():
    g = _irr_geom(xpos=np.arange(16) * 12.5)
    E = oracle.stolt.nudft_matrix(g)
    rng = np.random.default_rng(0)
    D = rng.standard_normal((g.nxp, 5)) + 1j * rng.standard_normal((g.nxp, 5))
    D[g.nxp // 2] = 0.0
    ref = np.fft.ifft(D, axis=0)[:16] * g.nxp
    assert np.allclose(E @ D, ref, rtol=1e-12, atol=1e-12)


def test_irregular_operator_reduces_to_regular_when_nyquist_is_empty():
    """At regular positions the irregular pair differs from the regular one
    only by the Nyquist wavenumber; a model band-limited below it gives the
    same data."""
    rng = np.random.default_rng(1)
    greg = _irr_geom()
    girr = _irr_geom(xpos=np.arange(16) * 12.5)
    m = rng.standard_normal((2, 16, 48))
    # remove the Nyquist wavenumber of the padded x grid from the model
    Mx = np.fft.fft(m, n=greg.nxp, axis=1)
    Mx[:, greg.nxp // 2] = 0.0
    m = np.real(np.fft.ifft(Mx, axis=1))[:, :16]
    # the model-side transforms zero-pad the truncated model, so compare the
    # part that does not see the Nyquist term: both operators on the same m
    d_reg = oracle.forward(greg, m)
    d_irr = oracle.forward(girr, m)
    # the difference is exactly the Nyquist-row contribution of the regular operator
    diff = d_reg - d_irr
    D = np.zeros((greg.nxp, greg.H), complex)
    for p in range(2):
        Mp = oracle.stolt._F(greg, m[p])
        Dp = (oracle.stolt_matrix(greg, p) @ Mp.ravel()).reshape(greg.nxp, greg.H)
        D += oracle.data_bin_factor(greg, p)[None, :] * Dp
    Dn = np.zeros_like(D)
    Dn[greg.nxp // 2] = D[greg.nxp // 2]
    assert np.allclose(diff, oracle.stolt._Finv(greg, Dn), rtol=1e-10, atol=1e-12)


def test_irregular_dot_product():
    rng = np.random.default_rng(2)
    xpos = np.sort(rng.uniform(0, 15 * 12.5, 16))
    g = _irr_geom(xpos=xpos)
    m = rng.standard_normal((2, 16, 48))
    d = rng.standard_normal((16, 48))
    lhs = np.sum(oracle.forward(g, m) * d)
    rhs = np.sum(m * oracle.adjoint(g, d))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(oracle.forward(g, m)) * np.linalg.norm(d)


def test_irregular_forward_is_the_trigonometric_interpolant():
    """Data at shifted positions equal the band-limited (Fourier-series)
    interpolation, on the padded periodic x grid, of the data at regular
    positions."""
    rng = np.random.default_rng(3)
    m = rng.standard_normal((2, 16, 48))
    shift = 0.37 * 12.5
    g0 = _irr_geom(xpos=np.arange(16) * 12.5)
    g1 = _irr_geom(xpos=np.arange(16) * 12.5 + shift)
    # full padded-grid data of g0's spectrum, then shift by the Fourier phase
    D = np.zeros((g0.nxp, g0.H), complex)
    for p in range(2):
        Mp = oracle.stolt._F(g0, m[p])
        Dp = (oracle.stolt_matrix(g0, p) @ Mp.ravel()).reshape(g0.nxp, g0.H)
        D += oracle.data_bin_factor(g0, p)[None, :] * Dp
    D[g0.nxp // 2] = 0.0
    lp = oracle.stolt.signed_kx_index(g0.nxp)
    Ds = D * np.exp(2j * np.pi * lp * shift / (g0.nxp * 12.5))[:, None]
    ref = oracle.stolt._Finv(g0, Ds)
    assert np.allclose(oracle.forward(g1, m), ref, rtol=1e-10, atol=1e-12)
