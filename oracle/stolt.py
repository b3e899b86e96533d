"""FP64 oracle of the Stolt-based (A)ASHRT forward operator L and its adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (thesis Chapter 5, equations ch5_forward_operator and
ch5_adj_operator; Chapter 6, equations ch6_forward_operator and
ch6_adj_operator):

    L  = S  F^-1_{w,kx}  T  M  F_{tau,x}          (per panel, then summed)
    L' = F^-1_{wtau,kx}  M' T' F_{t,x}  S'        (sprayed to every panel)

* F is the 2-D DFT of the zero-padded gather: real FFT along time (numpy
  ``rfft``), then complex FFT along x; both unnormalised.  F^-1 is the
  inverse along x *first*, then the inverse real FFT along time; both carry
  numpy's 1/N.  Padding (nt, nx) -> (ntp, nxp) with the smallest 2^a or
  3*2^a >= 2n (the thesis asks for padding, Chapter 5, but gives no factor).
* M is the Stolt map from apex-time frequency w_tau to data frequency w at
  fixed kx, through the dispersion relation w_tau = sqrt(w^2 - (v kx)^2)
  (equation after ch5_Stolt_adj1).  In bins: data bin j, model bin k, kx bin l
  with signed index l'; a_{p,l} = v_p |l'| ntp dt / (nxp dx) is v|kx|/dw and
  u = sqrt(j^2 - a^2) is the model coordinate that feeds data bin j.  The
  forward *interpolates* the model spectrum at u with a Hann-windowed sinc of
  half-width R (taps k = floor(u)-R+1 .. floor(u)+R), and only for j inside
  the signal cone (j >= a) and inside the mapped band; it has no Jacobian,
  as the forward integral of ch5_Stolt_forward has none.  The adjoint is the
  exact transpose, which reproduces the change-of-variables factor
  C = w_tau / w of ch5_Stolt_adj through the tap density.
* Only the interior positive-frequency bins 1..ntp/2-1 take part (the thesis
  maps positive frequencies and uses the Fourier symmetry for the negative
  ones); DC and Nyquist are zero on both sides.
* T (Chapter 6) is the asymptote shift tau0 = n0*dt applied as the phase ramp
  exp(-i w_j tau0) on *data* bins in the forward and its conjugate in the
  adjoint.  An optional real per-panel scale s_p and per-bin weight W_j (the
  zero-phase wavelet of Chapter 4's "C L" variant) multiply the same factor.
* S (Chapter 6) is the trace-sampling mask; the sum over panels and its
  spraying adjoint are the ch5 "summation operator".

* Irregular data traces (positions x_i given): the data-side x transform is
  a non-uniform DFT, D[l] = sum_i exp(-2 pi i l' x_i / (nxp dx)) d_i and
  d_i = (1/nxp) sum_l exp(+2 pi i l' x_i / (nxp dx)) D[l], without the
  Nyquist wavenumber (its phase is not real off the grid); the model (apex)
  grid stays regular.  The thesis names non-uniform transforms as the way
  to irregular sampling (Chapters 5 and 7) without detail: a reading.

The map is stored as an explicit sparse matrix per panel so the adjoint is
literally its transpose.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp


def fft_len(n: int) -> int:
    """Smallest 2^a or 3*2^a that is >= 2n (the padding reading)."""
    target = 2 * n
    best = None
    p = 1
    while p < 2 * target + 8:
        for c in (p, 3 * p):
            if c >= target and (best is None or c < best):
                best = c
        p *= 2
    return best


@dataclass
class Geometry:
    nt: int
    nx: int
    dt: float
    dx: float
    ntp: int
    nxp: int
    vel: np.ndarray          # [P] m/s
    tau0: np.ndarray         # [P] int samples
    scale: np.ndarray        # [P]
    fmin: float
    fmax: float
    R: int
    wavelet: Optional[np.ndarray]  # [ntp//2+1] real or None
    xpos: Optional[np.ndarray] = None  # [nx] data trace positions (m) or None = regular i*dx
    _cache: dict = field(default_factory=dict, repr=False, compare=False)

    @property
    def npanel(self):
        return len(self.vel)

    @property
    def H(self):
        return self.ntp // 2 + 1


def geometry(nt, nx, dt, dx, vel, tau0=None, scale=None, ntp=0, nxp=0, fmin=0.0,
             fmax=0.0, R=4, wavelet=None, xpos=None) -> Geometry:
    vel = np.asarray(vel, dtype=np.float64).ravel()
    P = len(vel)
    tau0 = np.zeros(P, np.int64) if tau0 is None else np.asarray(tau0, np.int64).ravel()
    scale = np.ones(P) if scale is None else np.asarray(scale, np.float64).ravel()
    ntp = fft_len(nt) if not ntp else int(ntp)
    nxp = fft_len(nx) if not nxp else int(nxp)
    if wavelet is not None:
        wavelet = np.asarray(wavelet, np.float64).ravel()
        assert wavelet.shape == (ntp // 2 + 1,)
    if xpos is not None:
        xpos = np.asarray(xpos, np.float64).ravel()
        assert xpos.shape == (nx,)
    return Geometry(nt, nx, float(dt), float(dx), ntp, nxp, vel, tau0, scale,
                    float(fmin), float(fmax), int(R), wavelet, xpos)


def band(g: Geometry):
    """Inclusive data-bin range [jlo, jhi] of the mapped band.

    jlo = max(1, ceil(fmin*ntp*dt)), jhi = min(ntp/2-1, floor(fmax*ntp*dt));
    fmax <= 0 means "up to just below Nyquist".
    """
    jlo = max(1, int(np.ceil(g.fmin * g.ntp * g.dt)))
    jhi = g.ntp // 2 - 1
    if g.fmax > 0:
        jhi = min(jhi, int(np.floor(g.fmax * g.ntp * g.dt)))
    return jlo, jhi


def hann_sinc(x, R):
    """Interpolation kernel h(x) = sinc(x) * (1/2 + 1/2 cos(pi x / R)) on |x| < R."""
    x = np.asarray(x, dtype=np.float64)
    w = np.sinc(x) * (0.5 + 0.5 * np.cos(np.pi * x / R))
    return np.where(np.abs(x) < R, w, 0.0)


def signed_kx_index(nxp):
    l = np.arange(nxp)
    return np.where(l < nxp // 2, l, l - nxp)


def apex_shift_bins(g: Geometry, p: int):
    """a_{p,l} = v_p |l'| ntp dt / (nxp dx): v|kx| measured in data-frequency bins."""
    return g.vel[p] * np.abs(signed_kx_index(g.nxp)) * g.ntp * g.dt / (g.nxp * g.dx)


def stolt_matrix(g: Geometry, p: int) -> sp.csr_matrix:
    """Sparse real matrix B_p with D[l, j] = sum_k B_p[(l,j), (l,k)] M_p[l, k].

    Rows are data bins (l, j) flattened as l*H + j; columns are model bins
    (l, k) flattened the same way.  Built from the definition: for j in the
    band and inside the cone j >= a_{p,l}, u = sqrt(j^2 - a^2), taps
    k = floor(u) + t for t = -R+1..R kept when 1 <= k <= ntp/2 - 1, weight
    h(u - k).  Cached per velocity (panels that differ only by tau0 or scale
    share it).
    """
    key = ("B", float(g.vel[p]))
    if key in g._cache:
        return g._cache[key]
    H = g.H
    jlo, jhi = band(g)
    j = np.arange(jlo, jhi + 1, dtype=np.float64)
    a = apex_shift_bins(g, p)
    L = np.arange(g.nxp)[:, None] * np.ones((1, len(j)), np.int64)
    J = np.ones((g.nxp, 1)) * j[None, :]
    A = a[:, None] * np.ones((1, len(j)))
    cone = J >= A
    U = np.sqrt(np.maximum(J * J - A * A, 0.0))
    K0 = np.floor(U).astype(np.int64)
    rows, cols, vals = [], [], []
    Ji = J.astype(np.int64)
    for t in range(-g.R + 1, g.R + 1):
        K = K0 + t
        ok = cone & (K >= 1) & (K <= g.ntp // 2 - 1)
        rows.append((L * H + Ji)[ok])
        cols.append((L * H + K)[ok])
        vals.append(hann_sinc(U - K, g.R)[ok])
    B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(g.nxp * H, g.nxp * H))
    g._cache[key] = B
    return B


def data_bin_factor(g: Geometry, p: int):
    """Per data bin j: W_j * s_p * exp(-2 pi i j n0_p / ntp) (ramp T of Chapter 6)."""
    j = np.arange(g.H)
    W = np.ones(g.H) if g.wavelet is None else g.wavelet
    ph = ((j * int(g.tau0[p])) % g.ntp) / g.ntp
    return W * g.scale[p] * np.exp(-2j * np.pi * ph)


def _F(g: Geometry, x2d):
    """F_{t,x}: zero-pad to (nxp, ntp); rfft along t then fft along x."""
    return np.fft.fft(np.fft.rfft(x2d, n=g.ntp, axis=1), n=g.nxp, axis=0)


def _Finv(g: Geometry, X):
    """F^-1: ifft along x first, then irfft along t; truncate to (nx, nt)."""
    return np.fft.irfft(np.fft.ifft(X, axis=0), n=g.ntp, axis=1)[: g.nx, : g.nt]


def nudft_matrix(g: Geometry):
    """E[i, l] = exp(+2 pi i l' x_i / (nxp dx)) for the data traces at
    g.xpos, with the Nyquist wavenumber column zero (irregular positions:
    the thesis' suggested extension of F_x to non-uniform sampling, Chapter
    5 and Chapter 7).  At x_i = i dx it is the inverse-DFT kernel without
    the Nyquist term."""
    lp = signed_kx_index(g.nxp).astype(np.float64)
    E = np.exp(2j * np.pi * np.outer(g.xpos, lp) / (g.nxp * g.dx))
    E[:, g.nxp // 2] = 0.0
    return E


def _F_data(g: Geometry, d):
    """Data-side F: as _F, with the x transform a non-uniform DFT when the
    traces sit at g.xpos: D[l] = sum_i exp(-2 pi i l' x_i / (nxp dx)) d_i."""
    if g.xpos is None:
        return _F(g, d)
    return nudft_matrix(g).conj().T @ np.fft.rfft(d, n=g.ntp, axis=1)


def _Finv_data(g: Geometry, D):
    """Data-side F^-1: as _Finv, with d_i = (1/nxp) sum_l exp(+2 pi i l' x_i /
    (nxp dx)) D[l] (x first), then the inverse real FFT along t."""
    if g.xpos is None:
        return _Finv(g, D)
    return np.fft.irfft((nudft_matrix(g) @ D) / g.nxp, n=g.ntp, axis=1)[:, : g.nt]


def forward(g: Geometry, m, mask=None):
    """d = S sum_p F^-1 T_p M_p F m_p  (model [P][nx][nt] -> data [nx][nt])."""
    m = np.asarray(m, dtype=np.float64)
    assert m.shape == (g.npanel, g.nx, g.nt), m.shape
    D = np.zeros((g.nxp, g.H), dtype=np.complex128)
    for p in range(g.npanel):
        Mp = _F(g, m[p])
        Dp = (stolt_matrix(g, p) @ Mp.ravel()).reshape(g.nxp, g.H)
        D += data_bin_factor(g, p)[None, :] * Dp
    d = _Finv_data(g, D)
    if mask is not None:
        d = d * np.asarray(mask, np.float64)[:, None]
    return d


def adjoint(g: Geometry, d, mask=None):
    """m_p = F^-1 M_p' T_p' F S d for every panel p  (data -> model)."""
    d = np.asarray(d, dtype=np.float64)
    assert d.shape == (g.nx, g.nt), d.shape
    if mask is not None:
        d = d * np.asarray(mask, np.float64)[:, None]
    D = _F_data(g, d)
    m = np.empty((g.npanel, g.nx, g.nt))
    for p in range(g.npanel):
        E = np.conj(data_bin_factor(g, p))[None, :] * D
        Mp = (stolt_matrix(g, p).T @ E.ravel()).reshape(g.nxp, g.H)
        m[p] = _Finv(g, Mp)
    return m
