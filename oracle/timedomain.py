"""Brute-force time-domain (A)ASHRT, used only to pin the kinematics of the
Stolt operator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Thesis Chapter 3, table ch3_table_Radon_operators (ASHRT and AASHRT rows),
and Chapter 6, equations ch6_AASHRT_forward and ch6_AASHRT_adjoint: a model
sample at apex time tau, velocity v, apex x_a (and asymptote shift tau0)
contributes to every trace x along t = tau0 + sqrt(tau^2 + (x - x_a)^2 / v^2);
the adjoint sums the data along the same curves.  Linear interpolation in time;
the apex grid is the receiver grid.  Cost O(P * nx^2 * nt): tiny gathers only.
"""
import numpy as np


def _curve(nt, nx, dt, dx, v, tau0_s):
    tau = np.arange(nt) * dt
    x = np.arange(nx) * dx
    X = x[None, :, None] - x[:, None, None]          # [x_a][x][1]
    return tau0_s + np.sqrt(tau[None, None, :] ** 2 + X ** 2 / (v * v))   # [x_a][x][tau]


def forward(m, dt, dx, vel, tau0=None):
    """d(t, x) = sum_{p, x_a, tau} m[p, x_a, tau] spread at t = tau0_p + sqrt(tau^2 + (x-x_a)^2/v_p^2)."""
    m = np.asarray(m, dtype=np.float64)
    P, nx, nt = m.shape
    tau0 = np.zeros(P, int) if tau0 is None else np.asarray(tau0)
    d = np.zeros(nx * nt)
    for p in range(P):
        T = _curve(nt, nx, dt, dx, vel[p], tau0[p] * dt) / dt   # fractional sample index
        i0 = np.floor(T).astype(np.int64)
        f = T - i0
        val = np.broadcast_to(m[p][:, None, :], T.shape)        # [x_a][x][tau]
        xi = np.broadcast_to(np.arange(nx)[None, :, None], T.shape)
        for off, w in ((0, 1.0 - f), (1, f)):
            idx = i0 + off
            ok = (idx >= 0) & (idx < nt)
            np.add.at(d, (xi * nt + idx)[ok], (val * w)[ok])
    return d.reshape(nx, nt)


def adjoint(d, dt, dx, vel, tau0=None, npanel=None):
    """m[p, x_a, tau] = sum_x d(t = tau0_p + sqrt(tau^2 + (x-x_a)^2/v_p^2), x)."""
    d = np.asarray(d, dtype=np.float64)
    nx, nt = d.shape
    P = len(vel)
    tau0 = np.zeros(P, int) if tau0 is None else np.asarray(tau0)
    flat = d.ravel()
    m = np.zeros((P, nx, nt))
    for p in range(P):
        T = _curve(nt, nx, dt, dx, vel[p], tau0[p] * dt) / dt
        i0 = np.floor(T).astype(np.int64)
        f = T - i0
        xi = np.broadcast_to(np.arange(nx)[None, :, None], T.shape)
        acc = np.zeros(T.shape)
        for off, w in ((0, 1.0 - f), (1, f)):
            idx = i0 + off
            ok = (idx >= 0) & (idx < nt)
            acc += np.where(ok, w * flat[np.clip(xi * nt + idx, 0, nx * nt - 1)], 0.0)
        m[p] = acc.sum(axis=1)
    return m
