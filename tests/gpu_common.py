"""Helpers shared by the GPU parity tests: build the HIP plan and the oracle
geometry from the same keyword arguments, feed both the same FP32-rounded
inputs, and measure relative L2 error."""
import numpy as np

import oracle


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def geom_kwargs(nt, nx, dt, dx, vel, tau0=None, scale=None, ntp=0, nxp=0, fmin=0.0, fmax=0.0,
                half_width=4, wavelet=None, xpos=None):
    return dict(nt=nt, nx=nx, dt=dt, dx=dx, vel=vel, tau0=tau0, scale=scale, ntp=ntp, nxp=nxp,
                fmin=fmin, fmax=fmax, half_width=half_width, wavelet=wavelet, xpos=xpos)


def oracle_geometry(kw):
    return oracle.geometry(kw["nt"], kw["nx"], kw["dt"], kw["dx"], kw["vel"], tau0=kw["tau0"],
                           scale=kw["scale"], ntp=kw["ntp"], nxp=kw["nxp"], fmin=kw["fmin"],
                           fmax=kw["fmax"], R=kw["half_width"], wavelet=kw["wavelet"], xpos=kw.get("xpos"))


def f32(x):
    """FP32 rounding of an FP64 array, returned as FP64 (what both sides see)."""
    return np.asarray(x, np.float32).astype(np.float64)
