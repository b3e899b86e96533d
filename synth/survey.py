"""Seeded synthetic multi-source survey: an unblended cube of shot gathers
and the dithered firing times of a one-vessel blended acquisition (inputs
only; no blending or separation arithmetic).

Sources and receivers share one line (spacing dx).  Each reflection with
zero-offset time t0 and velocity v arrives at t = sqrt(t0^2 + (xs - xr)^2 / v^2)
(25 Hz Ricker, unit amplitude); in a common receiver gather it is a
hyperbola in the source coordinate with its apex at the receiver.  Firing
times: source s fires at s * interval + U(0, dither) samples, with interval =
(1 - compression) * nt (50 % compression halves the time between shots).
"""
from dataclasses import dataclass

import numpy as np

from .gathers import ricker


@dataclass
class Survey:
    D: np.ndarray       # [ns][nr][nt] unblended shot gathers
    fire: np.ndarray    # [ns] firing times (samples)
    dt: float
    dx: float


def make_survey(ns=64, nt=512, dt=0.004, dx=12.5, n_events=6, compression=0.5, dither_s=0.4,
                v_range=(1500.0, 3200.0), seed=7) -> Survey:
    rng = np.random.default_rng(seed)
    nr = ns
    t = np.arange(nt) * dt
    x = np.arange(ns) * dx
    off = x[:, None] - x[None, :]                      # [s][r] source - receiver
    D = np.zeros((ns, nr, nt))
    t0s = rng.uniform(0.1, 0.8 * nt * dt, n_events)
    vs = rng.uniform(*v_range, n_events)
    amps = rng.uniform(0.5, 1.0, n_events) * rng.choice([-1.0, 1.0], n_events)
    for t0, v, a in zip(t0s, vs, amps):
        T = np.sqrt(t0 * t0 + (off / v) ** 2)          # [s][r]
        D += a * ricker(t[None, None, :] - T[:, :, None])
    interval = int(round((1.0 - compression) * nt))
    fire = np.arange(ns) * interval + rng.integers(0, int(round(dither_s / dt)) + 1, ns)
    return Survey(D=D, fire=fire.astype(np.int64), dt=dt, dx=dx)
