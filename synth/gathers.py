"""Seeded synthetic blended common receiver gathers.

Events are analytic hyperbolae evaluated at the sample times,
``d[x_j, i] += A * ricker(i*dt - T(x_j))`` with
``T = t0 + sqrt(tau^2 + (x - x_a)^2 / v^2)`` (reflections have t0 = 0; the
diffraction traveltime with an asymptote shift is the double-square-root form
of Chapter 6, where the source-side root becomes the constant t0).
Blended interference on a contaminated trace is the same trace of an
independent second-source gather, drawn by the same law, shifted by a random
firing delay and scaled (Chapter 2's pseudo-deblended gathers: incoherent
energy on a subset of receivers). Every draw comes from
``numpy.random.default_rng(seed)`` (PCG64).

Outputs are FP64 arrays laid out ``[nx][nt]`` (time contiguous).
"""
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .configs import Workload


def ricker(t, f=25.0):
    """Ricker wavelet with peak frequency f (Hz), peak value 1 at t = 0."""
    a = (np.pi * f * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


@dataclass
class Gather:
    workload: Workload
    nt: int
    nx: int
    d_clean: np.ndarray      # [nx][nt] primary-source signal (complete)
    d_blend: np.ndarray      # [nx][nt] observed: clean + interference, masked traces zeroed
    mask: np.ndarray         # [nx] uint8, 1 = live trace
    events: list
    interfered: np.ndarray   # indices of contaminated traces
    seed: int


def render_events(nt, nx, dt, dx, events, f=25.0, delays=None, traces=None):
    """Sum Ricker hyperbolae.  Each event is (tau, v, x_a, t0, amp).

    ``delays`` (per trace, s) shifts every event on that trace; ``traces``
    restricts rendering to a subset of trace indices (others stay zero).
    """
    d = np.zeros((nx, nt))
    t = np.arange(nt) * dt
    idx = range(nx) if traces is None else traces
    for j in idx:
        x = j * dx
        sh = 0.0 if delays is None else delays[j]
        for (tau, v, xa, t0, amp) in events:
            T = t0 + np.sqrt(tau * tau + (x - xa) ** 2 / (v * v)) + sh
            d[j] += amp * ricker(t - T, f)
    return d


def _draw_events(rng, w: Workload, nt, nx, n):
    tau_hi = w.tau_range[1]
    if w.tau_frac_of_record is not None:
        tau_hi = w.tau_frac_of_record * nt * w.dt
    ev = []
    for _ in range(n):
        tau = rng.uniform(w.tau_range[0], tau_hi)
        v = rng.uniform(*w.v_range)
        xa = rng.uniform(0.0, (nx - 1) * w.dx)
        ev.append((tau, v, xa, 0.0, w.amp))
    return ev


def make_gather(w: Workload, seed: Optional[int] = None, nt: Optional[int] = None,
                nx: Optional[int] = None) -> Gather:
    """Draw one gather of workload ``w``.

    For the batched workload the caller passes the per-gather nt/nx (see
    :func:`make_cfg3_batch`); otherwise the workload's geometry is used.
    """
    seed = w.seed if seed is None else seed
    nt = w.nt if nt is None else nt
    nx = w.nx if nx is None else nx
    rng = np.random.default_rng(seed)
    n_ev = int(rng.integers(w.n_events[0], w.n_events[1] + 1))
    events = _draw_events(rng, w, nt, nx, n_ev)
    for _ in range(w.n_diffractors):
        tau = rng.uniform(*w.tau_range)
        v = rng.uniform(*w.v_range)
        xa = rng.uniform(0.0, (nx - 1) * w.dx)
        t0 = rng.uniform(*w.diff_t0_range)
        events.append((tau, v, xa, t0, w.diff_amp))
    d_clean = render_events(nt, nx, w.dt, w.dx, events, f=w.ricker_hz)

    frac = rng.uniform(*w.interf_frac) if w.interf_frac[1] > w.interf_frac[0] else w.interf_frac[0]
    n_int = int(round(frac * nx))
    interfered = np.sort(rng.choice(nx, size=n_int, replace=False)) if n_int > 0 else np.zeros(0, int)
    d_blend = d_clean.copy()
    if n_int > 0:
        # the second source: an independent gather drawn by the same law
        n_ev2 = int(rng.integers(w.n_events[0], w.n_events[1] + 1))
        ev2 = _draw_events(rng, w, nt, nx, n_ev2)
        delays = np.zeros(nx)
        amps = np.zeros(nx)
        delays[interfered] = rng.uniform(*w.interf_delay, size=n_int)
        amps[interfered] = rng.uniform(*w.interf_amp, size=n_int)
        second = render_events(nt, nx, w.dt, w.dx, ev2, f=w.ricker_hz, delays=delays,
                               traces=interfered)
        d_blend += amps[:, None] * second

    mask = np.ones(nx, np.uint8)
    if w.decimate_frac > 0:
        n_dead = int(round(w.decimate_frac * nx))
        dead = rng.choice(nx, size=n_dead, replace=False)
        mask[dead] = 0
        d_blend[dead] = 0.0
    return Gather(workload=w, nt=nt, nx=nx, d_clean=d_clean, d_blend=d_blend, mask=mask,
                  events=events, interfered=interfered, seed=seed)


def batch_shapes(n: int, first_seed: int = 1000):
    """(nt, nx, seed) for the gathers of the batched workload.

    nx is uniform on {96..320}; nt uniform on {1024, 1536, 2048}.
    """
    out = []
    for g in range(n):
        s = first_seed + g
        rng = np.random.default_rng([s, 7])
        nx = int(rng.integers(96, 321))
        nt = int(rng.choice([1024, 1536, 2048]))
        out.append((nt, nx, s))
    return out


def make_cfg3_batch(w: Workload, n: int, first: int = 0) -> List[Gather]:
    shapes = batch_shapes(first + n, w.seed)[first:]
    return [make_gather(w, seed=s, nt=nt, nx=nx) for (nt, nx, s) in shapes]


def random_model(rng, npanel, nx, nt, dtype=np.float64):
    """Gaussian model cube [P][nx][nt]."""
    return rng.standard_normal((npanel, nx, nt)).astype(dtype)


def random_data(rng, nx, nt, dtype=np.float64):
    return rng.standard_normal((nx, nt)).astype(dtype)
