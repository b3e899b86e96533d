"""The synthetic workloads, by name.

Each workload fixes the gather geometry, the Radon panel list (one velocity
and one asymptote shift per panel), the inversion settings and the law the
seeded generator draws events and interference from. The event laws stand in
for the thesis' blended synthetic and field gathers (Chapter 4 and 5
examples; Chapter 6 diffraction example), whose geometry and data are not
published in numbers.

Names say what the workload is:

* ``crg-256x64-nv8``      small blended receiver gather, 8 velocities, 5x10 IRLS-CG
* ``crg-1024x256-nv32``   production-size blended receiver gather, 32 velocities, 10x20
* ``batch512-crg-nv24``   512 receiver gathers of uneven size, 24 velocities, 10x20
* ``aashrt-1024x256-nv24x16``  diffraction gather with half the traces missing;
  24 velocities x 16 asymptote shifts (0..75 samples, step 5), p=2, q=1
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    nt: int
    nx: int
    dt: float
    dx: float
    vel: Tuple[float, ...]          # one entry per panel (m/s)
    tau0: Tuple[int, ...]           # one entry per panel (asymptote shift, samples)
    fmin: float = 0.0
    fmax: float = 100.0
    half_width: int = 4
    p: int = 1
    q: int = 2
    n_outer: int = 10
    n_inner: int = 20
    seed: int = 0
    # generator law
    n_events: Tuple[int, int] = (3, 3)           # inclusive integer range
    tau_range: Tuple[float, float] = (0.2, 0.8)  # s
    v_range: Tuple[float, float] = (1500.0, 3000.0)
    amp: float = 1.0
    interf_frac: Tuple[float, float] = (0.2, 0.2)
    interf_amp: Tuple[float, float] = (5.0, 5.0)
    interf_delay: Tuple[float, float] = (-0.25, 0.25)
    n_diffractors: int = 0
    diff_t0_range: Tuple[float, float] = (0.0, 0.3)
    diff_amp: float = 0.5
    decimate_frac: float = 0.0
    ricker_hz: float = 25.0
    tau_frac_of_record: Optional[float] = None   # tau upper bound as a fraction of nt*dt

    @property
    def npanel(self) -> int:
        return len(self.vel)


def _panels(vels, tau0s=(0,)):
    v = []
    t = []
    for vv in vels:
        for tt in tau0s:
            v.append(float(vv))
            t.append(int(tt))
    return tuple(v), tuple(t)


def _mk():
    out = {}
    v, t = _panels(np.linspace(1500.0, 3000.0, 8))
    out["crg-256x64-nv8"] = Workload(
        name="crg-256x64-nv8", nt=256, nx=64, dt=0.004, dx=12.5, vel=v, tau0=t,
        p=1, q=2, n_outer=5, n_inner=10, seed=1,
        n_events=(3, 3), tau_range=(0.2, 0.8), v_range=(1500.0, 3000.0), amp=1.0,
        interf_frac=(0.2, 0.2), interf_amp=(5.0, 5.0), interf_delay=(-0.25, 0.25))
    v, t = _panels(np.linspace(1400.0, 4000.0, 32))
    out["crg-1024x256-nv32"] = Workload(
        name="crg-1024x256-nv32", nt=1024, nx=256, dt=0.004, dx=12.5, vel=v, tau0=t,
        p=1, q=2, n_outer=10, n_inner=20, seed=2,
        n_events=(12, 12), tau_range=(0.2, 3.6), v_range=(1400.0, 4000.0), amp=1.0,
        interf_frac=(0.4, 0.4), interf_amp=(3.0, 10.0), interf_delay=(0.0, 2.0))
    v, t = _panels(np.linspace(1400.0, 4000.0, 24))
    out["batch512-crg-nv24"] = Workload(
        name="batch512-crg-nv24", nt=0, nx=0, dt=0.004, dx=12.5, vel=v, tau0=t,
        p=1, q=2, n_outer=10, n_inner=20, seed=1000,
        n_events=(8, 16), tau_range=(0.2, 0.0), v_range=(1400.0, 4000.0), amp=1.0,
        interf_frac=(0.3, 0.5), interf_amp=(3.0, 10.0), interf_delay=(0.0, 2.0),
        tau_frac_of_record=0.85)
    v, t = _panels(np.linspace(1400.0, 4000.0, 24), tuple(range(0, 80, 5)))
    out["aashrt-1024x256-nv24x16"] = Workload(
        name="aashrt-1024x256-nv24x16", nt=1024, nx=256, dt=0.004, dx=12.5, vel=v, tau0=t,
        p=2, q=1, n_outer=10, n_inner=20, seed=4,
        n_events=(6, 6), tau_range=(0.2, 3.6), v_range=(1400.0, 4000.0), amp=1.0,
        interf_frac=(0.0, 0.0), n_diffractors=20, diff_t0_range=(0.0, 0.3), diff_amp=0.5,
        decimate_frac=0.5)
    return out


WORKLOADS = _mk()


def workload(name: str, **overrides) -> Workload:
    """Return a named workload, optionally with fields replaced."""
    w = WORKLOADS[name]
    if overrides:
        d = dict(w.__dict__)
        d.update(overrides)
        w = Workload(**d)
    return w
