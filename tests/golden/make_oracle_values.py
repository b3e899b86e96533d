"""Write tests/golden/oracle_separation.json: the FP64 oracle's separation
quality on the seeded synthetic workloads, used as the fixed-SNR target of
the benchmark (a GPU solve counts only if its Q_R is within 0.05 dB of the
oracle's on the same gather and iteration counts).

Calls only ``oracle`` and ``synth``.  Usage: python tests/golden/make_oracle_values.py [names...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle.irls import IrlsParams  # noqa: E402
from synth import make_gather, workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_separation.json")


def run(name):
    w = workload(name)
    gth = make_gather(w)
    g = oracle.geometry(gth.nt, gth.nx, w.dt, w.dx, w.vel, tau0=w.tau0, fmax=w.fmax, R=w.half_width)
    d = gth.d_blend.astype(np.float32).astype(np.float64)   # what the GPU sees
    prm = IrlsParams(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)
    t0 = time.time()
    _, drec, rep = oracle.robust_invert(g, d, prm, mask=gth.mask if w.decimate_frac > 0 else None)
    t = time.time() - t0
    return {
        "workload": name, "seed": w.seed, "p": w.p, "q": w.q,
        "n_outer": w.n_outer, "n_inner": w.n_inner,
        "q_pd_db": oracle.q_db(gth.d_clean, gth.d_blend),
        "q_r_db": oracle.q_db(gth.d_clean, drec),
        "misfit": rep["misfit"], "eps_r": rep["eps_r"],
        "oracle_seconds": t,
    }


if __name__ == "__main__":
    names = sys.argv[1:] or ["crg-256x64-nv8", "crg-1024x256-nv32"]
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    for n in names:
        print("oracle solve", n, flush=True)
        data[n] = run(n)
        print(json.dumps(data[n]), flush=True)
        json.dump(data, open(OUT, "w"), indent=1)
