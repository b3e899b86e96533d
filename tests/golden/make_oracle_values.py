"""Write tests/golden/oracle_separation.json: the FP64 oracle's separation
quality on the seeded synthetic workloads, used as the fixed-SNR target of
the benchmark (a GPU solve counts only if its Q_R is within 0.05 dB of the
oracle's on the same gather and iteration counts); and, with --operator,
tests/golden/oracle_operator_samples.json: the oracle's forward and adjoint
of seeded random inputs at a workload's full size, as norms plus sampled
output values (full-size operator parity where the oracle is too slow to
run inside a test).

Calls only ``oracle`` and ``synth``.  Usage:
    python tests/golden/make_oracle_values.py [names...]
    python tests/golden/make_oracle_values.py --operator [names...]
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
OUT_OP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_operator_samples.json")
N_SAMPLES = 512


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
        "misfit": rep["misfit"], "eps_r": rep["eps_r"], "eps_m": rep["eps_m"], "huber": rep["huber"],
        "oracle_seconds": t,
    }


def operator_samples(name, seed=77):
    """Oracle forward of a seeded Gaussian model and adjoint of seeded
    Gaussian data (both FP32-rounded, the workload's mask applied), stored
    as norms and values at seeded sample positions."""
    from synth import random_data, random_model
    w = workload(name)
    gth = make_gather(w)
    g = oracle.geometry(gth.nt, gth.nx, w.dt, w.dx, w.vel, tau0=w.tau0, fmax=w.fmax, R=w.half_width)
    mask = gth.mask if w.decimate_frac > 0 else None
    rng = np.random.default_rng(seed)
    m = random_model(rng, g.npanel, g.nx, g.nt, np.float32).astype(np.float64)
    d = random_data(rng, g.nx, g.nt, np.float32).astype(np.float64)
    fwd = oracle.forward(g, m, mask)
    adj = oracle.adjoint(g, d, mask)
    srng = np.random.default_rng(seed + 1)
    fi = srng.integers(0, fwd.size, N_SAMPLES)
    ai = srng.integers(0, adj.size, N_SAMPLES)
    return {
        "workload": name, "input_seed": seed,
        "forward_norm": float(np.linalg.norm(fwd)), "adjoint_norm": float(np.linalg.norm(adj)),
        "forward_index": fi.tolist(), "forward_value": fwd.ravel()[fi].tolist(),
        "adjoint_index": ai.tolist(), "adjoint_value": adj.ravel()[ai].tolist(),
    }


if __name__ == "__main__":
    if sys.argv[1:2] == ["--operator"]:
        names = sys.argv[2:] or ["aashrt-1024x256-nv24x16"]
        data = json.load(open(OUT_OP)) if os.path.exists(OUT_OP) else {}
        for n in names:
            print("oracle operator samples", n, flush=True)
            data[n] = operator_samples(n)
            json.dump(data, open(OUT_OP, "w"), indent=1)
        sys.exit(0)
    names = sys.argv[1:] or ["crg-256x64-nv8", "crg-1024x256-nv32"]
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    for n in names:
        print("oracle solve", n, flush=True)
        data[n] = run(n)
        print(json.dumps(data[n]), flush=True)
        json.dump(data, open(OUT, "w"), indent=1)
