"""Write the stored FP64 oracle values the GPU tests and the benchmark compare
against, for workloads whose oracle runs are too slow to repeat inside a test.

* tests/golden/oracle_separation.json: per workload, the oracle's robust
  solve (IRLS-CG at the workload's iteration counts, or the counts given in
  the name): separation quality Q_R and Q_PD (thesis Chapter 4, equations
  ch4_Qpd and ch4_Qr), the per-outer-iteration misfit, clips and objective,
  and the separated gather d_rec = L m and the model m as norms plus values
  at seeded sample positions (element-wise parity at full size).  Q_R is the
  benchmark's fixed-SNR target: a GPU solve counts only if its Q_R is within
  0.05 dB of the oracle's on the same gather and iteration counts.
* with --operator, tests/golden/oracle_operator_samples.json: the oracle's
  forward and adjoint of seeded Gaussian inputs at full size, as norms plus
  sampled output values.
* with --batch-subset FIRST N: Q_R, Q_PD and misfits of the oracle's solves
  of gathers FIRST .. FIRST+N-1 of the 512-gather batched workload (the
  benchmark's fixed-SNR check of the batched solve), stored under
  "batch512-crg-nv24" -> "gathers".

Workload names are those of ``synth.workload``; "batch512-crg-nv24:g31"
names gather 31 of the batched workload, and a suffix ":2x5" overrides the
outer x inner iteration counts.

Long runs can be split over processes: --out PATH writes a partial file,
--merge [--operator] PATH... folds partial files into the stored one.

Calls only ``oracle`` and ``synth``.  Usage:
    python tests/golden/make_oracle_values.py [--out PATH] [names...]
    python tests/golden/make_oracle_values.py --operator [--out PATH] [names...]
    python tests/golden/make_oracle_values.py --batch-subset FIRST N [--out PATH]
    python tests/golden/make_oracle_values.py --merge [--operator] PATH...
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
from synth import make_cfg3_batch, make_gather, workload  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "oracle_separation.json")
OUT_OP = os.path.join(HERE, "oracle_operator_samples.json")
N_SAMPLES = 512          # operator outputs
N_SOLVE_SAMPLES = 4096   # separated gather and model of a solve
BATCH = "batch512-crg-nv24"


def resolve(name):
    """(workload, gather, n_outer, n_inner) for a workload name, optionally
    with ":g<index>" (a gather of the batched workload) and ":<o>x<i>"."""
    parts = name.split(":")
    w = workload(parts[0])
    gth = None
    n_outer, n_inner = w.n_outer, w.n_inner
    for s in parts[1:]:
        if s.startswith("g"):
            gth = make_cfg3_batch(w, 1, int(s[1:]))[0]
        else:
            o, i = s.split("x")
            n_outer, n_inner = int(o), int(i)
    if gth is None:
        gth = make_gather(w)
    return w, gth, n_outer, n_inner


def _geometry(w, gth):
    return oracle.geometry(gth.nt, gth.nx, w.dt, w.dx, w.vel, tau0=w.tau0, fmax=w.fmax, R=w.half_width)


def _sample(arr, rng, n):
    idx = rng.integers(0, arr.size, n)
    return idx.tolist(), np.asarray(arr).ravel()[idx].tolist()


def run(name, samples=True):
    w, gth, n_outer, n_inner = resolve(name)
    g = _geometry(w, gth)
    d = gth.d_blend.astype(np.float32).astype(np.float64)   # what the GPU sees
    prm = IrlsParams(p=w.p, q=w.q, n_outer=n_outer, n_inner=n_inner)
    t0 = time.time()
    m, drec, rep = oracle.robust_invert(g, d, prm, mask=gth.mask if w.decimate_frac > 0 else None)
    t = time.time() - t0
    out = {
        "workload": name, "seed": gth.seed, "nt": gth.nt, "nx": gth.nx, "p": w.p, "q": w.q,
        "n_outer": n_outer, "n_inner": n_inner,
        "q_pd_db": oracle.q_db(gth.d_clean, gth.d_blend),
        "q_r_db": oracle.q_db(gth.d_clean, drec),
        "misfit": rep["misfit"], "eps_r": rep["eps_r"], "eps_m": rep["eps_m"], "huber": rep["huber"],
        "oracle_seconds": t,
    }
    if samples:
        srng = np.random.default_rng(gth.seed + 101)
        di, dv = _sample(drec, srng, N_SOLVE_SAMPLES)
        mi, mv = _sample(m, srng, N_SOLVE_SAMPLES)
        out.update({
            "drec_norm": float(np.linalg.norm(drec)), "drec_index": di, "drec_value": dv,
            "drec_trace_norm": np.linalg.norm(drec, axis=1).tolist(),
            "m_norm": float(np.linalg.norm(m)), "m_index": mi, "m_value": mv,
        })
    return out


def operator_samples(name, seed=77):
    """Oracle forward of a seeded Gaussian model and adjoint of seeded
    Gaussian data (both FP32-rounded, the workload's mask applied), stored
    as norms and values at seeded sample positions."""
    from synth import random_data, random_model
    w, gth, _, _ = resolve(name)
    g = _geometry(w, gth)
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
        "workload": name, "input_seed": seed, "nt": gth.nt, "nx": gth.nx,
        "forward_norm": float(np.linalg.norm(fwd)), "adjoint_norm": float(np.linalg.norm(adj)),
        "forward_index": fi.tolist(), "forward_value": fwd.ravel()[fi].tolist(),
        "adjoint_index": ai.tolist(), "adjoint_value": adj.ravel()[ai].tolist(),
    }


def batch_subset(first, n):
    """Oracle 10 x 20 solves of gathers first .. first+n-1 of the batch:
    Q_R, Q_PD and the misfit per outer iteration (no samples)."""
    out = {}
    for gi in range(first, first + n):
        r = run(f"{BATCH}:g{gi}", samples=False)
        print(f"  gather {gi}: nt {r['nt']} nx {r['nx']} Q_R {r['q_r_db']:.4f} dB "
              f"({r['oracle_seconds']:.0f} s)", flush=True)
        out[str(gi)] = r
    return out


def _load(path):
    return json.load(open(path)) if os.path.exists(path) else {}


def _save(path, data):
    tmp = path + ".tmp"
    json.dump(data, open(tmp, "w"), indent=1)
    os.replace(tmp, path)


def _merge_into(data, part):
    for k, v in part.items():
        if k == BATCH and isinstance(v, dict) and "gathers" in v:
            data.setdefault(BATCH, {"gathers": {}})
            data[BATCH].setdefault("gathers", {}).update(v["gathers"])
        else:
            data[k] = v


def main(argv):
    out = None
    if "--out" in argv:
        i = argv.index("--out")
        out = argv[i + 1]
        argv = argv[:i] + argv[i + 2:]
    if argv[:1] == ["--merge"]:
        argv = argv[1:]
        target = OUT
        if argv[:1] == ["--operator"]:
            target, argv = OUT_OP, argv[1:]
        data = _load(target)
        for p in argv:
            _merge_into(data, json.load(open(p)))
        _save(target, data)
        return
    if argv[:1] == ["--operator"]:
        names = argv[1:] or ["aashrt-1024x256-nv24x16"]
        path = out or OUT_OP
        for n in names:
            print("oracle operator samples", n, flush=True)
            data = _load(path)
            data[n] = operator_samples(n)
            _save(path, data)
        return
    if argv[:1] == ["--batch-subset"]:
        first, n = int(argv[1]), int(argv[2])
        path = out or OUT
        res = batch_subset(first, n)
        data = _load(path)
        _merge_into(data, {BATCH: {"gathers": res}})
        _save(path, data)
        return
    names = argv or ["crg-256x64-nv8", "crg-1024x256-nv32"]
    path = out or OUT
    for n in names:
        print("oracle solve", n, flush=True)
        r = run(n)
        data = _load(path)
        data[n] = r
        _save(path, data)
        print(json.dumps({k: v for k, v in r.items() if not k.endswith(("_index", "_value", "_norm"))}),
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
