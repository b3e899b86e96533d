#!/usr/bin/env python3
"""Benchmark of the robust Stolt-ASHRT separation on one MI355X.

A step is one whole IRLS-CG solve (10 reweightings x 20 CG iterations, l1
misfit, l2 model norm) of the production-size blended receiver gather
(1024 samples x 256 traces, dt 4 ms, dx 12.5 m, 32 velocities over
1400-4000 m/s), zero start, inputs resident in HBM.  ``value`` is gathers
solved per second; a solve counts only if its separated-signal SNR Q_R is
within 0.05 dB of the FP64 oracle's on the same gather and iteration counts
(stored in tests/golden/oracle_separation.json by a script that calls only
the oracle).

Also reported: forward+adjoint operator pairs per second, a roofline entry
for the dominant kernel (average launch time from HIP events recorded
around that kernel's launches on its stream, during the timed steps), and
the FP64 oracle timed on the host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak (counts packed FP32)
# The kernels are built without packed FP32, so their ceiling is one FP32 FMA
# per lane per clock: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
FP32_UNPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


# HBM bytes per launch of the row kernels on the production gather, by the
# plan's panel-chunk count (which sets their grid), from rocprofv3 --pmc
# FETCH_SIZE and --pmc WRITE_SIZE (KiB per dispatch) scaled by what the
# counters read for a 512 MiB device copy (reads x 2.0, writes x 1.0); valid
# only for the kernel sources with this digest.
_MIB = 1024.0 * 1024.0
MEASURED_TRAFFIC = {
    "digest": "ec246944c773b23e",
    "workload": "crg-1024x256-nv32",
    "bytes": {
        # nchunk -> read + write
        "k_rows_fwd": {1: (56.15 + 3.20) * _MIB, 2: (56.19 + 6.41) * _MIB, 4: (56.27 + 12.81) * _MIB,
                       8: (56.45 + 25.60) * _MIB},
        "k_rows_adj": {1: (2.32 + 55.92) * _MIB, 2: (4.36 + 55.92) * _MIB, 4: (8.45 + 55.92) * _MIB,
                       8: (16.67 + 55.92) * _MIB},
    },
}
_KERNEL_SOURCES = ["ashrt_internal.h", "block_reduce.h", "fft_lds.h", "fft_tpl.h", "kernels.h", "op_kernels.hip"]


def _kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in _KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_10214_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _measured_traffic(workload, kernel, nchunk):
    t = MEASURED_TRAFFIC
    if t["workload"] != workload or t["digest"] != _kernel_digest():
        return None
    return t["bytes"].get(kernel, {}).get(nchunk)


def fft_len(n):
    """Smallest 2^a or 3 * 2^a >= 2 n (the library's default padding)."""
    best, p = None, 1
    while p < 4 * n + 8:
        for c in (p, 3 * p):
            if c >= 2 * n and (best is None or c < best):
                best = c
        p *= 2
    return best


def _geometry_numbers(info, vel, dt, dx, nx, nt, P, R, cg_frac=0.0):
    """Per launch of each operator kernel family on one gather: (algorithmic
    bytes, method flops).

    Bytes are the kernel's compulsory traffic: what it must read and write
    in this decomposition (x-spectra only for the wavenumber rows that can
    reach the band; the forward's panel-sum partials once; the adjoint's data
    spectrum once, although each panel chunk re-reads it).  Flops are the
    method's: 5 N log2 N per complex FFT of length N (one time FFT per live
    model row and per data row, one x FFT per pair of time columns) and one
    complex-by-real multiply-add (4 flop) per tap of every in-cone map output.
    cg_frac: the fraction of model-transform launches that also apply the
    previous CG iteration's update (read m, g; write m, pdir: four more model
    streams)."""
    import numpy as np
    ntp, nxp, jlo, jhi = info["ntp"], info["nxp"], info["jlo"], info["jhi"]
    nrows = nxp // 2
    nband = jhi - jlo + 1
    f4, c8 = 4, 8
    model_b = P * nx * nt * f4
    data_b = nx * nt * f4
    bin_ = ntp * dt / (nxp * dx)
    live_rows = 0
    for v in vel:
        c2 = (v * bin_) ** 2
        rl = nrows if c2 <= 0 else min(nrows, 1 + sum(1 for r in range(1, nrows) if c2 * r * r <= jhi * jhi * (1 + 1e-9)))
        live_rows += rl
    X_b = live_rows * nt * c8
    H_b = nrows * nt * c8
    D_b = nrows * 2 * nband * c8
    fft_t = 5.0 * ntp * math.log2(ntp)
    fft_x = 5.0 * nxp * math.log2(nxp)
    j = np.arange(jlo, jhi + 1, dtype=np.float64)
    l = np.arange(nrows, dtype=np.float64)
    cone = 0
    for v in vel:
        a_up = v * bin_ * l
        a_lo = v * bin_ * np.where(l == 0, nrows, l)
        cone += int(np.sum(j[None, :] >= a_up[:, None])) + int(np.sum(j[None, :] >= a_lo[:, None]))
    map_flops = cone * 2 * R * 4
    return {
        "k_xfft_fwd(model)": (model_b + X_b + cg_frac * 4 * model_b, P * math.ceil(nt / 2) * fft_x),
        "k_xfft_fwd(data)": (data_b + H_b, math.ceil(nt / 2) * fft_x),
        "k_rows_fwd": (X_b + D_b, live_rows * fft_t + map_flops),
        "k_rows_fwd_fin": (D_b + H_b, nrows * fft_t),
        "k_xfft_inv(data)": (H_b + data_b, math.ceil(nt / 2) * fft_x),
        "k_rows_adj": (H_b + X_b, (nrows + live_rows) * fft_t + map_flops),
        "k_xfft_inv(model)": (X_b + model_b, P * math.ceil(nt / 2) * fft_x),
    }


def _roofline(dom, bytes_, flops, avg_s, launches, traffic):
    """Roofline entry of the dominant kernel: bound by HBM bandwidth (the
    operator's roofline), with its FP32 issue rate beside it."""
    ach = bytes_ / avg_s / 1e9
    alu = flops / avg_s / 1e12
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic, "kernel": dom, "avg_launch_us": avg_s * 1e6, "launches_timed": launches,
            "algorithmic_bytes_per_launch": bytes_, "method_flops_per_launch": flops,
            "alu_achieved_tflops": alu, "alu_peak_tflops": FP32_UNPACKED_PEAK_TFLOPS,
            "alu_frac": alu / FP32_UNPACKED_PEAK_TFLOPS}


def _profile_solve(lib, L, solve, reps=1):
    """Per-kernel time per solve from the library's HIP-event timing (events
    recorded around every launch on its stream), over reps solves; returns
    the per-kernel table and the wall time of the reps solves."""
    import ctypes as C
    import torch
    torch.cuda.synchronize()
    lib.ashrt_profile_enable((1 << L.K_COUNT) - 1)
    t0 = time.perf_counter()
    last = None
    for _ in range(reps):
        last = solve()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lib.ashrt_profile_enable(0)
    out = {}
    for k in range(L.K_COUNT):
        tot, n = C.c_double(), C.c_int64()
        L.check(lib.ashrt_profile_read(k, C.byref(tot), C.byref(n), 1), "ashrt_profile_read")
        out[lib.ashrt_kernel_name(k).decode()] = {"ms_total_per_solve": tot.value / reps,
                                                  "launches": n.value // reps, "kid": k}
    return out, wall, last


def _q_db(clean, est):
    """Separation quality 10 log10(|clean|^2 / |clean - est|^2) (thesis
    Chapter 4, equations ch4_Qpd and ch4_Qr)."""
    import numpy as np
    c = np.asarray(clean, dtype=np.float64)
    e = np.asarray(est, dtype=np.float64)
    return float(10.0 * np.log10(np.sum(c * c) / np.sum((c - e) ** 2)))


def _host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def _oracle_sample(args):
    """One bounded oracle sample on the host, in its own process with one
    thread: the Stolt-map set-up plus a 1 x 3 solve of the gather, scaled to
    the full solve by counting operator applications.  Returns seconds per
    gather and the parts."""
    name, n_outer_full, n_inner_full = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    import numpy as np
    import oracle
    from oracle.irls import IrlsParams
    from synth import make_gather, workload
    w = workload(name)
    gth = make_gather(w)
    g = oracle.geometry(gth.nt, gth.nx, w.dt, w.dx, w.vel, tau0=w.tau0, fmax=w.fmax, R=w.half_width)
    d = gth.d_blend.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    for p in range(g.npanel):
        oracle.stolt_matrix(g, p)
    t_setup = time.perf_counter() - t0
    n_outer, n_inner = 1, 3
    t1 = time.perf_counter()
    oracle.robust_invert(g, d, IrlsParams(p=w.p, q=w.q, n_outer=n_outer, n_inner=n_inner))
    t_sample = time.perf_counter() - t1
    apps_sample = 1 + n_outer * (2 * n_inner + 2)
    apps_full = 1 + n_outer_full * (2 * n_inner_full + 2)
    return t_setup + t_sample * apps_full / apps_sample, t_setup, t_sample, apps_sample, apps_full


def cpu_baseline(w, gth):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    gather.  One thread; and every core of the host's share running
    independent samples at once (gathers are independent, so that is the
    oracle's whole-host throughput)."""
    from concurrent.futures import ProcessPoolExecutor
    job = (w.name, w.n_outer, w.n_inner)
    with ProcessPoolExecutor(max_workers=1) as ex:
        t_full, t_setup, t_sample, apps_sample, apps_full = ex.submit(_oracle_sample, job).result()
    ncpu = os.cpu_count() or 1
    workers = max(1, min(ncpu, 16))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(_oracle_sample, [job] * workers))
    wall = time.perf_counter() - t0
    all_rate = sum(1.0 / r[0] for r in res)
    return {
        "value": 1.0 / t_full, "unit": "gathers/s", "cores": 1, "kind": "oracle",
        "host_cpu": _host_cpu(), "host_cpu_count": ncpu,
        "sample": (f"FP64 numpy/scipy oracle, one thread: stolt-map set-up {t_setup:.2f} s plus a 1x3 "
                   f"IRLS-CG solve of the same gather ({apps_sample} operator applications, {t_sample:.2f} s), "
                   f"scaled to the {w.n_outer}x{w.n_inner} solve ({apps_full} applications): "
                   f"{t_full:.1f} s per gather"),
        "all_cores": {"value": all_rate, "unit": "gathers/s", "cores": workers, "kind": "oracle",
                      "sample": (f"{workers} independent one-thread samples as above run at once on "
                                 f"{workers} of the host's {ncpu} cores ({wall:.1f} s wall); value = sum of "
                                 f"their per-gather rates (the oracle itself is single-threaded)")},
    }


def _gen_gather(args):
    from synth import make_gather, workload
    name, seed = args
    g = make_gather(workload(name), seed=seed)
    return g.d_blend.astype("float32"), g.d_clean


def _gen_batch_gather(args):
    from synth import make_gather, workload
    name, nt, nx, seed = args
    g = make_gather(workload(name), seed=seed, nt=nt, nx=nx)
    return g.d_blend.astype("float32"), g.d_clean.astype("float32")


def _draw_batch(n, name="batch512-crg-nv24"):
    """The batched workload's gathers, drawn on host worker processes (call
    before the GPU is touched)."""
    from concurrent.futures import ProcessPoolExecutor
    from synth import batch_shapes, workload
    w = workload(name)
    shapes = batch_shapes(n, w.seed)
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        gathers = list(ex.map(_gen_batch_gather, [(w.name, nt, nx, s) for nt, nx, s in shapes]))
    return w, shapes, gathers


def _band(ntp, dt, fmax):
    jhi = ntp // 2 - 1
    if fmax > 0:
        jhi = min(jhi, int(math.floor(fmax * ntp * dt)))
    return 1, jhi


def _workload_roofline(prof, per_gather_nums, classes):
    """Dominant operator kernel of a workload over one solve: its algorithmic
    bytes per solve (every gather passes through each launch family once per
    operator application; a family launches once per FFT size class) over its
    total time."""
    ops = [k for k in prof if k.startswith(("k_xfft", "k_rows")) and prof[k]["launches"] > 0]
    dom = max(ops, key=lambda k: prof[k]["ms_total_per_solve"])
    n_cls = classes["rows" if dom.startswith("k_rows") else "x"]
    passes = prof[dom]["launches"] / n_cls
    bytes_ = sum(g[dom][0] for g in per_gather_nums) * passes
    flops = sum(g[dom][1] for g in per_gather_nums) * passes
    t = prof[dom]["ms_total_per_solve"] / 1e3
    r = _roofline(dom, bytes_, flops, t, prof[dom]["launches"], None)
    r["avg_launch_us"] = t / max(prof[dom]["launches"], 1) * 1e6
    r["algorithmic_bytes_per_solve"] = r.pop("algorithmic_bytes_per_launch")
    r["method_flops_per_solve"] = r.pop("method_flops_per_launch")
    r["ms_per_solve"] = t * 1e3
    return r


def batch_leg(w, shapes, gathers, steps, warmup):
    """The batched workload: every gather solved by robust_invert_batched
    (10 x 20, l1 misfit), all stages one launch per FFT size class.  Fixed
    SNR: gathers 0..15 must reach the FP64 oracle's Q_R (stored by
    tests/golden/make_oracle_values.py --batch-subset) within 0.05 dB."""
    import numpy as np
    import torch
    import paper_1711_10214_amd as A
    from paper_1711_10214_amd import _lib as L
    descs = [dict(nt=nt, nx=nx, dt=w.dt, dx=w.dx, vel=list(w.vel), fmax=w.fmax, half_width=w.half_width)
             for nt, nx, _ in shapes]
    plan = A.BatchPlan(descs)
    d = plan.pack_data([g for g, _ in gathers])
    prm = A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)
    print(f"[bench] batch of {len(shapes)} gathers: model {plan.model_total * 4 / 2**30:.1f} GiB, "
          f"data {plan.data_total * 4 / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    for _ in range(max(warmup, 1)):
        plan.robust_invert(d, prm, want_report=False)
    # timed solves, with HIP events around every launch (a few per stage)
    prof, wall, out = _profile_solve(L.lib(), L, lambda: plan.robust_invert(d, prm, want_report=False), steps)
    _, drec, _ = out
    q = []
    for gi, (g, clean) in enumerate(gathers):
        rec = plan.unpack_data(drec, gi).cpu().numpy()
        q.append((_q_db(clean, rec), _q_db(clean, g)))
    q = np.array(q)
    fixed = {"checked": 0, "reached": 0, "worst_margin_db": None}
    gold = os.path.join(ROOT, "tests", "golden", "oracle_separation.json")
    if os.path.exists(gold):
        ref = json.load(open(gold)).get(w.name, {}).get("gathers", {})
        margins = []
        for k, r in ref.items():
            gi = int(k)
            if gi < len(shapes) and (r["nt"], r["nx"]) == shapes[gi][:2] and (r["n_outer"], r["n_inner"]) == (
                    w.n_outer, w.n_inner):
                margins.append(q[gi, 0] - r["q_r_db"])
        if margins:
            fixed = {"checked": len(margins), "reached": int(sum(m >= -0.05 for m in margins)),
                     "worst_margin_db": float(min(margins)), "max_abs_diff_db": float(max(abs(m) for m in margins))}
    nums = []
    for nt, nx, _ in shapes:
        ntp, nxp = fft_len(nt), fft_len(nx)
        jlo, jhi = _band(ntp, w.dt, w.fmax)
        info = {"ntp": ntp, "nxp": nxp, "jlo": jlo, "jhi": jhi}
        nums.append(_geometry_numbers(info, w.vel, w.dt, w.dx, nx, nt, w.npanel, w.half_width,
                                      cg_frac=(w.n_inner - 1) / (w.n_inner + 1)))
    classes = {"rows": len(set(fft_len(nt) for nt, _, _ in shapes)),
               "x": len(set(fft_len(nx) for _, nx, _ in shapes))}
    return {
        "value": len(shapes) * steps / wall, "unit": "gathers/s", "ms_per_step": wall / steps * 1e3,
        "steps": steps, "config": {"workload": w.name, "gathers": len(shapes), "npanel": w.npanel,
                                   "n_outer": w.n_outer, "n_inner": w.n_inner,
                                   "nt_set": sorted(set(s[0] for s in shapes)),
                                   "nx_range": [min(s[1] for s in shapes), max(s[1] for s in shapes)],
                                   "model_gib": plan.model_total * 4 / 2**30},
        "snr": {"q_r_db_mean": float(q[:, 0].mean()), "q_pd_db_mean": float(q[:, 1].mean()),
                "improved": int((q[:, 0] > q[:, 1]).sum()), "fixed_snr_vs_oracle": fixed},
        "kernels_ms_per_solve": {k: round(v["ms_total_per_solve"], 3) for k, v in prof.items() if v["launches"]},
        "roofline": _workload_roofline(prof, nums, classes),
    }


def aashrt_leg(steps, warmup, autotune=True):
    """The asymptote-shifted diffraction gather (1024 x 256, 24 velocities x
    16 asymptote shifts = 384 panels, half the traces decimated, p 2, q 1,
    10 x 20): gathers/s, with Q (against the complete clean gather) checked
    against the FP64 oracle's stored solve."""
    import torch
    import paper_1711_10214_amd as A
    from paper_1711_10214_amd import _lib as L
    from synth import make_gather, workload
    w = workload("aashrt-1024x256-nv24x16")
    gth = make_gather(w)
    plan = A.Plan(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), tau0=list(w.tau0), fmax=w.fmax,
                  half_width=w.half_width, tuning="auto" if autotune else None)
    d = torch.tensor(gth.d_blend, dtype=torch.float32, device="cuda")
    mask = torch.tensor(gth.mask, device="cuda")
    prm = A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)

    def solve():
        return plan.robust_invert(d, prm, mask=mask, want_report=False)

    for _ in range(max(warmup, 1)):
        solve()
    prof, wall, out = _profile_solve(L.lib(), L, solve, steps)
    q_r = _q_db(gth.d_clean, out[1].cpu().numpy())
    snr = {"q_r_db": q_r, "q_pd_db": _q_db(gth.d_clean, gth.d_blend)}
    gold = os.path.join(ROOT, "tests", "golden", "oracle_separation.json")
    if os.path.exists(gold):
        ref = json.load(open(gold)).get(w.name)
        if ref and (ref["n_outer"], ref["n_inner"]) == (w.n_outer, w.n_inner):
            snr["oracle_q_r_db"] = ref["q_r_db"]
            snr["reached"] = bool(q_r >= ref["q_r_db"] - 0.05)
    info = plan.info
    nums = _geometry_numbers(info, plan.vel, w.dt, w.dx, gth.nx, gth.nt, w.npanel, w.half_width,
                             cg_frac=(w.n_inner - 1) / (w.n_inner + 1))
    r = _workload_roofline(prof, [nums], {"rows": 1, "x": 1})
    return {"value": steps / wall, "unit": "gathers/s", "ms_per_step": wall / steps * 1e3, "steps": steps,
            "config": {"workload": w.name, "nt": gth.nt, "nx": gth.nx, "npanel": w.npanel, "p": w.p, "q": w.q,
                       "n_outer": w.n_outer, "n_inner": w.n_inner, "decimated_traces": int((gth.mask == 0).sum()),
                       "tiling": {k: info[k] for k in ("tile_model", "tile_data", "nchunk")}},
            "snr": snr,
            "kernels_ms_per_solve": {k: round(v["ms_total_per_solve"], 3) for k, v in prof.items() if v["launches"]},
            "roofline": r}


def run_batch(args):
    """The batched workload alone (--workload batch512-crg-nv24)."""
    w, shapes, gathers = _draw_batch(args.batch_gathers, args.workload)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    leg = batch_leg(w, shapes, gathers, args.steps, args.warmup)
    rec = {"metric": "robust ASHRT gathers solved/s (batched, IRLS-CG 10x20, l1 misfit)", "n_gpus": 1,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic"}
    rec.update(leg)
    print(json.dumps(rec), flush=True)


def run_speedratio(args):
    """Classical time-domain ASHRT against the Stolt-based operator on the
    same GPU (the thesis' Chapter 5 speed comparison, with and without zero
    padding): median wall time of a forward + adjoint pair for growing
    gathers with 32 velocities."""
    import numpy as np
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    vel = list(np.linspace(1400.0, 4000.0, 32))
    rows = []

    def pair_ms(fwd, adj, m, d, reps):
        for _ in range(2):
            fwd(m), adj(d)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fwd(m)
            adj(d)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    for nx, nt in [(64, 256), (128, 512), (256, 1024), (512, 2048)]:
        rng = np.random.default_rng(nx)
        m = torch.tensor(rng.standard_normal((32, nx, nt)), dtype=torch.float32, device="cuda")
        d = torch.tensor(rng.standard_normal((nx, nt)), dtype=torch.float32, device="cuda")
        padded = A.Plan(nt, nx, 0.004, 12.5, vel, fmax=100.0)
        unpadded = A.Plan(nt, nx, 0.004, 12.5, vel, fmax=100.0, ntp=nt, nxp=nx)
        t_td = pair_ms(padded.td_forward, padded.td_adjoint, m, d, 5)
        t_sp = pair_ms(padded.forward, padded.adjoint, m, d, 20)
        t_su = pair_ms(unpadded.forward, unpadded.adjoint, m, d, 20)
        rows.append({"nx": nx, "nt": nt, "npanel": 32, "time_domain_ms": t_td, "stolt_padded_ms": t_sp,
                     "stolt_unpadded_ms": t_su, "ratio_padded": t_td / t_sp, "ratio_unpadded": t_td / t_su})
        print(f"[bench] {nx}x{nt}: time-domain {t_td:.3f} ms, Stolt padded {t_sp:.3f} ms "
              f"(x{t_td / t_sp:.1f}), unpadded {t_su:.3f} ms (x{t_td / t_su:.1f})", file=sys.stderr, flush=True)
    rec = {"metric": "forward+adjoint pair time, classical time-domain ASHRT / Stolt-based ASHRT",
           "value": rows[-1]["ratio_padded"], "unit": "x (speed-up of the Stolt pair, padded, largest size)",
           "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "speedratio", "npanel": 32, "dt": 0.004, "dx": 12.5}, "sizes": rows}
    print(json.dumps(rec), flush=True)


def run_survey(args):
    """Survey-level separation: blend a seeded cube of shot gathers (one
    vessel, 50 % time compression, dithered firing), pseudo-deblend into
    common receiver gathers, separate all of them in one batched solve and
    re-sort to common source gathers."""
    import numpy as np
    import torch
    import paper_1711_10214_amd as A
    from paper_1711_10214_amd import survey as S
    from synth import make_survey
    ns, nt = args.survey_sources, 1024
    sv = make_survey(ns=ns, nt=nt, n_events=12, seed=11)
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    vel = list(np.linspace(1400.0, 4000.0, 24))
    D = torch.tensor(sv.D, dtype=torch.float32, device="cuda")
    prm = A.Params(p=1, q=2, n_outer=10, n_inner=20)
    b = S.blend(D, sv.fire)
    S.separate(b, sv.fire, ns, nt, sv.dt, sv.dx, vel, prm)   # warm-up (plans, graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = S.blend(D, sv.fire)
    csg = S.separate(b, sv.fire, ns, nt, sv.dt, sv.dx, vel, prm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pseudo = S.deblend(b, sv.fire, ns, nt, receiver_major=False).cpu().numpy()
    q_sep = _q_db(sv.D, csg.cpu().numpy())
    q_pd = _q_db(sv.D, pseudo)
    rec = {"metric": "survey separation: blend + pseudo-deblend + batched robust separation of every receiver "
                     "gather + re-sort, receiver gathers per second",
           "value": ns / wall, "unit": "receiver gathers/s", "n_gpus": 1, "higher_is_better": True,
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "ms_per_step": wall * 1e3,
           "config": {"workload": f"survey-{ns}x{ns}x{nt}", "sources": ns, "receivers": ns, "nt": nt,
                      "compression": 0.5, "dither_s": 0.4, "npanel": 24, "n_outer": 10, "n_inner": 20,
                      "record_samples": int(b.shape[1])},
           "snr": {"q_separated_db": q_sep, "q_pseudo_deblended_db": q_pd}}
    print(json.dumps(rec), flush=True)


# The warm-start leg of the default run: 4096 streamed training gathers
# labelled by the plain solve stopped at outer iteration 3 (where its Q_R
# peaks; a third of the cost of 10), 128 held-out gathers, Q_R curves on 16.
WS_DEFAULT = {"train_gathers": 4096, "heldout_gathers": 128, "label_outer": 3, "passes": 4.0, "curves": 16}


def _ws_prepare(n_train, n_held):
    """Host side of the warm-start workload, started before the GPU is
    touched: worker processes draw the held-out gathers now and keep
    drawing the training gathers lazily while the GPU labels and trains."""
    import multiprocessing as mp
    base = "crg-1024x256-nv32"
    pool = mp.get_context("fork").Pool(processes=max(1, min(16, os.cpu_count() or 1) - 1))
    t0 = time.perf_counter()
    held = pool.map(_gen_gather, [(base, 2_000_000 + i) for i in range(n_held)])
    t_gen = time.perf_counter() - t0
    # the training gathers are drawn only once the leg starts (idle workers
    # do not compete with the host side of other timed work)
    def train_iter():
        return (g for g, _ in pool.imap(_gen_gather, [(base, 1_000_000 + i) for i in range(n_train)], 8))
    return {"base": base, "pool": pool, "held": held, "t_gen": t_gen, "train_iter": train_iter,
            "n_train": n_train, "n_held": n_held}


def warmstart_leg(prep, label_outer=0, ws_buffer=512, passes=4.0, batch=4, ws_curves=16, lam_w=1.0):
    """Learned warm start against the plain zero start on the same GPU: CG
    iterations and wall time to reach the plain method's final separated-
    signal SNR (minus 0.05 dB) on held-out gathers drawn like the
    production gather.  Training labels are streamed: host workers draw
    gathers while the GPU labels them (plain solves; label_outer outer
    iterations, default the workload's) into a rolling buffer and trains on
    it."""
    import numpy as np
    import torch
    import paper_1711_10214_amd as A
    from paper_1711_10214_amd import warmstart as WS
    from synth import workload
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    base, held, n_train, n_held = prep["base"], prep["held"], prep["n_train"], prep["n_held"]
    w = workload(base)
    plan = A.Plan(w.nt, w.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    prm = A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)
    net = A.UNet(w.npanel, base=16)
    net.init_params(seed=0)
    print(f"[bench] warm start: streaming {n_train} training gathers (buffer {ws_buffer})",
          file=sys.stderr, flush=True)
    # labels: the plain solve, with the workload's outer-iteration count or
    # the one given
    n_lab = label_outer or w.n_outer
    prm_lab = A.Params(p=w.p, q=w.q, n_outer=n_lab, n_inner=w.n_inner)
    ws = WS.train_streaming(plan, net, prep["train_iter"](), n_train, prm_lab, A.TrainParams(lr=1e-3, lam_w=lam_w),
                            buffer=ws_buffer, chunk=128, passes=passes, batch=batch, seed=0, log_every=500)
    prep["pool"].close()
    prep["pool"].join()
    torch.cuda.empty_cache()
    # one warm-up of each path
    d0 = torch.tensor(held[0][0], device="cuda")
    WS.outer_to_target(plan, d0, held[0][1], 1e9, prm, max_outer=1)
    WS.outer_to_target(plan, d0, held[0][1], 1e9, prm, ws=ws, max_outer=1)
    rows = []
    for i, (g, clean) in enumerate(held):
        d = torch.tensor(g, device="cuda")
        _, d_rec, _ = plan.robust_invert(d, prm, want_report=False)
        target = WS.q_db(clean, d_rec.cpu().numpy())
        kp, qp, tp_, _ = WS.outer_to_target(plan, d, clean, target, prm)
        kw, qw, tw, start = WS.outer_to_target(plan, d, clean, target, prm, ws=ws)
        rows.append((target, kp, tp_, kw, tw, start, qw))
        if i % 16 == 0:
            print(f"[bench] held-out {i}: target {target:.2f} dB plain k={kp} warm k={kw} ({start})",
                  file=sys.stderr, flush=True)
    # separated-signal SNR after each outer iteration, plain and warm
    # started, with the weights-only start as the ablation of the model
    curves = {"plain": [], "model+weights": [], "weights only": []}
    for g, clean in held[:ws_curves]:
        d = torch.tensor(g, device="cuda")
        for kind in curves:
            qs = []
            for k in range(1, w.n_outer + 1):
                pk = A.Params(p=w.p, q=w.q, n_outer=k, n_inner=w.n_inner)
                if kind == "plain":
                    _, d_rec, _ = plan.robust_invert(d, pk, want_report=False)
                else:
                    _, d_rec, _, _ = WS.warm_solve(plan, ws, d, pk, use_model=(kind == "model+weights"))
                qs.append(WS.q_db(clean, d_rec.cpu().numpy()))
            curves[kind].append(qs)
    q_by_outer = {k: np.mean(np.array(v), axis=0).tolist() for k, v in curves.items() if v}
    kp = np.array([r[1] or 99 for r in rows], float)
    kw = np.array([r[3] or 99 for r in rows], float)
    tp_ = np.array([r[2] for r in rows])
    tw = np.array([r[4] for r in rows])
    reached = sum(r[3] is not None for r in rows)
    starts = [r[5] for r in rows]
    losses = ws.stats.get("losses", [])
    return {
        "metric": "learned warm start: wall time to the plain IRLS-CG separated-signal SNR, plain / warm",
        "value": float(np.mean(tp_) / np.mean(tw)),
        "unit": "x (speed-up of time-to-SNR)",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "bf16 network, f32 solver",
        "data": "synthetic",
        "config": {"workload": "warmstart-crg-1024x256-nv32", "train_gathers": n_train,
                   "label_buffer": ws_buffer, "passes": passes, "heldout_gathers": n_held,
                   "batch": batch, "params": net.n_params, "n_outer": w.n_outer, "n_inner": w.n_inner,
                   "label_outer": n_lab, "lam_w": lam_w, "model_label_scale": ws.m_scale},
        "plain": {"cg_iterations_mean": float(np.mean(kp) * w.n_inner), "outer_median": float(np.median(kp)),
                  "ms_mean": float(np.mean(tp_) * 1e3)},
        "warm": {"cg_iterations_mean": float(np.mean(kw) * w.n_inner), "outer_median": float(np.median(kw)),
                 "ms_mean": float(np.mean(tw) * 1e3), "reached_target": reached,
                 "model_start_rate": float(np.mean([s_ == "model+weights" for s_ in starts])),
                 "fallback_rate": float(np.mean([s_ != "model+weights" for s_ in starts]))},
        "seconds": {"generate_heldout": prep["t_gen"], "label": ws.stats.get("label_s"),
                    "train": ws.stats.get("train_s")},
        "q_r_by_outer_db": {"gathers": min(ws_curves, n_held), **q_by_outer},
        "train_steps": ws.stats.get("steps"),
        "train_loss": [losses[0], losses[-1]] if losses else None,
    }


def run_warmstart(args):
    """The warm-start workload alone (--workload warmstart)."""
    prep = _ws_prepare(args.train_gathers, args.heldout_gathers)
    rec = warmstart_leg(prep, label_outer=args.label_outer, ws_buffer=args.ws_buffer, passes=args.passes,
                        batch=args.batch, ws_curves=args.ws_curves, lam_w=args.lam_w)
    print(json.dumps(rec), flush=True)


def run_separation(args):
    """The separated-signal SNR study alone (--workload separation)."""
    print(json.dumps(separation_leg()), flush=True)


def separation_leg():
    """What limits the separated-signal SNR of the production gather:
    Q_R after each outer iteration of the plain
    solve; Q_R on the interfered and on the clean traces separately; the same
    solver fitting the clean gather alone (no interference: the operator's
    own limit); the non-robust l2 solve; and the solves with the Ricker
    wavelet's amplitude spectrum as Chapter 4's wavelet operator C."""
    import numpy as np
    import torch
    import paper_1711_10214_amd as A
    from synth import make_gather, workload
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    w = workload("crg-1024x256-nv32")
    gth = make_gather(w)
    dev = torch.device("cuda", 0)
    plan = A.Plan(w.nt, w.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    ntp = plan.info["ntp"]
    f = np.arange(ntp // 2 + 1) / (ntp * w.dt)
    ric = (f / w.ricker_hz) ** 2 * np.exp(-(f / w.ricker_hz) ** 2)   # Ricker amplitude spectrum
    ric /= ric.max()
    plan_c = A.Plan(w.nt, w.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax, wavelet=ric)
    d_blend = torch.tensor(gth.d_blend, dtype=torch.float32, device=dev)
    d_clean = torch.tensor(gth.d_clean, dtype=torch.float32, device=dev)
    hit = np.zeros(gth.nx, bool)
    hit[gth.interfered] = True

    def solve(pl, d, k, p=w.p):
        prm = A.Params(p=p, q=w.q, n_outer=k, n_inner=w.n_inner)
        _, d_rec, _ = pl.robust_invert(d, prm, want_report=False)
        return d_rec.cpu().numpy().astype(np.float64)

    def q(est, rows=None):
        c = gth.d_clean if rows is None else gth.d_clean[rows]
        e = est if rows is None else est[rows]
        return _q_db(c, e)

    solve(plan, d_blend, 1)   # warm-up
    by_outer = [q(solve(plan, d_blend, k)) for k in range(1, w.n_outer + 1)]
    final = solve(plan, d_blend, w.n_outer)
    final_c = solve(plan_c, d_blend, w.n_outer)

    # the best a warm start could predict: the plain solve's own final model
    # m* and final residual weights w* (made as the warm start's labels are)
    from paper_1711_10214_amd import warmstart as WS
    prm_f = A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)
    m_star, drec_star, rep_star = plan.robust_invert(d_blend, prm_f)
    w_star = WS.weight_target(d_blend, drec_star, rep_star["eps_r"][-1])

    def started(k, m0=None, w0=None):
        prm = A.Params(p=w.p, q=w.q, n_outer=k, n_inner=w.n_inner)
        _, d_rec, _ = plan.robust_invert(d_blend, prm, m0=m0, w0=w0, want_report=False)
        return q(d_rec.cpu().numpy().astype(np.float64))

    own_start = {
        "model+weights": [started(k, m_star, w_star) for k in (1, 2, 3)],
        "model only": [started(k, m_star, None) for k in (1, 2, 3)],
        "weights only": [started(k, None, w_star) for k in (1, 2, 3)],
    }
    rec = {
        "metric": "separated-signal SNR Q_R of the production gather under controlled changes (dB)",
        "value": by_outer[-1], "unit": "dB", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "separation-crg-1024x256-nv32", "p": w.p, "q": w.q, "n_outer": w.n_outer,
                   "n_inner": w.n_inner, "interfered_traces": int(hit.sum()), "nx": gth.nx},
        "q_pd_db": q(gth.d_blend),
        "q_r_by_outer_db": by_outer,
        "q_r_interfered_traces_db": q(final, hit),
        "q_r_clean_traces_db": q(final, ~hit),
        "q_pd_interfered_traces_db": q(gth.d_blend, hit),
        "clean_gather_fit_db": q(solve(plan, d_clean, w.n_outer)),
        "clean_gather_fit_l2_db": q(solve(plan, d_clean, w.n_outer, p=2)),
        "blended_l2_solve_db": q(solve(plan, d_blend, w.n_outer, p=2)),
        "start_from_own_solution_q_r_by_outer_db": own_start,
        "wavelet_c": {"q_r_db": q(final_c), "q_r_interfered_traces_db": q(final_c, hit),
                      "q_r_clean_traces_db": q(final_c, ~hit),
                      "clean_gather_fit_db": q(solve(plan_c, d_clean, w.n_outer))},
    }
    return rec


BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix-core peak


def _unet_conv_flops(H, W, base=16, cin=1):
    """Algorithmic FLOPs of the U-Net's eighteen 3x3 convolutions for one
    sample at H x W (2 * 9 * ci * co per output pixel): forward, input
    gradient (every layer but the first, whose input is the data) and weight
    gradient.  Same layer list as the library's graph (five levels, two
    convolutions each, skip concatenations on the decoder side)."""
    c1, c2, c3, c4, c5 = base, 2 * base, 4 * base, 8 * base, 8 * base
    spec = [(cin, c1, 0), (c1, c1, 0), (c1, c2, 1), (c2, c2, 1), (c2, c3, 2), (c3, c3, 2),
            (c3, c4, 3), (c4, c4, 3), (c4, c5, 4), (c5, c5, 4), (c5 + c4, c4, 3), (c4, c4, 3),
            (c4 + c3, c3, 2), (c3, c3, 2), (c3 + c2, c2, 1), (c2, c2, 1), (c2 + c1, c1, 0),
            (c1, c1, 0)]
    fwd = igrad = 0
    for i, (ci, co, lev) in enumerate(spec):
        f = 2 * 9 * ci * co * (H >> lev) * (W >> lev)
        fwd += f
        if i > 0:
            igrad += f
    return fwd, igrad, fwd


def unet_leg(batch=4, steps=20, warmup=3):
    """Training steps (forward, backward, AdamW) and inference of the
    warm-start U-Net at the production gather's shape, against the dense BF16
    matrix-core peak."""
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda", 0)
    B, H, W, P = batch, 256, 1024, 32
    net = A.UNet(P, base=16)
    net.init_params(seed=0)
    g = torch.Generator(device="cpu").manual_seed(0)
    x = torch.randn((B, H, W), generator=g).to(dev)
    t_m = (0.1 * torch.randn((B, P, H, W), generator=g)).to(dev)
    t_w = torch.rand((B, H, W), generator=g).to(dev)
    tp = A.TrainParams(lr=1e-4)
    for _ in range(max(warmup, 1)):
        net.train_step(x, t_m, t_w, tp, want_loss=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        net.train_step(x, t_m, t_w, tp, want_loss=False)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_s = e0.elapsed_time(e1) / 1e3 / steps
    x1 = x[:1].contiguous()
    for _ in range(3):
        net.forward(x1)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        net.forward(x1)
    e1.record()
    torch.cuda.synchronize()
    inf_s = e0.elapsed_time(e1) / 1e3 / steps
    fwd, igrad, wgrad = _unet_conv_flops(H, W)
    step_flops = B * (fwd + igrad + wgrad)
    achieved = step_flops / step_s / 1e12
    rec = {
        "metric": "warm-start U-Net training steps/s (batch 4, 256 x 1024 gathers, 32 output panels)",
        "value": steps / wall, "unit": "steps/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
        "config": {"workload": "unet-train-b4-256x1024-p32", "batch": B, "height": H, "width": W,
                   "out_panels": P, "params": net.n_params},
        "inference_ms_per_gather": inf_s * 1e3,
        "inference_tflops": fwd / inf_s / 1e12,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / BF16_MFMA_PEAK_TFLOPS, "traffic": None,
                     "kernel": "whole training step: algorithmic FLOPs of the 3x3 convolutions "
                               "(forward, input and weight gradients) / step time",
                     "algorithmic_flops_per_step": step_flops},
    }
    return rec


def run_unet(args):
    """The U-Net workload alone (one JSON line)."""
    print(json.dumps(unet_leg(args.batch, args.steps, args.warmup)), flush=True)


def headline(args, w, gth):
    """The production gather's 10 x 20 solve: K timed solves (plain
    launches, HIP events around the dominant kernel's launches on its
    stream), the same solves replayed through the CG hipGraph, and
    forward + adjoint pairs."""
    import numpy as np
    import torch
    import paper_1711_10214_amd as A
    from paper_1711_10214_amd import _lib as L
    import ctypes as C
    dev = torch.device("cuda", 0)
    print(f"[bench] workload {w.name}: nt={gth.nt} nx={gth.nx} P={w.npanel} "
          f"{w.n_outer}x{w.n_inner} p={w.p} q={w.q}", file=sys.stderr, flush=True)
    # tiling chosen by the library's autotuner (timed forward + adjoint pairs)
    plan = A.Plan(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), tau0=list(w.tau0), fmax=w.fmax,
                  half_width=w.half_width, device=0, tuning=None if args.no_autotune else "auto")
    print(f"[bench] tiling {plan.tuning}", file=sys.stderr, flush=True)
    d = torch.tensor(gth.d_blend, dtype=torch.float32, device=dev)
    mask = None if w.decimate_frac == 0 else torch.tensor(gth.mask, device=dev)
    prm = A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)
    lib = L.lib()

    def solve(graph=True):
        prm.cg_graph = graph
        return plan.robust_invert(d, prm, mask=mask, want_report=False)

    for _ in range(max(args.warmup, 1)):
        solve()
    per_kernel, _, _ = _profile_solve(lib, L, solve)
    op_kernels = [k for k in per_kernel if k.startswith(("k_xfft", "k_rows"))]
    dom = max(op_kernels, key=lambda k: per_kernel[k]["ms_total_per_solve"])
    dom_kid = per_kernel[dom]["kid"]
    print("[bench] per-kernel ms per solve: " +
          ", ".join(f"{k}={v['ms_total_per_solve']:.2f}" for k, v in per_kernel.items()),
          file=sys.stderr, flush=True)

    # timed region: K solves; events around the dominant kernel's launches only
    lib.ashrt_profile_enable(1 << dom_kid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(args.steps):
        out = solve(graph=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lib.ashrt_profile_enable(0)
    tot, n = C.c_double(), C.c_int64()
    L.check(lib.ashrt_profile_read(dom_kid, C.byref(tot), C.byref(n), 1), "ashrt_profile_read")
    dom_avg_s = tot.value / max(n.value, 1) / 1e3

    # fixed-SNR check against the oracle's stored separation of this gather,
    # and the separated gather against the stored oracle values element-wise
    m_out, drec, _ = out
    drec_np = drec.cpu().numpy().astype(np.float64)
    q_r = _q_db(gth.d_clean, drec_np)
    snr = {"q_r_db": q_r, "q_pd_db": _q_db(gth.d_clean, gth.d_blend)}
    err = None
    gold = os.path.join(ROOT, "tests", "golden", "oracle_separation.json")
    if os.path.exists(gold):
        ref = json.load(open(gold)).get(w.name)
        if ref and ref["n_outer"] == w.n_outer and ref["n_inner"] == w.n_inner:
            snr["oracle_q_r_db"] = ref["q_r_db"]
            snr["reached"] = bool(q_r >= ref["q_r_db"] - 0.05)
            if "drec_index" in ref:
                idx = np.asarray(ref["drec_index"])
                sv = np.asarray(ref["drec_value"])
                mi = np.asarray(ref["m_index"])
                mv = np.asarray(ref["m_value"])
                mm = m_out.cpu().numpy().astype(np.float64).ravel()
                err = {"d_rec_sampled_rel_l2": float(np.linalg.norm(drec_np.ravel()[idx] - sv) / np.linalg.norm(sv)),
                       "d_rec_norm_rel": float(abs(np.linalg.norm(drec_np) / ref["drec_norm"] - 1)),
                       "m_sampled_rel_l2": float(np.linalg.norm(mm[mi] - mv) / np.linalg.norm(mv)),
                       "samples": int(idx.size), "against": "FP64 oracle solve, stored"}

    # the same solves with the CG iterations replayed from a hipGraph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solve(graph=True)
    torch.cuda.synchronize()
    graph_wall = time.perf_counter() - t0

    # operator pairs per second
    rng = np.random.default_rng(0)
    mm_ = torch.tensor(rng.standard_normal((w.npanel, gth.nx, gth.nt)), dtype=torch.float32, device=dev)
    dd = torch.empty((gth.nx, gth.nt), dtype=torch.float32, device=dev)
    m2 = torch.empty_like(mm_)
    for _ in range(3):
        plan.forward(mm_, out=dd)
        plan.adjoint(dd, out=m2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.pairs):
        plan.forward(mm_, out=dd)
        plan.adjoint(dd, out=m2)
    torch.cuda.synchronize()
    pair_s = (time.perf_counter() - t0) / args.pairs

    # roofline of the dominant kernel; in the solve, the model transforms of
    # CG iterations 1 .. n_inner-1 carry the fused update
    info = plan.info
    nums = _geometry_numbers(info, plan.vel, w.dt, w.dx, gth.nx, gth.nt, w.npanel, w.half_width,
                             cg_frac=(w.n_inner - 1) / (w.n_inner + 1) if w.n_inner > 0 else 0.0)
    bytes_, flops = nums[dom]
    roof = _roofline(dom, bytes_, flops, dom_avg_s, n.value, _measured_traffic(w.name, dom, info["nchunk"]))
    op_nums = _geometry_numbers(info, plan.vel, w.dt, w.dx, gth.nx, gth.nt, w.npanel, w.half_width)
    pair_bytes = sum(v[0] for v in op_nums.values())
    compulsory = 2 * (w.npanel + 1) * gth.nx * gth.nt * 4   # model and data read and written once each
    if args.copy_calibration:
        # plain device copies of known size for the HBM counters: 512 MiB
        # and 4 GiB (16 times the 256 MB last-level cache, so that cache
        # hits cannot hide a share of the reads), each source written first
        # and then pushed out of the caches by a 1 GiB fill
        for n in (128 * 1024 * 1024, 1024 * 1024 * 1024):
            x = torch.empty(n, dtype=torch.float32, device=dev)
            x.fill_(1.0)
            z = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
            z.fill_(2.0)
            y = x.clone()
            torch.cuda.synchronize()
            del x, y, z
    rec = {
        "metric": "robust ASHRT gathers solved/s to fixed SNR (IRLS-CG 10x20, l1 misfit); also fwd+adj pairs/s, HBM GB/s",
        "value": args.steps / wall,
        "unit": "gathers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nt": gth.nt, "nx": gth.nx, "ntp": info["ntp"],
                   "tiling": {"tile_model": info["tile_model"], "tile_data": info["tile_data"],
                              "nchunk": info["nchunk"]},
                   "nxp": info["nxp"], "npanel": w.npanel, "p": w.p, "q": w.q,
                   "n_outer": w.n_outer, "n_inner": w.n_inner, "fmax_hz": w.fmax,
                   "reductions": "f64", "seed": w.seed},
        "graph_gathers_per_s": args.steps / graph_wall,
        "pairs_per_s": 1.0 / pair_s,
        "pair_ms": pair_s * 1e3,
        "pair_algorithmic_gbs": pair_bytes / pair_s / 1e9,
        "pair_compulsory_gbs": compulsory / pair_s / 1e9,
        "snr": snr,
        "error_vs_oracle": err,
        "kernels_ms_per_solve": {k: round(v["ms_total_per_solve"], 4) for k, v in per_kernel.items()},
        "roofline": roof,
    }
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="crg-1024x256-nv32")
    ap.add_argument("--pairs", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched, asymptote-shifted and warm-start workloads after the headline solve")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 512 MiB and a 4 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--train-gathers", type=int, default=4096, help="warm-start workload: training gathers (streamed)")
    ap.add_argument("--ws-buffer", type=int, default=512, help="warm-start workload: resident label buffer")
    ap.add_argument("--passes", type=float, default=4.0, help="warm-start workload: expected uses of each label")
    ap.add_argument("--heldout-gathers", type=int, default=256, help="warm-start workload: held-out gathers")
    ap.add_argument("--lam-w", type=float, default=1.0,
                    help="warm-start workload: weight of the residual-weight term in the training loss")
    ap.add_argument("--label-outer", type=int, default=0,
                    help="warm-start workload: outer iterations of the labelling solves (default: the workload's)")
    ap.add_argument("--ws-curves", type=int, default=16,
                    help="warm-start workload: held-out gathers for the SNR-by-outer-iteration curves")
    ap.add_argument("--batch", type=int, default=4, help="warm-start and unet workloads: batch size")
    ap.add_argument("--batch-gathers", type=int, default=512, help="batched workload: number of gathers")
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in tiling rule")
    ap.add_argument("--survey-sources", type=int, default=128, help="survey workload: sources (= receivers)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library solves each gather on one GPU and has no "
              "multi-GPU path (gathers are independent, so a larger job shards by gather). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload.startswith("warmstart"):
        return run_warmstart(args)
    if args.workload.startswith("batch"):
        return run_batch(args)
    if args.workload == "speedratio":
        return run_speedratio(args)
    if args.workload == "survey":
        return run_survey(args)
    if args.workload == "unet":
        return run_unet(args)
    if args.workload == "separation":
        return run_separation(args)

    from synth import make_gather, workload
    w = workload(args.workload)
    gth = make_gather(w)
    # host work first: worker processes are started before the GPU is touched
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host (bounded samples)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, gth)
    batch_in = ws_prep = None
    if not args.no_extra:
        # warm-start workers first (forked while the process is small and
        # before the GPU is touched), then the batched gathers
        ws_prep = _ws_prepare(WS_DEFAULT["train_gathers"], WS_DEFAULT["heldout_gathers"])
        print(f"[bench] drawing the {args.batch_gathers} batched gathers", file=sys.stderr, flush=True)
        batch_in = _draw_batch(args.batch_gathers)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    rec = headline(args, w, gth)
    if cpu is not None:
        rec["cpu_baseline"] = cpu
    if batch_in is not None:
        print("[bench] batched workload", file=sys.stderr, flush=True)
        rec["batch512"] = batch_leg(*batch_in, steps=1, warmup=1)
        del batch_in
        torch.cuda.empty_cache()
        print("[bench] asymptote-shifted workload", file=sys.stderr, flush=True)
        rec["aashrt"] = aashrt_leg(steps=3, warmup=1, autotune=not args.no_autotune)
        torch.cuda.empty_cache()
        print("[bench] separated-signal SNR study", file=sys.stderr, flush=True)
        rec["separation"] = separation_leg()
        print("[bench] learned warm start", file=sys.stderr, flush=True)
        rec["warmstart"] = warmstart_leg(ws_prep, label_outer=WS_DEFAULT["label_outer"],
                                         passes=WS_DEFAULT["passes"], ws_curves=WS_DEFAULT["curves"])
        print("[bench] warm-start U-Net training and inference", file=sys.stderr, flush=True)
        rec["unet"] = unet_leg(batch=4, steps=20, warmup=3)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
