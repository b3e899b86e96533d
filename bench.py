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
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak


# HBM bytes per launch of the row kernels on the production gather, by the
# plan's panel-chunk count (which sets their grid), from rocprofv3 --pmc
# FETCH_SIZE and --pmc WRITE_SIZE (KiB per dispatch) scaled by what the
# counters read for a 512 MiB device copy (reads x 2.0, writes x 1.0); valid
# only for the kernel sources with this digest.
_MIB = 1024.0 * 1024.0
MEASURED_TRAFFIC = {
    "digest": "58434cb17159bd17",
    "workload": "crg-1024x256-nv32",
    "bytes": {
        # nchunk -> read + write
        "k_rows_fwd": {1: (56.16 + 3.20) * _MIB, 2: (56.19 + 6.41) * _MIB, 4: (56.26 + 12.81) * _MIB,
                       8: (56.43 + 25.59) * _MIB},
        "k_rows_adj": {1: (2.28 + 55.92) * _MIB, 2: (4.31 + 55.92) * _MIB, 4: (8.37 + 55.92) * _MIB,
                       8: (16.53 + 55.92) * _MIB},
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


def _geometry_numbers(plan, nx, nt, P, R, cg_frac=0.0):
    """Algorithmic bytes and flops per launch of each kernel family.  cg_frac:
    the fraction of model-transform launches that also apply the previous CG
    iteration's update (read m, g; write m, pdir: four more model streams)."""
    import numpy as np
    info = plan.info
    ntp, nxp, jlo, jhi, nchunk = info["ntp"], info["nxp"], info["jlo"], info["jhi"], info["nchunk"]
    nrows = nxp // 2
    nband = jhi - jlo + 1
    f4, c8 = 4, 8
    model_b = P * nx * nt * f4
    data_b = nx * nt * f4
    # x-spectrum rows that can reach the band (c2 r^2 <= jhi^2, row 0 always):
    # the only ones written and read
    bin_ = ntp * plan.dt / (nxp * plan.dx)
    live_rows = 0
    for v in plan.vel:
        c2 = (v * bin_) ** 2
        rl = nrows if c2 <= 0 else min(nrows, 1 + sum(1 for r in range(1, nrows) if c2 * r * r <= jhi * jhi * (1 + 1e-9)))
        live_rows += rl
    X_b = live_rows * nt * c8
    H_b = nrows * nt * c8
    Dp_b = nchunk * nrows * 2 * nband * c8
    fft_t = 5.0 * ntp * math.log2(ntp)          # one complex time FFT
    fft_x = 5.0 * nxp * math.log2(nxp)          # one complex x FFT (two real columns)
    # in-cone map outputs: for each panel, row and band bin with j >= a (up and lo rows)
    vel = plan.vel
    j = np.arange(jlo, jhi + 1, dtype=np.float64)
    l = np.arange(nrows, dtype=np.float64)
    cone = 0
    for v in vel:
        a_up = v * bin_ * l
        a_lo = v * bin_ * np.where(l == 0, nrows, l)
        cone += int(np.sum(j[None, :] >= a_up[:, None])) + int(np.sum(j[None, :] >= a_lo[:, None]))
    # per in-cone output: one complex x real multiply-add per tap, plus ~40
    # flops to evaluate the bin's tap weights (the survey's per-unit figure)
    map_flops = cone * (2 * R * 4 + 40)
    return {
        "k_xfft_fwd(model)": (model_b + X_b + cg_frac * 4 * model_b, P * math.ceil(nt / 2) * fft_x),
        "k_xfft_fwd(data)": (data_b + H_b, math.ceil(nt / 2) * fft_x),
        "k_rows_fwd": (X_b + Dp_b, live_rows * fft_t + map_flops),
        "k_rows_fwd_fin": (Dp_b + H_b, nrows * fft_t),
        "k_xfft_inv(data)": (H_b + data_b, math.ceil(nt / 2) * fft_x),
        "k_rows_adj": (nchunk * H_b + X_b, (nchunk * nrows + live_rows) * fft_t + map_flops),
        "k_xfft_inv(model)": (X_b + model_b, P * math.ceil(nt / 2) * fft_x),
    }


def _q_db(clean, est):
    """Separation quality 10 log10(|clean|^2 / |clean - est|^2) (thesis
    Chapter 4, equations ch4_Qpd and ch4_Qr)."""
    import numpy as np
    c = np.asarray(clean, dtype=np.float64)
    e = np.asarray(est, dtype=np.float64)
    return float(10.0 * np.log10(np.sum(c * c) / np.sum((c - e) ** 2)))


def cpu_baseline(w, gth, budget_s=25.0):
    """The FP64 oracle on the host: a short solve of the same gather, scaled
    to a full solve by counting operator applications."""
    import numpy as np
    import oracle
    from oracle.irls import IrlsParams
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:  # pragma: no cover
        lim = None
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
    apps_full = 1 + w.n_outer * (2 * w.n_inner + 2)
    t_full = t_setup + t_sample * apps_full / apps_sample
    if lim is not None:
        lim.unregister() if hasattr(lim, "unregister") else None
    return {
        "value": 1.0 / t_full, "unit": "gathers/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 numpy/scipy oracle, one thread: stolt-map setup {t_setup:.2f} s plus a "
                   f"{n_outer}x{n_inner} IRLS-CG solve of the same gather ({apps_sample} operator "
                   f"applications, {t_sample:.2f} s), scaled to the {w.n_outer}x{w.n_inner} solve "
                   f"({apps_full} applications): {t_full:.1f} s per gather"),
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


def run_batch(args):
    """The batched workload: 512 receiver gathers of uneven size (nx in
    96..320, nt in {1024, 1536, 2048}, 24 velocities) solved together by
    robust_invert_batched (every stage one launch per FFT size class)."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    from synth import batch_shapes, workload
    w = workload(args.workload)
    n = args.batch_gathers
    shapes = batch_shapes(n, w.seed)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        gathers = list(ex.map(_gen_batch_gather, [(w.name, nt, nx, s) for nt, nx, s in shapes]))
    t_gen = time.perf_counter() - t0
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    descs = [dict(nt=nt, nx=nx, dt=w.dt, dx=w.dx, vel=list(w.vel), fmax=w.fmax, half_width=w.half_width)
             for nt, nx, _ in shapes]
    plan = A.BatchPlan(descs)
    d = plan.pack_data([g for g, _ in gathers])
    prm = A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)
    print(f"[bench] batch of {n} gathers: model {plan.model_total * 4 / 2**30:.1f} GiB, "
          f"data {plan.data_total * 4 / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    for _ in range(max(args.warmup, 0)):
        plan.robust_invert(d, prm, want_report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(args.steps):
        out = plan.robust_invert(d, prm, want_report=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, drec, _ = out
    q = []
    for gi, (g, clean) in enumerate(gathers):
        rec = plan.unpack_data(drec, gi).cpu().numpy()
        q.append((_q_db(clean, rec), _q_db(clean, g)))
    q = np.array(q)
    rec = {
        "metric": "robust ASHRT gathers solved/s (batched, IRLS-CG 10x20, l1 misfit)",
        "value": n * args.steps / wall, "unit": "gathers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "gathers": n, "npanel": w.npanel, "n_outer": w.n_outer,
                   "n_inner": w.n_inner, "nt_set": sorted(set(s[0] for s in shapes)),
                   "nx_range": [min(s[1] for s in shapes), max(s[1] for s in shapes)],
                   "model_gib": plan.model_total * 4 / 2**30, "reductions": "f64"},
        "snr": {"q_r_db_mean": float(q[:, 0].mean()), "q_pd_db_mean": float(q[:, 1].mean()),
                "improved": int((q[:, 0] > q[:, 1]).sum())},
        "seconds_generate": t_gen,
    }
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


def run_warmstart(args):
    """Learned warm start against the plain zero start on the same GPU: CG
    iterations and wall time to reach the plain method's final separated-
    signal SNR (minus 0.05 dB) on held-out gathers drawn like the
    production gather."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    base = "crg-1024x256-nv32"
    n_train, n_held = args.train_gathers, args.heldout_gathers
    t0 = time.perf_counter()
    # draw the gathers on host worker processes before the GPU is touched
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        train = [g for g, _ in ex.map(_gen_gather, [(base, 1_000_000 + i) for i in range(n_train)])]
        held = list(ex.map(_gen_gather, [(base, 2_000_000 + i) for i in range(n_held)]))
    t_gen = time.perf_counter() - t0
    import torch
    import paper_1711_10214_amd as A
    from paper_1711_10214_amd import warmstart as WS
    from synth import workload
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    w = workload(base)
    plan = A.Plan(w.nt, w.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    prm = A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner)
    print(f"[bench] warm start: labelling {n_train} gathers", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lab = WS.make_labels(plan, train, prm)
    torch.cuda.synchronize()
    t_lab = time.perf_counter() - t0
    net = A.UNet(w.npanel, base=16)
    net.init_params(seed=0)
    print(f"[bench] warm start: training {args.epochs} epochs", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    losses = WS.train(net, lab, epochs=args.epochs, batch=args.batch, tp=A.TrainParams(lr=1e-3), seed=0,
                      log_every=max(1, n_train // args.batch))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del lab
    # one warm-up of each path
    d0 = torch.tensor(held[0][0], device="cuda")
    WS.outer_to_target(plan, d0, held[0][1], 1e9, prm, max_outer=1)
    WS.outer_to_target(plan, d0, held[0][1], 1e9, prm, net=net, max_outer=1)
    rows = []
    for i, (g, clean) in enumerate(held):
        d = torch.tensor(g, device="cuda")
        _, d_rec, _ = plan.robust_invert(d, prm, want_report=False)
        target = WS.q_db(clean, d_rec.cpu().numpy())
        kp, qp, tp_, _ = WS.outer_to_target(plan, d, clean, target, prm)
        kw, qw, tw, start = WS.outer_to_target(plan, d, clean, target, prm, net=net)
        rows.append((target, kp, tp_, kw, tw, start, qw))
        if i % 16 == 0:
            print(f"[bench] held-out {i}: target {target:.2f} dB plain k={kp} warm k={kw} ({start})",
                  file=sys.stderr, flush=True)
    kp = np.array([r[1] or 99 for r in rows], float)
    kw = np.array([r[3] or 99 for r in rows], float)
    tp_ = np.array([r[2] for r in rows])
    tw = np.array([r[4] for r in rows])
    reached = sum(r[3] is not None for r in rows)
    rec = {
        "metric": "learned warm start: wall time to the plain IRLS-CG separated-signal SNR, plain / warm",
        "value": float(np.mean(tp_) / np.mean(tw)),
        "unit": "x (speed-up of time-to-SNR)",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "bf16 network, f32 solver",
        "data": "synthetic",
        "config": {"workload": "warmstart-crg-1024x256-nv32", "train_gathers": n_train,
                   "heldout_gathers": n_held, "epochs": args.epochs, "batch": args.batch,
                   "params": net.n_params, "n_outer": w.n_outer, "n_inner": w.n_inner},
        "plain": {"cg_iterations_mean": float(np.mean(kp) * w.n_inner), "outer_median": float(np.median(kp)),
                  "ms_mean": float(np.mean(tp_) * 1e3)},
        "warm": {"cg_iterations_mean": float(np.mean(kw) * w.n_inner), "outer_median": float(np.median(kw)),
                 "ms_mean": float(np.mean(tw) * 1e3), "reached_target": reached,
                 "model_start_rate": float(np.mean([r[5] == "model+weights" for r in rows]))},
        "seconds": {"generate": t_gen, "label": t_lab, "train": t_train},
        "train_loss": [losses[0], losses[-1]] if losses else None,
    }
    print(json.dumps(rec), flush=True)


BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix-core peak


def _unet_conv_flops(H, W, base=16, cin=1):
    """Algorithmic FLOPs of the U-Net's fourteen 3x3 convolutions for one
    sample at H x W (2 * 9 * ci * co per output pixel): forward, input
    gradient (every layer but the first, whose input is the data) and weight
    gradient.  Same layer list as the library's graph (four levels, two
    convolutions each, skip concatenations on the decoder side)."""
    c1, c2, c3, c4 = base, 2 * base, 4 * base, 8 * base
    spec = [(cin, c1, 0), (c1, c1, 0), (c1, c2, 1), (c2, c2, 1), (c2, c3, 2), (c3, c3, 2), (c3, c4, 3),
            (c4, c4, 3), (c4 + c3, c3, 2), (c3, c3, 2), (c3 + c2, c2, 1), (c2, c2, 1), (c2 + c1, c1, 0),
            (c1, c1, 0)]
    fwd = igrad = 0
    for i, (ci, co, lev) in enumerate(spec):
        f = 2 * 9 * ci * co * (H >> lev) * (W >> lev)
        fwd += f
        if i > 0:
            igrad += f
    return fwd, igrad, fwd


def run_unet(args):
    """Training steps (forward, backward, AdamW) and inference of the
    warm-start U-Net at the production gather's shape, against the dense BF16
    matrix-core peak."""
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda", 0)
    B, H, W, P = args.batch, 256, 1024, 32
    net = A.UNet(P, base=16)
    net.init_params(seed=0)
    g = torch.Generator(device="cpu").manual_seed(0)
    x = torch.randn((B, H, W), generator=g).to(dev)
    t_m = (0.1 * torch.randn((B, P, H, W), generator=g)).to(dev)
    t_w = torch.rand((B, H, W), generator=g).to(dev)
    tp = A.TrainParams(lr=1e-4)
    for _ in range(max(args.warmup, 1)):
        net.train_step(x, t_m, t_w, tp, want_loss=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        net.train_step(x, t_m, t_w, tp, want_loss=False)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_s = e0.elapsed_time(e1) / 1e3 / args.steps
    x1 = x[:1].contiguous()
    for _ in range(3):
        net.forward(x1)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        net.forward(x1)
    e1.record()
    torch.cuda.synchronize()
    inf_s = e0.elapsed_time(e1) / 1e3 / args.steps
    fwd, igrad, wgrad = _unet_conv_flops(H, W)
    step_flops = B * (fwd + igrad + wgrad)
    achieved = step_flops / step_s / 1e12
    rec = {
        "metric": "warm-start U-Net training steps/s (batch 4, 256 x 1024 gathers, 32 output panels)",
        "value": args.steps / wall, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak",
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
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="crg-1024x256-nv32")
    ap.add_argument("--pairs", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 512 MiB device copy (for HBM counter calibration)")
    ap.add_argument("--train-gathers", type=int, default=1024, help="warm-start workload: training gathers")
    ap.add_argument("--heldout-gathers", type=int, default=256, help="warm-start workload: held-out gathers")
    ap.add_argument("--epochs", type=int, default=12, help="warm-start workload: training epochs")
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

    import numpy as np
    import torch

    import paper_1711_10214_amd as A
    from paper_1711_10214_amd import _lib as L
    from synth import make_gather, workload

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda", 0)
    w = workload(args.workload)
    gth = make_gather(w)
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

    # warm-up, plus one fully profiled solve to find the dominant kernel
    for _ in range(max(args.warmup, 1)):
        solve()
    torch.cuda.synchronize()
    lib.ashrt_profile_enable((1 << L.K_COUNT) - 1)
    solve()
    torch.cuda.synchronize()
    lib.ashrt_profile_enable(0)
    per_kernel = {}
    import ctypes as C
    for k in range(L.K_COUNT):
        tot, n = C.c_double(), C.c_int64()
        L.check(lib.ashrt_profile_read(k, C.byref(tot), C.byref(n), 1), "ashrt_profile_read")
        per_kernel[lib.ashrt_kernel_name(k).decode()] = {"ms_total_per_solve": tot.value, "launches": n.value,
                                                        "kid": k}
    op_kernels = [k for k in per_kernel if k.startswith(("k_xfft", "k_rows"))]
    dom = max(op_kernels, key=lambda k: per_kernel[k]["ms_total_per_solve"])
    dom_kid = per_kernel[dom]["kid"]
    print(f"[bench] per-kernel ms per solve: " +
          ", ".join(f"{k}={v['ms_total_per_solve']:.2f}" for k, v in per_kernel.items()),
          file=sys.stderr, flush=True)

    # timed region: K solves; events around the dominant kernel's launches only
    lib.ashrt_profile_enable(1 << dom_kid)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    out = None
    for _ in range(args.steps):
        out = solve(graph=False)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lib.ashrt_profile_enable(0)
    tot, n = C.c_double(), C.c_int64()
    L.check(lib.ashrt_profile_read(dom_kid, C.byref(tot), C.byref(n), 1), "ashrt_profile_read")
    dom_avg_s = tot.value / max(n.value, 1) / 1e3
    ms_per_step = wall / args.steps * 1e3
    value = args.steps / wall

    # fixed-SNR check against the oracle's stored separation of this gather
    m_out, drec, _ = out
    q_r = _q_db(gth.d_clean, drec.cpu().numpy())
    q_pd = _q_db(gth.d_clean, gth.d_blend)
    snr = {"q_r_db": q_r, "q_pd_db": q_pd}
    gold = os.path.join(ROOT, "tests", "golden", "oracle_separation.json")
    if os.path.exists(gold):
        ref = json.load(open(gold)).get(w.name)
        if ref and ref["n_outer"] == w.n_outer and ref["n_inner"] == w.n_inner:
            snr["oracle_q_r_db"] = ref["q_r_db"]
            snr["reached"] = bool(q_r >= ref["q_r_db"] - 0.05)

    # the same solves with the CG iterations replayed from a hipGraph (no
    # per-kernel events, which keep the timed region above on plain launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solve(graph=True)
    torch.cuda.synchronize()
    graph_wall = time.perf_counter() - t0

    # operator pairs per second
    rng = np.random.default_rng(0)
    mm = torch.tensor(rng.standard_normal((w.npanel, gth.nx, gth.nt)), dtype=torch.float32, device=dev)
    dd = torch.empty((gth.nx, gth.nt), dtype=torch.float32, device=dev)
    m2 = torch.empty_like(mm)
    for _ in range(3):
        plan.forward(mm, out=dd)
        plan.adjoint(dd, out=m2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.pairs):
        plan.forward(mm, out=dd)
        plan.adjoint(dd, out=m2)
    torch.cuda.synchronize()
    pair_s = (time.perf_counter() - t0) / args.pairs

    # roofline of the dominant kernel
    # in the solve, the model transforms of CG iterations 1 .. n_inner-1 carry
    # the fused update; iteration 0 and the residual forward of each outer
    # step do not
    nums = _geometry_numbers(plan, gth.nx, gth.nt, w.npanel, w.half_width,
                             cg_frac=(w.n_inner - 1) / (w.n_inner + 1) if w.n_inner > 0 else 0.0)
    bytes_, flops = nums[dom]
    hbm_frac = (bytes_ / dom_avg_s / 1e9) / HBM_PEAK_GBS
    alu_frac = (flops / dom_avg_s / 1e12) / FP32_VECTOR_PEAK_TFLOPS
    if hbm_frac >= alu_frac:
        roof = {"bound": "hbm", "achieved": bytes_ / dom_avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": flops / dom_avg_s / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = _measured_traffic(w.name, dom, plan.info["nchunk"])
    roof["kernel"] = dom
    roof["avg_launch_us"] = dom_avg_s * 1e6
    roof["launches_timed"] = n.value
    roof["algorithmic_bytes_per_launch"] = bytes_
    roof["algorithmic_flops_per_launch"] = flops
    roof["hbm_frac"] = hbm_frac
    roof["alu_frac"] = alu_frac
    pair_bytes = sum(v[0] for v in _geometry_numbers(plan, gth.nx, gth.nt, w.npanel, w.half_width).values())
    if args.copy_calibration:
        x = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device=dev)
        x.fill_(1.0)
        y = x.clone()
        torch.cuda.synchronize()
        del x, y

    rec = {
        "metric": "robust ASHRT gathers solved/s to fixed SNR (IRLS-CG 10x20, l1 misfit); also fwd+adj pairs/s, HBM GB/s",
        "value": value,
        "unit": "gathers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nt": gth.nt, "nx": gth.nx, "ntp": plan.info["ntp"],
                   "tiling": {"tile_model": plan.info["tile_model"], "tile_data": plan.info["tile_data"],
                              "nchunk": plan.info["nchunk"]},
                   "nxp": plan.info["nxp"], "npanel": w.npanel, "p": w.p, "q": w.q,
                   "n_outer": w.n_outer, "n_inner": w.n_inner, "fmax_hz": w.fmax,
                   "reductions": "f64", "seed": w.seed},
        "graph_gathers_per_s": args.steps / graph_wall,
        "pairs_per_s": 1.0 / pair_s,
        "pair_ms": pair_s * 1e3,
        "pair_algorithmic_gbs": pair_bytes / pair_s / 1e9,
        "snr": snr,
        "kernels_ms_per_solve": {k: round(v["ms_total_per_solve"], 4) for k, v in per_kernel.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host (bounded sample)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w, gth)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
