"""GPU parity of the Stolt (A)ASHRT forward and adjoint against the FP64 oracle.

Bar: relative L2 <= 1e-5 per application (FP32 FFTs and map, FP64 map
coordinates).  The GPU dot-product test checks the exact-transpose pairing
at FP32 level.  Every call goes through the C ABI via the ctypes binding.
"""
import zlib

import numpy as np
import pytest

import oracle
from tests.gpu_common import f32, geom_kwargs, oracle_geometry, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def A():
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return A


def _run_pair(A, kw, seed, mask_frac=0.0):
    import torch
    rng = np.random.default_rng(seed)
    g = oracle_geometry(kw)
    m = f32(rng.standard_normal((g.npanel, g.nx, g.nt)))
    d = f32(rng.standard_normal((g.nx, g.nt)))
    mask = None
    if mask_frac > 0:
        mask = (rng.uniform(size=g.nx) >= mask_frac).astype(np.uint8)
    plan = A.Plan(**kw)
    assert (plan.info["ntp"], plan.info["nxp"]) == (g.ntp, g.nxp)
    assert (plan.info["jlo"], plan.info["jhi"]) == oracle.band(g)
    mt = torch.tensor(m, dtype=torch.float32, device="cuda")
    dt_ = torch.tensor(d, dtype=torch.float32, device="cuda")
    mk = None if mask is None else torch.tensor(mask, device="cuda")
    d_gpu = plan.forward(mt, mask=mk).cpu().numpy()
    m_gpu = plan.adjoint(dt_, mask=mk).cpu().numpy()
    d_ref = oracle.forward(g, m, mask)
    m_ref = oracle.adjoint(g, d, mask)
    return g, m, d, d_gpu, m_gpu, d_ref, m_ref


CASES = {
    # name: (kwargs, mask fraction)
    "crg-256x64-nv8": (geom_kwargs(256, 64, 0.004, 12.5, list(np.linspace(1500, 3000, 8)), fmax=100.0), 0.0),
    "ragged-odd-nt": (geom_kwargs(203, 37, 0.004, 12.5, [1400.0, 2200.0, 3900.0], fmax=90.0), 0.0),
    "radix3-both": (geom_kwargs(190, 90, 0.004, 12.5, [1600.0, 2500.0], ntp=384, nxp=192, fmax=120.0), 0.0),
    "full-band-no-pad": (geom_kwargs(128, 32, 0.002, 10.0, [0.0, 1800.0, 5000.0], ntp=128, nxp=32), 0.0),
    "aashrt-ramp-scale-mask": (geom_kwargs(256, 48, 0.004, 12.5, [1500.0, 1500.0, 2400.0, 2400.0],
                                           tau0=[0, 7, 0, 23], scale=[1.0, 0.5, 2.0, 1.5],
                                           fmin=5.0, fmax=80.0), 0.3),
    "half-width-2": (geom_kwargs(160, 40, 0.004, 12.5, [1500.0, 2600.0], fmax=100.0, half_width=2), 0.0),
    "irregular-jittered": (geom_kwargs(256, 48, 0.004, 12.5, [1500.0, 2200.0, 3100.0], fmax=100.0,
                                       xpos=list(np.arange(48) * 12.5 + np.random.default_rng(8).uniform(-5, 5, 48))),
                           0.2),
    "irregular-aashrt-random": (geom_kwargs(200, 40, 0.004, 10.0, [1700.0, 1700.0, 2600.0], tau0=[0, 9, 0],
                                            fmax=90.0,
                                            xpos=list(np.sort(np.random.default_rng(9).uniform(0, 390.0, 40)))),
                                0.0),
    "half-width-8": (geom_kwargs(160, 40, 0.004, 12.5, [1500.0, 2600.0], fmax=100.0, half_width=8), 0.0),
    "tiny": (geom_kwargs(2, 2, 0.004, 12.5, [2000.0], ntp=8, nxp=4), 0.0),
    # long traces: the 3072- and 4096-point row kernels (512-thread workgroups)
    # widest x transforms the plans take (nxp 4096, and 3072 = 3 * 2^10)
    "wide-nxp4096": (geom_kwargs(48, 2048, 0.004, 12.5, [1500.0, 3000.0], fmax=100.0), 0.0),
    "wide-nxp3072-mask": (geom_kwargs(40, 1500, 0.004, 12.5, [1800.0, 2900.0, 4200.0], fmax=100.0, nxp=3072), 0.15),
    "long-ntp3072": (geom_kwargs(1536, 16, 0.004, 12.5, [1500.0, 2600.0, 3800.0], fmax=110.0), 0.0),
    "long-ntp4096-ragged-mask": (geom_kwargs(1900, 10, 0.004, 12.5, [1500.0, 2600.0, 3800.0], tau0=[0, 11, 3],
                                             fmax=110.0), 0.2),
    # the remaining compile-time lengths: x 256 / time 768, x 384 / time 1024,
    # x 768 / time 1536 (the batched workload's widest gathers use x 768) and x 1024
    "x256-t768": (geom_kwargs(300, 100, 0.004, 12.5, [1500.0, 2300.0, 3600.0], fmax=100.0), 0.0),
    "x384-t1024-ramp": (geom_kwargs(450, 150, 0.004, 12.5, [1400.0, 1400.0, 2900.0], tau0=[0, 13, 0],
                                    fmax=100.0), 0.0),
    "x768-t1536-mask": (geom_kwargs(700, 300, 0.004, 12.5, [1600.0, 2500.0, 3900.0], fmax=100.0), 0.2),
    "x1024-t512": (geom_kwargs(200, 500, 0.004, 12.5, [1500.0, 2600.0], fmax=100.0), 0.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_forward_adjoint_match_oracle(A, name):
    kw, mf = CASES[name]
    print(f"[gpu] operator parity case={name}", flush=True)
    g, m, d, d_gpu, m_gpu, d_ref, m_ref = _run_pair(A, kw, seed=zlib.crc32(name.encode()) % 1000, mask_frac=mf)
    assert np.all(np.isfinite(d_gpu)) and np.all(np.isfinite(m_gpu))
    ef, ea = rel_l2(d_gpu, d_ref), rel_l2(m_gpu, m_ref)
    print(f"  rel-L2 forward {ef:.2e} adjoint {ea:.2e}", flush=True)
    assert ef <= TOL, ef
    assert ea <= TOL, ea


def test_wavelet_weight(A):
    kw = geom_kwargs(200, 40, 0.004, 12.5, [1500.0, 2500.0], fmax=100.0)
    H = oracle.fft_len(200) // 2 + 1
    kw["wavelet"] = np.exp(-((np.arange(H) - 60.0) / 40.0) ** 2)
    print("[gpu] operator parity case=wavelet", flush=True)
    _, _, _, d_gpu, m_gpu, d_ref, m_ref = _run_pair(A, kw, seed=5)
    assert rel_l2(d_gpu, d_ref) <= TOL
    assert rel_l2(m_gpu, m_ref) <= TOL


@pytest.mark.parametrize("name", ["crg-256x64-nv8", "aashrt-ramp-scale-mask", "radix3-both"])
def test_dot_product_fp32(A, name):
    kw, mf = CASES[name]
    print(f"[gpu] dot test case={name}", flush=True)
    g, m, d, d_gpu, m_gpu, _, _ = _run_pair(A, kw, seed=11, mask_frac=mf)
    lhs = float(np.sum(d_gpu.astype(np.float64) * d))
    rhs = float(np.sum(m * m_gpu.astype(np.float64)))
    rel = abs(lhs - rhs) / (np.linalg.norm(d_gpu) * np.linalg.norm(d))
    print(f"  dot rel {rel:.2e}", flush=True)
    assert rel < 1e-6


def test_production_size_sampled(A):
    """Production geometry (1024 x 256, 32 velocities): full forward/adjoint
    parity against the oracle (the oracle runs it in a few seconds)."""
    kw = geom_kwargs(1024, 256, 0.004, 12.5, list(np.linspace(1400, 4000, 32)), fmax=100.0)
    print("[gpu] operator parity case=crg-1024x256-nv32", flush=True)
    _, _, _, d_gpu, m_gpu, d_ref, m_ref = _run_pair(A, kw, seed=2)
    ef, ea = rel_l2(d_gpu, d_ref), rel_l2(m_gpu, m_ref)
    print(f"  rel-L2 forward {ef:.2e} adjoint {ea:.2e}", flush=True)
    assert ef <= TOL and ea <= TOL


def test_linearity_and_zero(A):
    import torch
    kw = geom_kwargs(128, 32, 0.004, 12.5, [1500.0, 2500.0], fmax=100.0)
    plan = A.Plan(**kw)
    z = torch.zeros((2, 32, 128), device="cuda")
    assert float(plan.forward(z).abs().max()) == 0.0
    rng = np.random.default_rng(3)
    a = torch.tensor(rng.standard_normal((2, 32, 128)), dtype=torch.float32, device="cuda")
    b = torch.tensor(rng.standard_normal((2, 32, 128)), dtype=torch.float32, device="cuda")
    lhs = plan.forward(a + 2 * b).cpu().numpy()
    rhs = (plan.forward(a) + 2 * plan.forward(b)).cpu().numpy()
    assert rel_l2(lhs, rhs) < 1e-6


def test_full_size_operators_match_stored_oracle_samples(A):
    """Full-size workloads: the asymptote-shifted gather (1024 x 256, 24
    velocities x 16 asymptote shifts = 384 panels, half the traces
    decimated), the production gather (1024 x 256, 32 velocities) and the
    batched workload's gather 31 (2048 x 318, 24 velocities): forward and
    adjoint of seeded Gaussian inputs against the FP64 oracle's outputs
    stored by tests/golden/make_oracle_values.py --operator (norms and 512
    sampled values each; the oracle needs tens of seconds per pair, too slow
    to run inside the test)."""
    import json
    import os
    import torch
    from synth import make_gather, random_data, random_model, workload
    from synth import make_cfg3_batch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_operator_samples.json")))
    # "batch512-crg-nv24:g31": gather 31 of the 512-gather workload, nt 2048 x
    # nx 318 with 24 velocities (time FFT 4096, x FFT 768)
    for name in ("aashrt-1024x256-nv24x16", "crg-1024x256-nv32", "batch512-crg-nv24:g31"):
        ref = gold[name]
        base, _, gi = name.partition(":g")
        w = workload(base)
        gth = make_cfg3_batch(w, 1, int(gi))[0] if gi else make_gather(w)
        print(f"[gpu] full-size operator vs stored oracle samples case={name}", flush=True)
        plan = A.Plan(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), tau0=list(w.tau0), fmax=w.fmax,
                      half_width=w.half_width)
        mask = torch.tensor(gth.mask, device="cuda") if w.decimate_frac > 0 else None
        rng = np.random.default_rng(ref["input_seed"])
        m = random_model(rng, w.npanel, gth.nx, gth.nt, np.float32)
        d = random_data(rng, gth.nx, gth.nt, np.float32)
        # FP64 copies: a norm over 1e8 values needs an FP64 accumulator
        fwd = plan.forward(torch.tensor(m, device="cuda"), mask=mask).cpu().numpy().ravel().astype(np.float64)
        adj = plan.adjoint(torch.tensor(d, device="cuda"), mask=mask).cpu().numpy().ravel().astype(np.float64)
        for out, key in ((fwd, "forward"), (adj, "adjoint")):
            e_norm = abs(np.linalg.norm(out) / ref[f"{key}_norm"] - 1.0)
            idx = np.asarray(ref[f"{key}_index"])
            sv = np.asarray(ref[f"{key}_value"])
            e_s = rel_l2(out[idx], sv)
            print(f"  {key}: norm rel err {e_norm:.2e}, sampled rel-L2 {e_s:.2e}", flush=True)
            assert e_norm <= TOL
            # 512 samples estimate the whole-output relative L2 error
            assert e_s <= 3 * TOL


def test_tuned_tilings_give_the_same_operator(A):
    """Every tiling the autotuner may choose computes the same operator (only
    the panel-chunk partial sums change the FP32 summation order)."""
    import torch
    kw = geom_kwargs(203, 37, 0.004, 12.5, [1400.0, 2200.0, 3900.0, 2600.0, 1800.0], fmax=90.0)
    rng = np.random.default_rng(41)
    m = torch.tensor(rng.standard_normal((5, 37, 203)), dtype=torch.float32, device="cuda")
    d = torch.tensor(rng.standard_normal((37, 203)), dtype=torch.float32, device="cuda")
    base = A.Plan(**kw)
    f0, a0 = base.forward(m).cpu().numpy(), base.adjoint(d).cpu().numpy()
    for tm, td, ch in [(8, 2, 1), (32, 8, 5), (16, 4, 2), (64, 2, 8)]:
        plan = A.Plan(**kw, tuning={"tile_model": tm, "tile_data": td, "nchunk": ch})
        assert (plan.info["tile_model"], plan.info["tile_data"]) == (tm, td)
        assert plan.info["nchunk"] == min(ch, 5)
        ef = rel_l2(plan.forward(m).cpu().numpy(), f0)
        ea = rel_l2(plan.adjoint(d).cpu().numpy(), a0)
        print(f"[gpu] tiling {tm}/{td}/{ch}: forward {ef:.1e} adjoint {ea:.1e}", flush=True)
        assert ef <= 1e-6 and ea <= 1e-6
    with pytest.raises(A.AshrtError):
        A.Plan(**kw, tuning={"tile_model": 7})


def test_autotune_is_cached_and_usable(A):
    kw = geom_kwargs(256, 64, 0.004, 12.5, list(np.linspace(1500, 3000, 8)), fmax=100.0)
    t1 = A.autotune(**kw)
    t2 = A.autotune(**kw)
    print(f"[gpu] autotune crg-256x64-nv8: {t1}", flush=True)
    assert t1 == t2
    assert t1["tile_model"] in (8, 16, 32) and t1["tile_data"] in (2, 4, 8) and 1 <= t1["nchunk"] <= 8
    plan = A.Plan(**kw, tuning="auto")
    assert plan.info["tile_model"] == t1["tile_model"] and plan.info["nchunk"] == t1["nchunk"]


def test_autotune_file_cache(A, tmp_path, monkeypatch):
    """With ASHRT_TUNE_CACHE set, a tuned tiling is appended to the file under
    the device's architecture name, and an entry already in the file is
    returned without timing (here one written by hand for a geometry this
    process has not tuned)."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("ASHRT_TUNE_CACHE", str(path))
    kw = geom_kwargs(192, 40, 0.004, 12.5, [1600.0, 2500.0, 3100.0], fmax=100.0)
    t1 = A.autotune(**kw)
    lines = path.read_text().splitlines()
    print(f"[gpu] autotune file cache: {lines}", flush=True)
    assert len(lines) == 1
    key, tm, td, ch, ms = lines[0].split()
    arch = key.split("|")[0]
    assert arch.startswith("gfx")
    assert (int(tm), int(td), int(ch)) == (t1["tile_model"], t1["tile_data"], t1["nchunk"])
    # a geometry not tuned yet in this process, with a made-up entry
    kw2 = geom_kwargs(176, 40, 0.004, 12.5, [1600.0, 2500.0, 3100.0], fmax=100.0)
    g = oracle_geometry(kw2)
    jlo, jhi = oracle.band(g)
    fake = f"{arch}|{176},{40},{g.ntp},{g.nxp},{3},{4},{jlo},{jhi},0 32 8 2 9.5"
    with open(path, "a") as f:
        f.write(fake + "\n")
    t2 = A.autotune(**kw2)
    assert (t2["tile_model"], t2["tile_data"], t2["nchunk"]) == (32, 8, 2)
