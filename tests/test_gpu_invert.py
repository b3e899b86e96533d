"""GPU parity of the robust IRLS-CG inversion against the FP64 oracle.

Same seeded blended gather on both sides (FP32-rounded input).  Bar: relative
L2 <= 1e-4 on the separated gather d_rec = L m after the whole solve, and the
per-outer-iteration misfit / clip within 1e-4 relative.  Every call goes
through the C ABI (robust_invert) via the ctypes binding.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.irls import IrlsParams
from synth import make_gather, workload
from tests.gpu_common import f32, geom_kwargs, oracle_geometry, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available()
    return A


def _solve_both(A, kw, d, prm: IrlsParams, mask=None, w0=None):
    import torch
    g = oracle_geometry(kw)
    plan = A.Plan(**kw)
    dt_ = torch.tensor(d, dtype=torch.float32, device="cuda")
    mk = None if mask is None else torch.tensor(mask, device="cuda")
    w0t = None if w0 is None else torch.tensor(w0, dtype=torch.float32, device="cuda")
    P = A.Params(p=prm.p, q=prm.q, n_outer=prm.n_outer, n_inner=prm.n_inner, b_r=prm.b_r,
                 b_m=prm.b_m, tol=prm.tol, eps_floor_rel=prm.eps_floor_rel, freeze_eps=prm.freeze_eps)
    m_gpu, drec_gpu, rep = plan.robust_invert(dt_, P, mask=mk, w0=w0t)
    m_ref, drec_ref, rep_ref = oracle.robust_invert(g, d, prm, mask=mask, w0=w0)
    return m_gpu.cpu().numpy(), drec_gpu.cpu().numpy(), rep, m_ref, drec_ref, rep_ref


def _cfg1(nt=None, nx=None):
    w = workload("crg-256x64-nv8")
    gth = make_gather(w)
    kw = geom_kwargs(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    return w, gth, kw


@pytest.mark.parametrize("pq", [(1, 2), (2, 2), (1, 1), (2, 1)])
def test_small_crg_solve_matches_oracle(A, pq):
    p, q = pq
    w, gth, kw = _cfg1()
    prm = IrlsParams(p=p, q=q, n_outer=w.n_outer, n_inner=w.n_inner)
    print(f"[gpu] invert parity crg-256x64-nv8 p={p} q={q}", flush=True)
    m_g, d_g, rep, m_r, d_r, rep_r = _solve_both(A, kw, f32(gth.d_blend), prm)
    e_d = rel_l2(d_g, d_r)
    e_m = rel_l2(m_g, m_r)
    print(f"  d_rec rel-L2 {e_d:.2e}  m rel-L2 {e_m:.2e}", flush=True)
    print(f"  misfit gpu {rep['misfit']}\n  misfit ref {rep_r['misfit']}", flush=True)
    assert rep["outer_done"] == rep_r["outer_done"]
    assert rep["inner"] == rep_r["inner"]
    assert e_d <= 1e-4
    np.testing.assert_allclose(rep["misfit"], rep_r["misfit"], rtol=1e-4)
    # eps_r is an order statistic (median of |r - median r|): its error is the
    # absolute FP32 error of one residual sample over the MAD, and that error
    # scales with the residual's largest (interference) amplitudes, not with
    # the MAD -- hence a looser bound than the 1e-4 on the separated gather.
    np.testing.assert_allclose(rep["eps_r"], rep_r["eps_r"], rtol=1e-3, atol=1e-12)
    np.testing.assert_allclose(rep["huber"], rep_r["huber"], rtol=1e-4)
    if q == 1:
        np.testing.assert_allclose(rep["eps_m"][1:], rep_r["eps_m"], rtol=1e-4)


@pytest.mark.parametrize("nt_nx_inner", [(203, 37, 5), (250, 40, 4), (256, 64, 1), (256, 64, 2)])
def test_solve_edge_shapes_match_oracle(A, nt_nx_inner):
    """Odd nt (the element-pair tails of the fused CG update), even nt with a
    ragged last model tile (250 = 3 x 64 + 58: full tiles take the batched
    loads, the last one the per-element path) and one or two CG iterations
    per outer step (no fused update / one, no graph), q = 1."""
    nt, nx, n_inner = nt_nx_inner
    w = workload("crg-256x64-nv8", nt=nt, nx=nx)
    gth = make_gather(w)
    kw = geom_kwargs(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    prm = IrlsParams(p=1, q=1, n_outer=3, n_inner=n_inner)
    print(f"[gpu] invert parity nt={nt} nx={nx} n_inner={n_inner}", flush=True)
    m_g, d_g, rep, m_r, d_r, rep_r = _solve_both(A, kw, f32(gth.d_blend), prm)
    e_d = rel_l2(d_g, d_r)
    print(f"  d_rec rel-L2 {e_d:.2e}", flush=True)
    assert rep["inner"] == rep_r["inner"]
    assert e_d <= 1e-4
    np.testing.assert_allclose(rep["misfit"], rep_r["misfit"], rtol=1e-4)


def test_long_trace_solve_matches_oracle(A):
    """1536-sample traces (3072-point time FFTs, 512-thread row workgroups)
    through the fused CG iterations."""
    w = workload("crg-256x64-nv8", nt=1536, nx=24, vel=(1500.0, 2200.0, 3300.0))
    gth = make_gather(w)
    kw = geom_kwargs(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    prm = IrlsParams(p=1, q=2, n_outer=2, n_inner=5)
    print("[gpu] invert parity long traces nt=1536", flush=True)
    m_g, d_g, rep, m_r, d_r, rep_r = _solve_both(A, kw, f32(gth.d_blend), prm)
    e_d = rel_l2(d_g, d_r)
    print(f"  d_rec rel-L2 {e_d:.2e}", flush=True)
    assert e_d <= 1e-4
    np.testing.assert_allclose(rep["misfit"], rep_r["misfit"], rtol=1e-4)


def test_separation_quality_matches_oracle(A):
    w, gth, kw = _cfg1()
    prm = IrlsParams(p=1, q=2, n_outer=w.n_outer, n_inner=w.n_inner)
    m_g, d_g, rep, m_r, d_r, rep_r = _solve_both(A, kw, f32(gth.d_blend), prm)
    q_gpu = oracle.q_db(gth.d_clean, d_g)
    q_ref = oracle.q_db(gth.d_clean, d_r)
    q_pd = oracle.q_db(gth.d_clean, gth.d_blend)
    print(f"[gpu] Q_PD {q_pd:.3f} dB  Q_R gpu {q_gpu:.4f}  oracle {q_ref:.4f}", flush=True)
    assert q_gpu >= q_ref - 0.05
    assert q_gpu > q_pd


def test_decimated_aashrt_interpolation(A):
    """Masked (decimated) gather with asymptote-shifted panels, p = 2, q = 1."""
    w = workload("aashrt-1024x256-nv24x16", nt=200, nx=48, vel=(1600.0, 1600.0, 2600.0, 2600.0),
                 tau0=(0, 10, 0, 10), n_diffractors=4, n_events=(2, 2), tau_range=(0.1, 0.5))
    gth = make_gather(w)
    kw = geom_kwargs(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), tau0=list(w.tau0), fmax=w.fmax)
    prm = IrlsParams(p=2, q=1, n_outer=4, n_inner=8)
    print("[gpu] invert parity aashrt decimated", flush=True)
    m_g, d_g, rep, m_r, d_r, rep_r = _solve_both(A, kw, f32(gth.d_blend), prm, mask=gth.mask)
    e_d = rel_l2(d_g, d_r)
    print(f"  d_rec rel-L2 {e_d:.2e}", flush=True)
    assert e_d <= 1e-4
    np.testing.assert_allclose(rep["misfit"], rep_r["misfit"], rtol=1e-4)


def test_warm_start_weights_and_frozen_clip(A):
    w, gth, kw = _cfg1()
    rng = np.random.default_rng(9)
    w0 = f32(rng.uniform(0.2, 1.0, gth.d_blend.shape))
    prm = IrlsParams(p=1, q=2, n_outer=4, n_inner=6, freeze_eps=True)
    m_g, d_g, rep, m_r, d_r, rep_r = _solve_both(A, kw, f32(gth.d_blend), prm, w0=w0)
    assert rel_l2(d_g, d_r) <= 1e-4
    assert len(set(np.round(rep["eps_r"], 12))) == 1
    h = rep["huber"]
    assert all(b <= a * (1 + 1e-5) for a, b in zip(h, h[1:]))


def test_tolerance_early_stop(A):
    w, gth, kw = _cfg1()
    prm = IrlsParams(p=1, q=2, n_outer=30, n_inner=10, tol=0.01)
    m_g, d_g, rep, m_r, d_r, rep_r = _solve_both(A, kw, f32(gth.d_blend), prm)
    assert rep["outer_done"] == rep_r["outer_done"] < 30


def test_zero_data_is_finite(A):
    import torch
    w, gth, kw = _cfg1()
    plan = A.Plan(**kw)
    d = torch.zeros((gth.nx, gth.nt), device="cuda")
    m, drec, rep = plan.robust_invert(d, A.Params(n_outer=2, n_inner=3))
    assert float(m.abs().max()) == 0.0
    assert rep["inner"] == [0, 0]
    assert all(np.isfinite(rep["misfit"]))


def test_production_solve_matches_stored_oracle(A):
    """Full 10 x 20 solve of the production gather (1024 x 256, 32 velocities)
    against the FP64 oracle's solve stored by tests/golden/make_oracle_values.py
    (which calls only the oracle): the separated gather element-wise, the
    model, Q_R, and the per-iteration misfits and clips."""
    import torch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_separation.json")))
    ref = gold["crg-1024x256-nv32"]
    w = workload("crg-1024x256-nv32")
    gth = make_gather(w)
    plan = A.Plan(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    d = torch.tensor(gth.d_blend, dtype=torch.float32, device="cuda")
    print("[gpu] invert parity crg-1024x256-nv32 10x20 vs stored oracle", flush=True)
    m, drec, rep = plan.robust_invert(d, A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner))
    _check_stored_solve(gth, ref, m, drec, rep)


def _check_stored_solve(gth, ref, m, drec, rep):
    """The separated gather against the stored oracle solve, element-wise:
    4096 seeded sample values (their relative L2 error estimates the whole
    gather's), the norm and the 256 per-trace norms, each <= 1e-4; Q_R within
    1e-4 dB; misfits per outer iteration within 1e-4."""
    out = drec.cpu().numpy().astype(np.float64)
    mm = m.cpu().numpy().astype(np.float64)
    q_r = oracle.q_db(gth.d_clean, out)
    idx = np.asarray(ref["drec_index"])
    e_s = rel_l2(out.ravel()[idx], np.asarray(ref["drec_value"]))
    e_n = abs(np.linalg.norm(out) / ref["drec_norm"] - 1.0)
    e_t = rel_l2(np.linalg.norm(out, axis=1), np.asarray(ref["drec_trace_norm"]))
    e_m = rel_l2(mm.ravel()[np.asarray(ref["m_index"])], np.asarray(ref["m_value"]))
    e_mn = abs(np.linalg.norm(mm) / ref["m_norm"] - 1.0)
    e_mis = np.max(np.abs(np.array(rep["misfit"]) / np.array(ref["misfit"]) - 1))
    print(f"  d_rec: sampled rel-L2 {e_s:.2e}, norm {e_n:.2e}, trace norms {e_t:.2e}", flush=True)
    print(f"  m: sampled rel-L2 {e_m:.2e}, norm {e_mn:.2e}", flush=True)
    print(f"  Q_R gpu {q_r:.7f} dB oracle {ref['q_r_db']:.7f} dB (diff {q_r - ref['q_r_db']:.1e}); "
          f"misfit rel err {e_mis:.2e}", flush=True)
    assert e_s <= 1e-4 and e_n <= 1e-4 and e_t <= 1e-4
    assert abs(q_r - ref["q_r_db"]) < 1e-4
    np.testing.assert_allclose(rep["misfit"], ref["misfit"], rtol=1e-4)
    # the clips are order statistics (eps_r, a median) and an extreme value
    # (eps_m, a maximum) of FP32 vectors: each moves by at most a few times
    # the largest single-sample error, which is set by the largest amplitudes
    # rather than by the clip, so their bound is 1e-3
    if ref["p"] == 1:
        e_r = np.max(np.abs(np.array(rep["eps_r"]) / np.array(ref["eps_r"]) - 1))
        print(f"  eps_r max rel err {e_r:.2e}", flush=True)
        assert e_r <= 1e-3
    if ref["q"] == 1:
        e_q = np.max(np.abs(np.array(rep["eps_m"][1:]) / np.array(ref["eps_m"]) - 1))
        print(f"  eps_m max rel err {e_q:.2e}", flush=True)
        assert e_q <= 1e-3


def test_aashrt_production_solve_matches_stored_oracle(A):
    """Full 10 x 20 solve of the decimated diffraction gather (1024 x 256,
    24 velocities x 16 asymptote shifts = 384 panels, half the traces
    missing, p = 2, q = 1) against the FP64 oracle's solve stored by
    tests/golden/make_oracle_values.py (which calls only the oracle):
    the reconstructed gather and the model element-wise at seeded samples,
    per-trace norms, SNR, per-iteration misfits and model clips."""
    import torch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_separation.json")))
    ref = gold["aashrt-1024x256-nv24x16"]
    w = workload("aashrt-1024x256-nv24x16")
    gth = make_gather(w)
    assert (ref["p"], ref["q"], ref["n_outer"], ref["n_inner"]) == (w.p, w.q, w.n_outer, w.n_inner)
    plan = A.Plan(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), tau0=list(w.tau0), fmax=w.fmax)
    d = torch.tensor(gth.d_blend, dtype=torch.float32, device="cuda")
    mask = torch.tensor(gth.mask, device="cuda")
    print("[gpu] invert parity aashrt-1024x256-nv24x16 10x20 vs stored oracle", flush=True)
    m, drec, rep = plan.robust_invert(d, A.Params(p=w.p, q=w.q, n_outer=w.n_outer, n_inner=w.n_inner), mask=mask)
    _check_stored_solve(gth, ref, m, drec, rep)


@pytest.mark.parametrize("pq_inner", [(1, 2, 7), (1, 1, 6)])
def test_cg_graph_replays_match_eager_launches(A, pq_inner):
    """CG iterations replayed from the captured hipGraph give bit-identical
    results to launching them one by one: two solves in a row on different
    data (the cached graph replays against new contents, with the solver's
    eager work between replays), odd and even CG counts."""
    import torch
    p, q, n_inner = pq_inner
    w, gth, kw = _cfg1()
    plan = A.Plan(**kw)
    rng = np.random.default_rng(31)
    d1 = torch.tensor(f32(gth.d_blend), dtype=torch.float32, device="cuda")
    d2 = (0.5 * d1 + torch.tensor(rng.standard_normal(d1.shape) * 0.05, dtype=torch.float32, device="cuda"))
    print(f"[gpu] cg graph vs eager p={p} q={q} n_inner={n_inner}", flush=True)
    for d in (d1, d2, d1):
        res = {}
        for graph in (False, True):
            prm = A.Params(p=p, q=q, n_outer=3, n_inner=n_inner, cg_graph=graph)
            res[graph] = plan.robust_invert(d, prm)
        (m_e, dr_e, rep_e), (m_g, dr_g, rep_g) = res[False], res[True]
        assert torch.equal(m_e, m_g)
        assert torch.equal(dr_e, dr_g)
        assert rep_e["misfit"] == rep_g["misfit"]
        assert rep_e["inner"] == rep_g["inner"]


@pytest.mark.parametrize("pq_missing", [(1, 2, 0.0), (2, 1, 0.4)])
def test_irregular_traces_solve_matches_oracle(A, pq_missing):
    """Robust solve on a gather whose traces sit at jittered positions (the
    data-side x transforms are non-uniform DFTs); the second case also drops
    40 % of the traces and weights the model (interpolation of irregular,
    incomplete data)."""
    p, q, missing = pq_missing
    w, gth, kw = _cfg1()
    kw = dict(kw, xpos=list(np.arange(gth.nx) * w.dx + np.random.default_rng(12).uniform(-4, 4, gth.nx)))
    prm = IrlsParams(p=p, q=q, n_outer=3, n_inner=6)
    mask = None
    if missing > 0:
        mask = (np.random.default_rng(13).uniform(size=gth.nx) >= missing).astype(np.uint8)
    print(f"[gpu] invert parity irregular traces p={p} q={q} missing={missing}", flush=True)
    m_g, d_g, rep, m_r, d_r, rep_r = _solve_both(A, kw, f32(gth.d_blend), prm, mask=mask)
    e = rel_l2(d_g, d_r)
    print(f"  d_rec rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-4
    np.testing.assert_allclose(rep["misfit"], rep_r["misfit"], rtol=1e-4)
