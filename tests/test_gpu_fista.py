"""GPU FISTA (l2-l1 sparse inversion of the thesis' Chapter 6) against the
FP64 oracle on the same seeded inputs, through the C ABI (fista_invert).

Bar: the power-method Lipschitz constant and mu to 1e-4 relative, and after
the iterations the reconstructed gather L m and the objective to 1e-4
relative (soft thresholding is not smooth, so the FP32 iterates may differ
from the FP64 ones in which tiny coefficients sit exactly at zero)."""
import numpy as np
import pytest

import oracle
from oracle.fista import FistaParams
from synth import make_gather, workload
from tests.gpu_common import f32, geom_kwargs, oracle_geometry, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available()
    return A


def _both(A, kw, d, prm: FistaParams, mask=None):
    import torch
    g = oracle_geometry(kw)
    plan = A.Plan(**kw)
    mk = None if mask is None else torch.tensor(mask, device="cuda")
    m_g, dr_g, rep = plan.fista(torch.tensor(d, dtype=torch.float32, device="cuda"), n_iter=prm.n_iter,
                                n_power=prm.n_power, mu=prm.mu, mu_rel=prm.mu_rel, lip_safety=prm.lip_safety,
                                mask=mk)
    m_r, dr_r, rep_r = oracle.fista.fista(g, d, prm, mask=mask)
    return m_g.cpu().numpy(), dr_g.cpu().numpy(), rep, m_r, dr_r, rep_r


def test_fista_blended_gather_matches_oracle(A):
    w = workload("crg-256x64-nv8")
    gth = make_gather(w)
    kw = geom_kwargs(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    prm = FistaParams(n_iter=30, n_power=20, mu_rel=0.05)
    print("[gpu] fista crg-256x64-nv8 30 iterations", flush=True)
    m_g, dr_g, rep, m_r, dr_r, rep_r = _both(A, kw, f32(gth.d_blend), prm)
    print(f"  Lf {rep['lipschitz']:.6g} / {rep_r['lipschitz']:.6g}  mu {rep['mu']:.6g} / {rep_r['mu']:.6g}", flush=True)
    print(f"  objective {rep['objective']:.6g} / {rep_r['objective']:.6g}  d_rec rel-L2 {rel_l2(dr_g, dr_r):.2e}"
          f"  m rel-L2 {rel_l2(m_g, m_r):.2e}", flush=True)
    assert abs(rep["lipschitz"] / rep_r["lipschitz"] - 1) <= 1e-4
    assert abs(rep["mu"] / rep_r["mu"] - 1) <= 1e-4
    assert abs(rep["objective"] / rep_r["objective"] - 1) <= 1e-4
    assert rel_l2(dr_g, dr_r) <= 1e-4


def test_fista_decimated_aashrt_interpolation_matches_oracle(A):
    """Chapter 6's use: reconstruct a decimated gather with the asymptote-
    shifted model (FISTA, sampling mask)."""
    w = workload("aashrt-1024x256-nv24x16", nt=200, nx=48, vel=(1600.0, 1600.0, 2600.0, 2600.0),
                 tau0=(0, 10, 0, 10), n_diffractors=4, n_events=(2, 2), tau_range=(0.1, 0.5))
    gth = make_gather(w)
    kw = geom_kwargs(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), tau0=list(w.tau0), fmax=w.fmax)
    prm = FistaParams(n_iter=40, n_power=15, mu_rel=0.02)
    print("[gpu] fista aashrt decimated", flush=True)
    m_g, dr_g, rep, m_r, dr_r, rep_r = _both(A, kw, f32(gth.d_blend), prm, mask=gth.mask)
    e = rel_l2(dr_g, dr_r)
    print(f"  d_rec rel-L2 {e:.2e}; Q gpu {oracle.q_db(gth.d_clean, dr_g):.3f} dB oracle "
          f"{oracle.q_db(gth.d_clean, dr_r):.3f} dB (decimated {oracle.q_db(gth.d_clean, gth.d_blend):.3f})", flush=True)
    assert e <= 1e-4
    assert abs(rep["objective"] / rep_r["objective"] - 1) <= 1e-4


def test_fista_irregular_traces_with_missing_matches_oracle(A):
    """FISTA on jittered trace positions (non-uniform DFTs on the data side)
    with a third of the traces missing: the thesis' interpolation on
    irregular, incomplete data."""
    w = workload("crg-256x64-nv8")
    gth = make_gather(w)
    kw = geom_kwargs(gth.nt, gth.nx, w.dt, w.dx, list(w.vel), fmax=w.fmax)
    kw = dict(kw, xpos=list(np.arange(gth.nx) * w.dx + np.random.default_rng(21).uniform(-4, 4, gth.nx)))
    mask = (np.random.default_rng(22).uniform(size=gth.nx) >= 0.33).astype(np.uint8)
    prm = FistaParams(n_iter=30, n_power=20, mu_rel=0.05)
    print("[gpu] fista irregular traces, a third missing", flush=True)
    m_g, dr_g, rep, m_r, dr_r, rep_r = _both(A, kw, f32(gth.d_blend), prm, mask=mask)
    e = rel_l2(dr_g, dr_r)
    print(f"  Lf {rep['lipschitz']:.6g} / {rep_r['lipschitz']:.6g}  d_rec rel-L2 {e:.2e}", flush=True)
    assert abs(rep["lipschitz"] / rep_r["lipschitz"] - 1) <= 1e-4
    assert abs(rep["objective"] / rep_r["objective"] - 1) <= 1e-4
    assert e <= 1e-4


def test_fista_rejects_bad_params(A):
    import torch
    kw = geom_kwargs(64, 16, 0.004, 12.5, [1500.0], fmax=100.0)
    plan = A.Plan(**kw)
    d = torch.zeros((16, 64), device="cuda")
    with pytest.raises(A.AshrtError):
        plan.fista(d, n_iter=0)
    with pytest.raises(A.AshrtError):
        plan.fista(d, mu=0.0, mu_rel=0.0)
    with pytest.raises(A.AshrtError):
        plan.fista(d, lip_safety=0.5)
