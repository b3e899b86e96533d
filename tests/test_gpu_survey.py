"""GPU blending, pseudo-deblending, re-sorting and survey-level separation
against the FP64 oracle (oracle/blending.py, oracle.robust_invert per
receiver gather), through the C ABI."""
import numpy as np
import pytest

import oracle
from oracle import blending as OB
from oracle.irls import IrlsParams
from synth import make_survey
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available()
    return A


def test_blend_deblend_resort_match_oracle(A):
    import torch
    from paper_1711_10214_amd import survey as S
    sv = make_survey(ns=12, nt=128, seed=3)
    D = torch.tensor(sv.D, dtype=torch.float32, device="cuda")
    b = S.blend(D, sv.fire)
    Df = sv.D.astype(np.float32).astype(np.float64)
    b_ref = OB.blend(Df, sv.fire)
    assert rel_l2(b.cpu().numpy(), b_ref) <= 1e-6
    c_ref = OB.deblend(b_ref, sv.fire, 128)
    bt = torch.tensor(b_ref, dtype=torch.float32, device="cuda")
    c_src = S.deblend(bt, sv.fire, 12, 128, receiver_major=False).cpu().numpy()
    c_rcv = S.deblend(bt, sv.fire, 12, 128, receiver_major=True).cpu().numpy()
    assert rel_l2(c_src, c_ref) <= 1e-7
    assert np.array_equal(c_rcv, np.transpose(c_src, (1, 0, 2)))
    assert np.array_equal(S.resort(torch.tensor(c_src, device="cuda")).cpu().numpy(), c_rcv)


def test_survey_separation_matches_oracle(A):
    """16 sources x 16 receivers: every receiver gather separated in one
    batched solve equals the oracle's per-gather solve."""
    import torch
    from paper_1711_10214_amd import survey as S
    sv = make_survey(ns=16, nt=256, seed=4, n_events=4)
    vel = list(np.linspace(1500.0, 3200.0, 6))
    D = torch.tensor(sv.D, dtype=torch.float32, device="cuda")
    b = S.blend(D, sv.fire)
    prm = A.Params(p=1, q=2, n_outer=3, n_inner=5)
    print("[gpu] survey separation 16 x 16 x 256", flush=True)
    csg = S.separate(b, sv.fire, 16, 256, sv.dt, sv.dx, vel, prm, fmax=100.0).cpu().numpy()
    b_np = b.cpu().numpy().astype(np.float64)
    crg = np.transpose(OB.deblend(b_np, sv.fire, 256), (1, 0, 2))
    g = oracle.geometry(256, 16, sv.dt, sv.dx, vel, fmax=100.0)
    sep = np.stack([oracle.robust_invert(g, crg[r], IrlsParams(p=1, q=2, n_outer=3, n_inner=5))[1]
                    for r in range(16)])
    csg_ref = np.transpose(sep, (1, 0, 2))
    e = rel_l2(csg, csg_ref)
    q_sep = oracle.q_db(sv.D, csg)
    q_pd = oracle.q_db(sv.D, np.transpose(crg, (1, 0, 2)))
    print(f"  rel-L2 vs oracle {e:.2e}; Q separated {q_sep:.2f} dB, pseudo-deblended {q_pd:.2f} dB", flush=True)
    assert e <= 1e-4
    assert q_sep > q_pd
