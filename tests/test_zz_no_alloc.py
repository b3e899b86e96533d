"""The allocation-free forward (ashrt_forward_noalloc: the library's static
device scratch in place of a caller workspace) against ashrt_forward, through
the C ABI: two calls in a row, the production gather and then a smaller one
with a trace mask, each bit-identical to the workspace entry point (same
kernels, same order); and a plan whose forward needs more than the static
scratch is refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    import paper_1711_10214_amd as A
    assert torch.cuda.is_available()
    return A


def test_forward_noalloc_matches_forward_on_two_calls(A):
    import torch
    rng = np.random.default_rng(7)
    cases = [(1024, 256, list(np.linspace(1400.0, 4000.0, 32)), 0.0),   # 79 MiB of scratch
             (200, 48, [1500.0, 2300.0, 3100.0], 0.25)]
    for nt, nx, vel, mfrac in cases:
        print(f"[gpu] forward_noalloc nt={nt} nx={nx} P={len(vel)} mask={mfrac}", flush=True)
        plan = A.Plan(nt, nx, 0.004, 12.5, vel, fmax=100.0)
        m = torch.tensor(rng.standard_normal((len(vel), nx, nt)), dtype=torch.float32, device="cuda")
        mask = None
        if mfrac > 0:
            mask = torch.tensor((rng.uniform(size=nx) >= mfrac).astype(np.uint8), device="cuda")
        d_ref = plan.forward(m, mask=mask)
        out = torch.full((nx, nt), float("nan"), dtype=torch.float32, device="cuda")
        plan.forward_noalloc(m, out, mask=mask)
        torch.cuda.synchronize()
        assert torch.equal(out, d_ref)


def test_forward_noalloc_refuses_a_workspace_beyond_the_scratch(A):
    import torch
    vel = [float(v) for v in np.linspace(1400.0, 4000.0, 24) for _ in range(16)]   # 384 panels
    plan = A.Plan(1024, 256, 0.004, 12.5, vel, fmax=100.0)
    m = torch.zeros((384, 256, 1024), dtype=torch.float32, device="cuda")
    out = torch.zeros((256, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(A.AshrtError, match="allocation-free"):
        plan.forward_noalloc(m, out)
