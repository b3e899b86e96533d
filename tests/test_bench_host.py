"""Host-side checks of bench.py (no GPU): every workload the command line
dispatches to exists, --gpus above 1 is refused with a message, and the
per-launch algorithmic byte counts of the row kernels match a direct count
of what each launch must read and write."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_every_dispatched_workload_exists(bench):
    src = open(os.path.join(ROOT, "bench.py")).read()
    main = src[src.index("def main():"):]
    import re
    called = set(re.findall(r"return (run_\w+)\(args\)", main))
    assert called >= {"run_warmstart", "run_batch", "run_speedratio", "run_survey", "run_unet", "run_separation"}
    for name in called:
        assert callable(getattr(bench, name)), name
    for name in ("headline", "batch_leg", "aashrt_leg", "warmstart_leg", "separation_leg", "unet_leg",
                 "cpu_baseline"):
        assert callable(getattr(bench, name)), name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_row_kernel_bytes_match_a_direct_count(bench):
    """Forward row launch: the live x-spectrum rows (nt complex each) read
    once, the panel-sum partials (2 nband complex per row) written once;
    adjoint: the data spectrum read once, the live rows written once."""
    import numpy as np
    nt, nx, P, dt, dx = 1024, 256, 32, 0.004, 12.5
    vel = list(np.linspace(1400.0, 4000.0, P))
    ntp, nxp = 2048, 512
    fmax = 100.0
    jlo, jhi = 1, int(np.floor(fmax * ntp * dt))
    info = {"ntp": ntp, "nxp": nxp, "jlo": jlo, "jhi": jhi, "nchunk": 1}
    nums = bench._geometry_numbers(info, vel, dt, dx, nx, nt, P, 4)
    nrows = nxp // 2
    live = 0
    for v in vel:
        c2 = (v * ntp * dt / (nxp * dx)) ** 2
        live += sum(1 for r in range(nrows) if r == 0 or c2 * r * r <= jhi * jhi * (1 + 1e-9))
    nband = jhi - jlo + 1
    x_live = live * nt * 8
    partials = nrows * 2 * nband * 8
    data_spec = nrows * nt * 8
    fwd_bytes, _ = nums["k_rows_fwd"]
    adj_bytes, _ = nums["k_rows_adj"]
    assert fwd_bytes == pytest.approx(x_live + partials, rel=1e-12)
    assert adj_bytes == pytest.approx(data_spec + x_live, rel=1e-12)
