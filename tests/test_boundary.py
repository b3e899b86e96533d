"""Host-only checks of the C ABI boundary (no GPU needed): the library loads,
exports every function include/*.h declares, validates descriptors and
solver settings, names its status codes, and the Python binding turns error
codes into exceptions.  No compute call is made here."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


@pytest.fixture(scope="module")
def A():
    import paper_1711_10214_amd as A
    return A


def _declared_functions():
    src = "\n".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for")))


def test_header_functions_are_exported(A):
    names = _declared_functions()
    assert "ashrt_forward" in names and "robust_invert" in names and "robust_invert_batched" in names
    assert "unet_forward" in names and "unet_train_step" in names
    assert "ashrt_autotune" in names and "ashrt_plan_create_tuned" in names
    lib = A.lib()
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", A._lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_library_is_built_for_gfx950(A):
    # the fat binary carries a gfx950 code object
    data = open(A._lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def _desc(A, **kw):
    base = dict(nt=1024, nx=256, dt=0.004, dx=12.5, vel=np.linspace(1400, 4000, 32), fmax=100.0)
    base.update(kw)
    return A.validate_desc(**base)


def test_desc_validation(A):
    L = A._lib
    assert _desc(A) == L.ASHRT_OK
    assert _desc(A, nt=1) == L.ASHRT_E_INVALID_ARG
    assert _desc(A, dt=0.0) == L.ASHRT_E_INVALID_ARG
    assert _desc(A, dx=-1.0) == L.ASHRT_E_INVALID_ARG
    assert _desc(A, vel=[-1.0]) == L.ASHRT_E_INVALID_ARG
    assert _desc(A, vel=[float("nan")]) == L.ASHRT_E_INVALID_ARG
    assert _desc(A, ntp=1000) == L.ASHRT_E_UNSUPPORTED_SIZE        # not 2^a or 3*2^a
    assert _desc(A, ntp=512) == L.ASHRT_E_INVALID_ARG              # shorter than nt
    assert _desc(A, nt=4096) == L.ASHRT_E_UNSUPPORTED_SIZE         # auto ntp 8192 > 4096
    assert _desc(A, ntp=3072) == L.ASHRT_OK                        # radix 3
    assert _desc(A, half_width=9) == L.ASHRT_E_INVALID_ARG
    assert _desc(A, tau0=[-1] * 32) == L.ASHRT_E_INVALID_ARG
    assert _desc(A, fmin=200.0, fmax=100.0) == L.ASHRT_E_INVALID_ARG  # empty band
    assert "band" in A.lib().ashrt_last_error().decode()


def test_null_desc_and_params(A):
    lib = A.lib()
    assert lib.ashrt_desc_validate(None) == A._lib.ASHRT_E_INVALID_ARG
    assert lib.irls_params_validate(None) == A._lib.ASHRT_E_INVALID_ARG


def test_params_validation(A):
    lib = A.lib()
    L = A._lib

    def v(**kw):
        p = A.Params(**kw).c()
        return lib.irls_params_validate(C.byref(p))

    assert v() == L.ASHRT_OK
    assert v(p=3) == L.ASHRT_E_INVALID_ARG
    assert v(q=0) == L.ASHRT_E_INVALID_ARG
    assert v(n_outer=0) == L.ASHRT_E_INVALID_ARG
    assert v(n_outer=65) == L.ASHRT_E_INVALID_ARG
    assert v(n_inner=0) == L.ASHRT_E_INVALID_ARG
    assert v(b_r=0.0) == L.ASHRT_E_INVALID_ARG
    assert v(tol=-1.0) == L.ASHRT_E_INVALID_ARG
    d = L.IrlsParams()
    lib.irls_params_default(C.byref(d))
    assert (d.p, d.q, d.n_outer, d.n_inner, d.b_r, d.b_m, d.tol) == (1, 2, 10, 20, 1.345, 1.0, 0.0)


def test_status_strings(A):
    lib = A.lib()
    for code in range(0, -8, -1):
        s = lib.ashrt_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.ashrt_status_string(-99).decode() == "unknown status"
    import re
    hdr = open(os.path.join(ROOT, "include", "ashrt.h")).read()
    assert lib.ashrt_abi_version() == int(re.search(r"#define ASHRT_ABI_VERSION (\d+)", hdr).group(1))
    assert lib.ashrt_abi_version() == A._lib.ABI_VERSION


def test_null_plan_and_workspace_errors(A):
    lib = A.lib()
    L = A._lib
    n = C.c_size_t()
    assert lib.ashrt_workspace_bytes(None, 0, None, C.byref(n)) == L.ASHRT_E_INVALID_ARG
    assert lib.ashrt_forward(None, None, None, None, None, 0, None) == L.ASHRT_E_INVALID_ARG
    assert lib.robust_invert(None, None, None, None, None, None, None, None, None, 0, None) == L.ASHRT_E_INVALID_ARG
    with pytest.raises(A.AshrtError):
        L.check(L.ASHRT_E_INVALID_ARG, "test")


def test_plan_create_fails_cleanly_without_gpu(A):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(A.AshrtError) as ei:
        A.Plan(256, 64, 0.004, 12.5, [1500.0] * 8, fmax=100.0)
    assert ei.value.status == A._lib.ASHRT_E_HIP


def test_unet_entry_points_reject_bad_arguments_without_gpu(A):
    lib = A.lib()
    L = A._lib
    out = C.c_void_p()
    assert lib.unet_create(None, 0, C.byref(out)) == L.ASHRT_E_INVALID_ARG
    bad = L.UnetDesc(2, 8, 16)
    assert lib.unet_create(C.byref(bad), 0, C.byref(out)) == L.ASHRT_E_UNSUPPORTED_SIZE
    bad = L.UnetDesc(1, 8, 12)
    assert lib.unet_create(C.byref(bad), 0, C.byref(out)) == L.ASHRT_E_UNSUPPORTED_SIZE
    assert lib.unet_param_count(None) == -1
    n = C.c_size_t()
    assert lib.unet_workspace_bytes(None, 1, 16, 16, 0, C.byref(n)) == L.ASHRT_E_INVALID_ARG
