"""Survey-level source separation (thesis Chapters 2 and 4): blend a cube of
shot gathers into continuous receiver records, pseudo-deblend them into
common receiver gathers, separate every gather in one batched robust
inversion, and re-sort the separated gathers to common source gathers.

Binding only: blending, pseudo-deblending, re-sorting and the inversion run
in the library's HIP kernels (ashrt_blend, ashrt_deblend, ashrt_resort,
robust_invert_batched).  Tensors are torch CUDA tensors; firing times are
int32 samples.
"""
import ctypes as C

import torch

from . import _lib as L
from .ashrt import BatchPlan, Params


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream(dev):
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _fire(fire, dev):
    return torch.as_tensor(fire, dtype=torch.int32, device=dev).contiguous()


def record_length(fire, nt):
    return int(max(int(f) for f in fire)) + int(nt)


def blend(D, fire, nrec=None):
    """D [ns][nr][nt] -> continuous records b [nr][nrec]."""
    ns, nr, nt = D.shape
    f = _fire(fire, D.device)
    nrec = nrec or record_length(f.tolist(), nt)
    b = torch.empty((nr, nrec), dtype=torch.float32, device=D.device)
    L.check(L.lib().ashrt_blend(_ptr(D), ns, nr, nt, _ptr(f), _ptr(b), nrec, _stream(D.device)), "ashrt_blend")
    return b


def deblend(b, fire, ns, nt, receiver_major=True):
    """Pseudo-deblended cube: [nr][ns][nt] (receiver gathers) or [ns][nr][nt]."""
    nr, nrec = b.shape
    f = _fire(fire, b.device)
    shape = (nr, ns, nt) if receiver_major else (ns, nr, nt)
    out = torch.empty(shape, dtype=torch.float32, device=b.device)
    L.check(L.lib().ashrt_deblend(_ptr(b), ns, nr, nt, _ptr(f), nrec, _ptr(out), int(bool(receiver_major)),
                                  _stream(b.device)), "ashrt_deblend")
    return out


def resort(x):
    """[a][b][nt] -> [b][a][nt]."""
    na, nb, nt = x.shape
    out = torch.empty((nb, na, nt), dtype=torch.float32, device=x.device)
    L.check(L.lib().ashrt_resort(_ptr(x), na, nb, nt, _ptr(out), _stream(x.device)), "ashrt_resort")
    return out


def separate(b, fire, ns, nt, dt, dx, vel, params: Params, fmax=100.0, tuning=None, want_report=False):
    """Separate every common receiver gather of the blended records b
    [nr][nrec] (apex grid = source grid) and return the separated common
    source gathers [ns][nr][nt], plus the reports if asked."""
    crg = deblend(b, fire, ns, nt, receiver_major=True)
    nr = crg.shape[0]
    plan = BatchPlan([dict(nt=nt, nx=ns, dt=dt, dx=dx, vel=list(vel), fmax=fmax)] * nr, device=b.device,
                     tuning=tuning)
    # identical gathers are packed back to back: the receiver-major cube is the packed batch
    assert int(plan.data_off[-1]) == (nr - 1) * ns * nt and plan.data_total == nr * ns * nt
    _, drec, reps = plan.robust_invert(crg.reshape(-1), params, want_report=want_report)
    csg = resort(drec.view(nr, ns, nt))
    return (csg, reps) if want_report else csg
