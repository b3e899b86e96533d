"""Python binding of libashrt with PyTorch tensors as device memory.

Every step of the operator and of the solver runs in the library's HIP
kernels; this module only builds descriptors, allocates tensors and
workspaces with torch, and passes pointers and the current stream.
"""
import ctypes as C
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _dptr(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


@dataclass
class Params:
    """Robust inversion settings (thesis Chapter 4)."""
    p: int = 1
    q: int = 2
    n_outer: int = 10
    n_inner: int = 20
    b_r: float = 1.345
    b_m: float = 1.0
    tol: float = 0.0
    eps_floor_rel: float = 1e-6
    freeze_eps: bool = False
    cg_graph: bool = True

    def c(self):
        return L.IrlsParams(self.p, self.q, self.n_outer, self.n_inner, self.b_r, self.b_m,
                            self.tol, self.eps_floor_rel, int(bool(self.freeze_eps)),
                            int(bool(self.cg_graph)))


def report_dict(r: L.IrlsReport):
    n = r.outer_done
    return {"status": r.status, "outer_done": n,
            "inner": list(r.inner[:n]), "misfit": list(r.misfit[:n]),
            "huber": list(r.huber[:n]), "eps_r": list(r.eps_r[:n]), "eps_m": list(r.eps_m[:n])}


class _Desc:
    """Owns the host arrays a descriptor points to."""

    def __init__(self, nt, nx, dt, dx, vel, tau0=None, scale=None, ntp=0, nxp=0, fmin=0.0,
                 fmax=0.0, half_width=4, wavelet=None, xpos=None):
        self.vel = np.ascontiguousarray(np.asarray(vel, np.float64).ravel())
        self.xpos = None if xpos is None else np.ascontiguousarray(np.asarray(xpos, np.float64).ravel())
        P = len(self.vel)
        self.tau0 = None if tau0 is None else np.ascontiguousarray(np.asarray(tau0, np.int32).ravel())
        self.scale = None if scale is None else np.ascontiguousarray(np.asarray(scale, np.float64).ravel())
        self.wavelet = None if wavelet is None else np.ascontiguousarray(np.asarray(wavelet, np.float64).ravel())
        d = L.AshrtDesc()
        L.lib().ashrt_desc_default(C.byref(d))
        d.nt, d.nx, d.ntp, d.nxp = int(nt), int(nx), int(ntp), int(nxp)
        d.dt, d.dx = float(dt), float(dx)
        d.npanel = P
        d.vel = _dptr(self.vel, C.c_double)
        d.tau0_samples = _dptr(self.tau0, C.c_int32) if self.tau0 is not None else None
        d.panel_scale = _dptr(self.scale, C.c_double) if self.scale is not None else None
        d.fmin_hz, d.fmax_hz = float(fmin), float(fmax)
        d.half_width = int(half_width)
        d.wavelet_amp = _dptr(self.wavelet, C.c_double) if self.wavelet is not None else None
        if self.xpos is not None:
            assert self.xpos.size == int(nx), "xpos needs one position per trace"
        d.x_pos = _dptr(self.xpos, C.c_double) if self.xpos is not None else None
        self.c = d


def validate_desc(**kw) -> int:
    """Host-only check of a descriptor; returns the C status code."""
    return L.lib().ashrt_desc_validate(C.byref(_Desc(**kw).c))


def _desc_kwargs(nt, nx, dt, dx, vel, tau0, scale, ntp, nxp, fmin, fmax, half_width, wavelet, xpos=None):
    return dict(nt=nt, nx=nx, dt=dt, dx=dx, vel=vel, tau0=tau0, scale=scale, ntp=ntp, nxp=nxp, fmin=fmin,
                fmax=fmax, half_width=half_width, wavelet=wavelet, xpos=xpos)


def _tuning(t):
    if t is None:
        return None
    return L.Tuning(int(t.get("tile_model", 0)), int(t.get("tile_data", 0)), int(t.get("nchunk", 0)))


def autotune(device=0, repeats=3, **geom):
    """Fastest tiling of one forward + adjoint pair for this geometry (the
    library's autotuner; cached per geometry for the process)."""
    d = _Desc(**geom)
    best = L.Tuning()
    ms = C.c_double()
    L.check(L.lib().ashrt_autotune(C.byref(d.c), int(device), int(repeats), C.byref(best), C.byref(ms)),
            "ashrt_autotune")
    return {"tile_model": best.tile_model, "tile_data": best.tile_data, "nchunk": best.nchunk, "pair_ms": ms.value}


class Plan:
    """One gather geometry and its panel list (velocity, asymptote shift, scale)."""

    def __init__(self, nt, nx, dt, dx, vel, tau0=None, scale=None, ntp=0, nxp=0, fmin=0.0,
                 fmax=0.0, half_width=4, wavelet=None, device=0, tuning=None, xpos=None):
        """tuning: None (built-in tiling), "auto" (run the autotuner, cached
        per geometry) or a dict with tile_model / tile_data / nchunk."""
        self._desc = _Desc(nt, nx, dt, dx, vel, tau0, scale, ntp, nxp, fmin, fmax, half_width, wavelet, xpos)
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if isinstance(tuning, str) and tuning == "auto":
            tuning = autotune(device=self.device.index or 0, **_desc_kwargs(nt, nx, dt, dx, vel, tau0, scale, ntp,
                                                                          nxp, fmin, fmax, half_width, wavelet,
                                                                          xpos))
        self.tuning = tuning
        tn = _tuning(tuning)
        h = C.c_void_p()
        L.check(L.lib().ashrt_plan_create_tuned(C.byref(self._desc.c), C.byref(tn) if tn is not None else None,
                                                self.device.index or 0, C.byref(h)), "ashrt_plan_create")
        self._h = h
        info = L.PlanInfo()
        L.check(L.lib().ashrt_plan_get_info(self._h, C.byref(info)), "ashrt_plan_get_info")
        self.info = {k: getattr(info, k) for k, _ in L.PlanInfo._fields_}
        self.nt, self.nx, self.npanel = int(nt), int(nx), len(self._desc.vel)
        self.dt, self.dx = float(dt), float(dx)
        self.vel = self._desc.vel
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and L is not None and L._lib is not None:
            L.lib().ashrt_plan_destroy(h)
        self._h = None

    # ---------------------------------------------------------------- workspace
    def workspace_bytes(self, op, params: Optional[Params] = None):
        n = C.c_size_t()
        prm = params.c() if params is not None else None
        L.check(L.lib().ashrt_workspace_bytes(self._h, op, C.byref(prm) if prm is not None else None,
                                              C.byref(n)), "ashrt_workspace_bytes")
        return n.value

    def workspace(self, op, params: Optional[Params] = None):
        n = self.workspace_bytes(op, params)
        ws = self._ws.get(op)
        if ws is None or ws.numel() < n:
            ws = torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
            self._ws[op] = ws
        return ws

    # ---------------------------------------------------------------- operators
    def _check_model(self, m):
        assert m.dtype == torch.float32 and m.is_contiguous() and m.device == self.device
        assert tuple(m.shape) == (self.npanel, self.nx, self.nt), tuple(m.shape)

    def _check_data(self, d):
        assert d.dtype == torch.float32 and d.is_contiguous() and d.device == self.device
        assert tuple(d.shape) == (self.nx, self.nt), tuple(d.shape)

    def _mask(self, mask):
        if mask is None:
            return None
        mask = mask.to(device=self.device, dtype=torch.uint8).contiguous()
        assert tuple(mask.shape) == (self.nx,)
        return mask

    def forward(self, m, mask=None, out=None):
        """d = S L m."""
        self._check_model(m)
        mask = self._mask(mask)
        d = out if out is not None else torch.empty((self.nx, self.nt), dtype=torch.float32, device=self.device)
        self._check_data(d)
        ws = self.workspace(L.OP_FORWARD)
        L.check(L.lib().ashrt_forward(self._h, _ptr(m), _ptr(d), _ptr(mask), _ptr(ws), ws.numel(),
                                      _stream(self.device)), "ashrt_forward")
        return d

    def forward_noalloc(self, m, out, mask=None):
        """d = S L m through ashrt_forward_noalloc: the library's static
        device scratch instead of a workspace (the caller passes the output;
        nothing is allocated)."""
        self._check_model(m)
        self._check_data(out)
        mk = self._mask(mask)
        L.check(L.lib().ashrt_forward_noalloc(self._h, _ptr(m), _ptr(out), _ptr(mk), _stream(self.device)),
                "ashrt_forward_noalloc")
        return out

    def adjoint(self, d, mask=None, out=None):
        """m = L' S d."""
        self._check_data(d)
        mask = self._mask(mask)
        m = out if out is not None else torch.empty((self.npanel, self.nx, self.nt), dtype=torch.float32,
                                                    device=self.device)
        self._check_model(m)
        ws = self.workspace(L.OP_ADJOINT)
        L.check(L.lib().ashrt_adjoint(self._h, _ptr(d), _ptr(m), _ptr(mask), _ptr(ws), ws.numel(),
                                      _stream(self.device)), "ashrt_adjoint")
        return m

    def fista(self, d, n_iter=50, n_power=20, mu=0.0, mu_rel=0.05, lip_safety=1.05, mask=None, m0=None,
              want_report=True):
        """l2-l1 inversion by FISTA (thesis Chapter 6).  Returns (m, L m, report)."""
        self._check_data(d)
        mask = self._mask(mask)
        m = (torch.zeros((self.npanel, self.nx, self.nt), dtype=torch.float32, device=self.device)
             if m0 is None else m0.clone())
        self._check_model(m)
        drec = torch.empty_like(d)
        prm = L.FistaParams(int(n_iter), int(n_power), float(mu), float(mu_rel), float(lip_safety))
        ws = self.workspace(L.OP_FISTA)
        rep = L.FistaReport() if want_report else None
        L.check(L.lib().fista_invert(self._h, C.byref(prm), _ptr(d), _ptr(mask), _ptr(m), _ptr(drec),
                                     C.byref(rep) if rep is not None else None, _ptr(ws), ws.numel(),
                                     _stream(self.device)), "fista_invert")
        out = None if rep is None else {k: getattr(rep, k) for k, _ in L.FistaReport._fields_}
        return m, drec, out

    def td_forward(self, m, mask=None, out=None):
        """Time-domain (classical) forward operator (no padding, band or wavelet)."""
        self._check_model(m)
        d = out if out is not None else torch.empty((self.nx, self.nt), dtype=torch.float32, device=self.device)
        L.check(L.lib().ashrt_td_forward(self._h, _ptr(m), _ptr(d), _ptr(self._mask(mask)), _stream(self.device)),
                "ashrt_td_forward")
        return d

    def td_adjoint(self, d, mask=None, out=None):
        """Time-domain (classical) adjoint operator."""
        self._check_data(d)
        m = out if out is not None else torch.empty((self.npanel, self.nx, self.nt), dtype=torch.float32,
                                                    device=self.device)
        L.check(L.lib().ashrt_td_adjoint(self._h, _ptr(d), _ptr(m), _ptr(self._mask(mask)), _stream(self.device)),
                "ashrt_td_adjoint")
        return m

    def robust_invert(self, d, params: Params, mask=None, m0=None, w0=None, want_drec=True,
                      want_report=True):
        """IRLS-CG solve.  Returns (m, d_rec or None, report dict or None)."""
        self._check_data(d)
        mask = self._mask(mask)
        m = (torch.zeros((self.npanel, self.nx, self.nt), dtype=torch.float32, device=self.device)
             if m0 is None else m0.clone())
        self._check_model(m)
        if w0 is not None:
            self._check_data(w0)
        drec = torch.empty_like(d) if want_drec else None
        prm = params.c()
        ws = self.workspace(L.OP_INVERT, params)
        rep = L.IrlsReport() if want_report else None
        L.check(L.lib().robust_invert(self._h, C.byref(prm), _ptr(d), _ptr(mask), _ptr(m), _ptr(w0),
                                      _ptr(drec), C.byref(rep) if rep is not None else None, _ptr(ws),
                                      ws.numel(), _stream(self.device)), "robust_invert")
        return m, drec, (report_dict(rep) if rep is not None else None)


class BatchPlan:
    """Many gathers of uneven size in one plan; arrays are packed."""

    def __init__(self, descs: Sequence[dict], device=0, tuning=None):
        """tuning: None or a dict (tile_model / tile_data / nchunk) applied to every gather."""
        self._descs = [_Desc(**kw) for kw in descs]
        arr = (L.AshrtDesc * len(self._descs))(*[d.c for d in self._descs])
        self._arr = arr
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        tn = _tuning(tuning)
        h = C.c_void_p()
        L.check(L.lib().ashrt_batch_plan_create_tuned(arr, len(self._descs), C.byref(tn) if tn is not None else None,
                                                      self.device.index or 0, C.byref(h)),
                "ashrt_batch_plan_create")
        self._h = h
        n = len(self._descs)
        do, mo, ko = (np.zeros(n, np.int64) for _ in range(3))
        tot = [C.c_int64() for _ in range(3)]
        L.check(L.lib().ashrt_batch_layout(self._h, _dptr(do, C.c_int64), _dptr(mo, C.c_int64),
                                           _dptr(ko, C.c_int64), *[C.byref(t) for t in tot]),
                "ashrt_batch_layout")
        self.data_off, self.model_off, self.mask_off = do, mo, ko
        self.data_total, self.model_total, self.mask_total = (t.value for t in tot)
        self.shapes = [(int(kw["nt"]), int(kw["nx"]), len(np.ravel(kw["vel"]))) for kw in descs]
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and L is not None and L._lib is not None:
            L.lib().ashrt_batch_plan_destroy(h)
        self._h = None

    def workspace(self, op, params: Optional[Params] = None):
        n = C.c_size_t()
        prm = params.c() if params is not None else None
        L.check(L.lib().ashrt_batch_workspace_bytes(self._h, op, C.byref(prm) if prm is not None else None,
                                                    C.byref(n)), "ashrt_batch_workspace_bytes")
        ws = self._ws.get(op)
        if ws is None or ws.numel() < n.value:
            ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=self.device)
            self._ws[op] = ws
        return ws

    def pack_data(self, arrays):
        out = torch.zeros(self.data_total, dtype=torch.float32, device=self.device)
        for g, a in enumerate(arrays):
            a = torch.as_tensor(a, dtype=torch.float32).reshape(-1)
            out[self.data_off[g]: self.data_off[g] + a.numel()] = a.to(self.device)
        return out

    def pack_model(self, arrays):
        out = torch.zeros(self.model_total, dtype=torch.float32, device=self.device)
        for g, a in enumerate(arrays):
            a = torch.as_tensor(a, dtype=torch.float32).reshape(-1)
            out[self.model_off[g]: self.model_off[g] + a.numel()] = a.to(self.device)
        return out

    def pack_mask(self, masks):
        out = torch.ones(self.mask_total, dtype=torch.uint8, device=self.device)
        for g, a in enumerate(masks):
            if a is None:
                continue
            a = torch.as_tensor(a, dtype=torch.uint8).reshape(-1)
            out[self.mask_off[g]: self.mask_off[g] + a.numel()] = a.to(self.device)
        return out

    def unpack_data(self, packed, g):
        nt, nx, _ = self.shapes[g]
        return packed[self.data_off[g]: self.data_off[g] + nt * nx].view(nx, nt)

    def unpack_model(self, packed, g):
        nt, nx, P = self.shapes[g]
        return packed[self.model_off[g]: self.model_off[g] + P * nt * nx].view(P, nx, nt)

    def forward(self, m_packed, mask_packed=None, out=None):
        d = out if out is not None else torch.empty(self.data_total, dtype=torch.float32, device=self.device)
        ws = self.workspace(L.OP_FORWARD)
        L.check(L.lib().ashrt_forward_batched(self._h, _ptr(m_packed), _ptr(d), _ptr(mask_packed), _ptr(ws),
                                              ws.numel(), _stream(self.device)), "ashrt_forward_batched")
        return d

    def adjoint(self, d_packed, mask_packed=None, out=None):
        m = out if out is not None else torch.empty(self.model_total, dtype=torch.float32, device=self.device)
        ws = self.workspace(L.OP_ADJOINT)
        L.check(L.lib().ashrt_adjoint_batched(self._h, _ptr(d_packed), _ptr(m), _ptr(mask_packed), _ptr(ws),
                                              ws.numel(), _stream(self.device)), "ashrt_adjoint_batched")
        return m

    def robust_invert(self, d_packed, params: Params, mask_packed=None, m0_packed=None, w0_packed=None,
                      want_drec=True, want_report=True):
        m = (torch.zeros(self.model_total, dtype=torch.float32, device=self.device)
             if m0_packed is None else m0_packed.clone())
        drec = torch.empty(self.data_total, dtype=torch.float32, device=self.device) if want_drec else None
        prm = params.c()
        ws = self.workspace(L.OP_INVERT, params)
        n = len(self._descs)
        reps = (L.IrlsReport * n)() if want_report else None
        L.check(L.lib().robust_invert_batched(self._h, C.byref(prm), _ptr(d_packed), _ptr(mask_packed), _ptr(m),
                                              _ptr(w0_packed), _ptr(drec), reps, _ptr(ws), ws.numel(),
                                              _stream(self.device)), "robust_invert_batched")
        return m, drec, ([report_dict(r) for r in reps] if reps is not None else None)
