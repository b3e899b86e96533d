"""Binding of the warm-start U-Net (include/unet.h): argument marshalling only.

Tensors are torch CUDA tensors (FP32, contiguous) on the network's device;
every compute step runs in the library's HIP kernels.
"""
import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class TrainParams:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    weight_decay: float = 0.0
    lam_w: float = 1.0

    def c(self):
        return L.UnetTrainParams(self.lr, self.beta1, self.beta2, self.eps, self.weight_decay, self.lam_w)


class UNet:
    """U-Net with four 2x down-samplings: gather [H][W] -> model [P][H][W] and weights [H][W]
    (H, W multiples of 16)."""

    def __init__(self, pout, base=16, cin=1, device=0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        d = L.UnetDesc(cin, pout, base)
        h = C.c_void_p()
        L.check(L.lib().unet_create(C.byref(d), self.device.index or 0, C.byref(h)), "unet_create")
        self._h = h
        self.pout, self.base, self.cin = pout, base, cin
        self.n_params = int(L.lib().unet_param_count(h))
        self._ws = {}
        self._loss = torch.zeros(1, dtype=torch.float64, device=self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and L is not None and L._lib is not None:
            L.lib().unet_destroy(h)
        self._h = None

    def set_params(self, theta):
        a = np.ascontiguousarray(np.asarray(theta, np.float32).ravel())
        L.check(L.lib().unet_set_params(self._h, a.ctypes.data_as(C.c_void_p), a.size), "unet_set_params")

    def init_params(self, seed=0):
        """He-normal weights (fan-in), zero biases, drawn on the host."""
        rng = np.random.default_rng(seed)
        c1, c2, c3, c4 = (self.base * f for f in (1, 2, 4, 8))
        c5 = c4
        convs = [(self.cin, c1, 3), (c1, c1, 3), (c1, c2, 3), (c2, c2, 3), (c2, c3, 3), (c3, c3, 3),
                 (c3, c4, 3), (c4, c4, 3), (c4, c5, 3), (c5, c5, 3), (c5 + c4, c4, 3), (c4, c4, 3),
                 (c4 + c3, c3, 3), (c3, c3, 3), (c3 + c2, c2, 3), (c2, c2, 3),
                 (c2 + c1, c1, 3), (c1, c1, 3), (c1, self.pout, 1), (c1, 1, 1)]
        parts = []
        for ci, co, k in convs:
            parts.append(rng.standard_normal(co * ci * k * k) * np.sqrt(2.0 / (ci * k * k)))
            parts.append(np.zeros(co))
        theta = np.concatenate(parts)
        assert theta.size == self.n_params
        self.set_params(theta)
        return theta

    def get_params(self):
        a = np.empty(self.n_params, np.float32)
        L.check(L.lib().unet_get_params(self._h, a.ctypes.data_as(C.c_void_p), a.size), "unet_get_params")
        return a

    def workspace(self, B, H, W, train):
        n = C.c_size_t()
        L.check(L.lib().unet_workspace_bytes(self._h, B, H, W, int(train), C.byref(n)), "unet_workspace_bytes")
        key = bool(train)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < n.value:
            ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def forward(self, x):
        """x [B][H][W] -> (y_model [B][P][H][W], y_w [B][H][W])."""
        B, H, W = x.shape
        y_m = torch.empty((B, self.pout, H, W), dtype=torch.float32, device=self.device)
        y_w = torch.empty((B, H, W), dtype=torch.float32, device=self.device)
        ws = self.workspace(B, H, W, False)
        L.check(L.lib().unet_forward(self._h, _ptr(x), B, H, W, _ptr(y_m), _ptr(y_w), _ptr(ws), ws.numel(),
                                     _stream(self.device)), "unet_forward")
        return y_m, y_w

    def loss_grad(self, x, t_m, t_w, lam_w=1.0):
        B, H, W = x.shape
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        ws = self.workspace(B, H, W, True)
        L.check(L.lib().unet_loss_grad(self._h, _ptr(x), _ptr(t_m), _ptr(t_w), B, H, W, float(lam_w),
                                       _ptr(self._loss), _ptr(g), _ptr(ws), ws.numel(), _stream(self.device)),
                "unet_loss_grad")
        return float(self._loss.item()), g

    def train_step(self, x, t_m, t_w, tp: TrainParams, want_loss=True):
        B, H, W = x.shape
        ws = self.workspace(B, H, W, True)
        prm = tp.c()
        L.check(L.lib().unet_train_step(self._h, C.byref(prm), _ptr(x), _ptr(t_m), _ptr(t_w), B, H, W,
                                        _ptr(self._loss), _ptr(ws), ws.numel(), _stream(self.device)),
                "unet_train_step")
        return float(self._loss.item()) if want_loss else None
