"""Python binding of the U-Net corrector entry points (argument marshalling only;
the network runs in the HIP library)."""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import check


def layer_table(base: int, levels: int):
    """(name, kind, c_in, c_out, weight_offset, bias_offset) in the flat parameter order."""
    rows, off = [], 0

    def add(name, kind, cin, cout):
        nonlocal off
        nw = {"conv": 9 * cin * cout, "up": 4 * cin * cout, "head": cin}[kind]
        rows.append((name, kind, cin, cout, off, off + nw))
        off += nw + (cout if kind != "head" else 1)

    for l in range(levels):
        c = base << l
        add(f"enc{l}a", "conv", 8 if l == 0 else base << (l - 1), c)
        add(f"enc{l}b", "conv", c, c)
    for l in range(levels - 2, -1, -1):
        c = base << l
        add(f"up{l}", "up", 2 * c, c)
        add(f"dec{l}a", "conv", 2 * c, c)
        add(f"dec{l}b", "conv", c, c)
    add("head", "head", base, 1)
    return rows, off


def init_params(base: int, levels: int, seed: int = 0) -> np.ndarray:
    """He-normal weights (fan-in of the real inputs), zero biases, zero head."""
    rows, n = layer_table(base, levels)
    rng = np.random.default_rng(np.random.SeedSequence([4, 7, seed]))
    p = np.zeros(n, dtype=np.float32)
    for name, kind, cin, cout, w, b in rows:
        if kind == "conv":
            real = 1 if name == "enc0a" else cin
            W = rng.standard_normal((cout, 9, cin)) * math.sqrt(2.0 / (9 * real))
            if name == "enc0a":
                W[:, :, 1:] = 0.0
            p[w:b] = W.ravel()
        elif kind == "up":
            p[w:b] = (rng.standard_normal((4, cout, cin)) * math.sqrt(2.0 / cin)).ravel()
    return p


class UNet:
    def __init__(self, batch: int, height: int, width: int, base: int = 32, levels: int = 4):
        self.L = _lib.lib()
        h = ctypes.c_void_p()
        check(self.L.pyhst_unet_create(batch, height, width, base, levels, ctypes.byref(h)), "pyhst_unet_create")
        self.handle = h
        n = ctypes.c_int64()
        check(self.L.pyhst_unet_num_params(h, ctypes.byref(n)), "pyhst_unet_num_params")
        self.n_params = n.value
        self.batch, self.height, self.width, self.base, self.levels = batch, height, width, base, levels
        self.layers, n2 = layer_table(base, levels)
        assert n2 == self.n_params, (n2, self.n_params)
        self.loss_buf = None

    @staticmethod
    def _p(t):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float32):
            raise ValueError("contiguous float32 device tensors only")
        return ctypes.c_void_p(t.data_ptr())

    @staticmethod
    def _s(stream=None):
        return ctypes.c_void_p((torch.cuda.current_stream() if stream is None else stream).cuda_stream)

    def set_scale(self, scale: float):
        """Data scale c: the network sees c x and returns x + f(c x)/c (it belongs with the weights)."""
        check(self.L.pyhst_unet_set_scale(self.handle, float(scale)), "pyhst_unet_set_scale")

    @property
    def scale(self) -> float:
        v = ctypes.c_float()
        check(self.L.pyhst_unet_get_scale(self.handle, ctypes.byref(v)), "pyhst_unet_get_scale")
        return v.value

    def set_params(self, params, stream=None):
        t = torch.as_tensor(params, dtype=torch.float32).to("cuda").contiguous()
        assert t.numel() == self.n_params
        check(self.L.pyhst_unet_set_params(self.handle, self._p(t), self._s(stream)), "pyhst_unet_set_params")
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def get_params(self, stream=None):
        t = torch.empty(self.n_params, device="cuda", dtype=torch.float32)
        check(self.L.pyhst_unet_get_params(self.handle, self._p(t), self._s(stream)), "pyhst_unet_get_params")
        return t

    def get_grads(self, stream=None):
        t = torch.empty(self.n_params, device="cuda", dtype=torch.float32)
        check(self.L.pyhst_unet_get_grads(self.handle, self._p(t), self._s(stream)), "pyhst_unet_get_grads")
        return t

    def _check_in(self, x):
        n = x.shape[0]
        if x.shape[1:] != (self.height, self.width) or n > self.batch:
            raise ValueError(f"input must be [n <= {self.batch}][{self.height}][{self.width}]")
        return n

    def forward(self, x, out=None, stream=None):
        n = self._check_in(x)
        out = torch.empty_like(x) if out is None else out
        check(self.L.pyhst_unet_forward(self.handle, self._p(x), n, self._p(out), self._s(stream)),
              "pyhst_unet_forward")
        return out

    def backward(self, x, target, stream=None):
        n = self._check_in(x)
        if self.loss_buf is None:
            self.loss_buf = torch.zeros(1, device="cuda", dtype=torch.float32)
        check(self.L.pyhst_unet_backward(self.handle, self._p(x), self._p(target), n, self._p(self.loss_buf),
                                         self._s(stream)), "pyhst_unet_backward")
        return self.loss_buf

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        check(self.L.pyhst_unet_adam(self.handle, float(lr), float(beta1), float(beta2), float(eps),
                                     self._s(stream)), "pyhst_unet_adam")

    def train_step(self, x, target, lr, stream=None):
        n = self._check_in(x)
        if self.loss_buf is None:
            self.loss_buf = torch.zeros(1, device="cuda", dtype=torch.float32)
        check(self.L.pyhst_unet_train_step(self.handle, self._p(x), self._p(target), n, float(lr),
                                           self._p(self.loss_buf), self._s(stream)), "pyhst_unet_train_step")
        return self.loss_buf

    KINDS = {"x8": 0, "ea": 1, "cat": 2, "pool": 3, "da": 4, "db": 5, "bott": 6}

    def tensor(self, kind: str, level: int = 0, grad: bool = False):
        """Internal activation (or its gradient) as float32 [batch][H_l][W_l][C] (BF16 values)."""
        H, W = self.height >> level, self.width >> level
        c = self.base << level
        C = {"x8": 8, "ea": c, "cat": 2 * c, "pool": c, "da": c, "db": c,
             "bott": self.base << (self.levels - 1)}[kind]
        if kind == "pool":
            H, W = H // 2, W // 2
        if kind == "bott":
            H, W = self.height >> (self.levels - 1), self.width >> (self.levels - 1)
        n = self.batch * H * W * C
        buf = torch.empty(n, device="cuda", dtype=torch.int16)
        check(self.L.pyhst_unet_tensor(self.handle, self.KINDS[kind], level, int(grad), ctypes.c_void_p(buf.data_ptr()),
                                       n, self._s()), "pyhst_unet_tensor")
        f = (buf.to(torch.int32) & 0xFFFF) << 16
        return f.view(torch.float32).reshape(self.batch, H, W, C)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.L.pyhst_unet_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
