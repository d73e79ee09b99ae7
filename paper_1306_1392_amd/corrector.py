"""Learned sparse-angle corrector with a TV fallback.

x_hat = FBP(y) + UNet(FBP(y)); a slice whose corrected image does not explain
its data (|A x_hat - y| / |y| above a threshold calibrated on validation data)
is reconstructed by the TV-regularised mode (eq. (3), FISTA or Chambolle-Pock) instead.
Every step runs in the HIP library (FBP, U-Net kernels, projector, residual,
TV-CP); this module only sequences the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api
from .cnn import UNet


def save_weights(path: str, params, scale: float, base: int, levels: int):
    """Trained corrector: master weights with the data scale and architecture they belong to (.npz)."""
    p = params.detach().cpu().numpy() if torch.is_tensor(params) else np.asarray(params)
    np.savez(path, params=p.astype(np.float32), scale=np.float32(scale), base=np.int32(base),
             levels=np.int32(levels))


def load_weights(path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {"params": z["params"], "scale": float(z["scale"]), "base": int(z["base"]), "levels": int(z["levels"])}


class Corrector:
    def __init__(self, geometry: api.Geometry, batch: int, params, base: int = 32, levels: int = 4,
                 tv_lambda: float = 0.01, tv_iters: int = 300, dc_threshold: float | None = None,
                 tv_method: int = api.FISTA, tv_inner: int = 10, scale: float = 1.0):
        self.geo = geometry
        self.batch = batch
        self.plan = api.Plan(geometry, n_slices=batch)
        self.net = UNet(batch, geometry.n_y, geometry.n_x, base, levels)
        self.net.set_scale(scale)
        self.net.set_params(params)
        self.tv_lambda, self.tv_iters = tv_lambda, tv_iters
        self.tv_method, self.tv_inner = tv_method, tv_inner
        self.dc_threshold = dc_threshold
        self.op_norm = 0.0
        self._tv_plans = {}

    def fbp(self, y):
        return api.reconstruct_slices(self.plan, sino=y, method=api.FBP)

    def correct(self, y, out=None, ax=None, res=None):
        """FBP + U-Net for a full batch y [batch][K][nb]; returns (x_hat, residual per slice)."""
        x0 = self.fbp(y)
        xh = self.net.forward(x0, out=out)
        ax = api.forward_project(self.plan, xh, out=ax)
        return xh, api.slice_residual(self.plan, ax, y, out=res)

    def tv(self, y):
        """TV reconstruction (eq. (3); FISTA or Chambolle-Pock) of the slices in y [n][K][nb]."""
        n = y.shape[0]
        plan = self._tv_plans.get(n)
        if plan is None:
            plan = self._tv_plans[n] = api.Plan(self.geo, n_slices=n)
        x = api.reconstruct_slices(plan, sino=y.contiguous(), method=self.tv_method, lam=self.tv_lambda,
                                   n_iter=self.tv_iters, op_norm=self.op_norm, n_inner=self.tv_inner)
        self.op_norm = plan.last_op_norm
        return x

    def reconstruct(self, y):
        """Corrected FBP, with the TV mode for slices failing the data-consistency check.
        Returns (x, fallback mask as a numpy bool array)."""
        xh, r = self.correct(y)
        mask = np.zeros(y.shape[0], dtype=bool)
        if self.dc_threshold is not None:
            mask = (r > self.dc_threshold).cpu().numpy()
            if mask.any():
                idx = torch.as_tensor(np.nonzero(mask)[0], device=y.device)
                xh[idx] = self.tv(y[idx])
        return xh, mask
