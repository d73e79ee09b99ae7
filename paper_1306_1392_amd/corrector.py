"""Learned sparse-angle corrector with a TV fallback.

x_hat = FBP(y) + UNet(FBP(y)); a slice whose corrected image does not explain
its data (|A x_hat - y| / |y| above a threshold calibrated on validation data)
is reconstructed by the TV-regularised mode (eq. (3), FISTA or Chambolle-Pock) instead.
Every step runs in the HIP library (FBP, U-Net kernels, projector, residual,
TV); this module only sequences the calls.  The network carries its data scale
(it sees scale * x and returns x + f(scale * x) / scale), so the corrector, its
training and its calibration all work in the units of the reconstruction.
"""
from __future__ import annotations

import math

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


def rmse(a, b) -> float:
    """Root-mean-square difference of two image stacks (evaluation only)."""
    return float(torch.sqrt(torch.mean((a.double() - b.double()) ** 2)))


def train(net: UNet, x, t, steps: int, lr: float = 1e-3, seed: int = 11, every: int = 100, log=None):
    """Adam on minibatches of net.batch pairs (FBP input x, truth t; [n][H][W], reconstruction units),
    reshuffled every epoch, cosine-decayed learning rate.  Returns [(step, loss)] every `every` steps."""
    n, B = x.shape[0], net.batch
    per_epoch = n // B
    if per_epoch < 1:
        raise ValueError("need at least one full batch of training pairs")
    rng = np.random.default_rng(seed)
    losses = []
    for st in range(steps):
        if st % per_epoch == 0:
            perm = torch.as_tensor(rng.permutation(n), device=x.device)
        idx = perm[(st % per_epoch) * B:(st % per_epoch + 1) * B]
        loss = net.train_step(x[idx].contiguous(), t[idx].contiguous(), lr * 0.5 * (1 + math.cos(math.pi * st / steps)))
        if st % every == 0 or st == steps - 1:
            losses.append((st, float(loss)))
            if log:
                log(f"corrector: step {st}/{steps} loss {losses[-1][1]:.4g}")
    return losses


def calibrate_tv_lambda(geometry: api.Geometry, y, truth, method: int = api.FISTA, n_iter: int = 300,
                        n_inner: int = 10, lam0: float = 1e-3, lam1: float = 3.2, widen: int = 4):
    """Regularisation weight of eq. (3) by ground-truth calibration (section 3.1): minimum RMSE against
    the truth on validation slices over a half-decade grid from lam0 to lam1, widened by half-decade
    steps (at most `widen` times) while the minimum sits at an end of the grid.  Chambolle-Pock runs
    with the balanced gradient block (mu = |A| / |grad|).
    Returns (lambda, {lambda: rmse}, op_norm, mu)."""
    plan = api.Plan(geometry, n_slices=y.shape[0])
    yc = y.contiguous()
    norm = [0.0]
    mu = api.balanced_mu(plan) if method == api.TV_CP else 1.0

    def ev(lam):
        x = api.reconstruct_slices(plan, sino=yc, method=method, lam=lam, n_iter=n_iter, op_norm=norm[0],
                                   n_inner=n_inner, tv_mu=mu)
        norm[0] = plan.last_op_norm
        return rmse(x, truth)

    grid = 10.0 ** np.arange(math.log10(lam0), math.log10(lam1) + 0.01, 0.5)
    cal = {lam: ev(lam) for lam in [float(f"{v:.3g}") for v in grid]}
    for _ in range(widen):
        best = min(cal, key=cal.get)
        if best == min(cal):
            lam = float(f"{best / 10 ** 0.5:.3g}")
        elif best == max(cal):
            lam = float(f"{best * 10 ** 0.5:.3g}")
        else:
            break
        cal[lam] = ev(lam)
    return min(cal, key=cal.get), cal, norm[0], mu


class Corrector:
    def __init__(self, geometry: api.Geometry, batch: int, params, base: int = 32, levels: int = 4,
                 tv_lambda: float = 0.01, tv_iters: int = 300, dc_threshold: float | None = None,
                 tv_method: int = api.FISTA, tv_inner: int = 10, scale: float = 1.0, op_norm: float = 0.0,
                 tv_mu: float = 1.0):
        self.geo = geometry
        self.batch = batch
        self.plan = api.Plan(geometry, n_slices=batch)
        self.net = UNet(batch, geometry.n_y, geometry.n_x, base, levels)
        self.net.set_scale(scale)
        self.net.set_params(params)
        self.tv_lambda, self.tv_iters = tv_lambda, tv_iters
        self.tv_method, self.tv_inner = tv_method, tv_inner
        self.dc_threshold = dc_threshold
        self.op_norm, self.tv_mu = op_norm, tv_mu
        self._tv_plans = {}
        self._fbp_work = None

    @classmethod
    def from_net(cls, geometry: api.Geometry, net: UNet, **kw):
        """Corrector around a trained network (its weights, architecture and data scale)."""
        return cls(geometry, net.batch, net.get_params(), base=net.base, levels=net.levels, scale=net.scale, **kw)

    def fbp(self, y):
        if self._fbp_work is None:
            self._fbp_work = torch.empty(api.work_bytes(self.plan, sino=y, method=api.FBP), device=y.device,
                                         dtype=torch.uint8)
        return api.reconstruct_slices(self.plan, sino=y, method=api.FBP, work=self._fbp_work)

    def _full(self, y):
        """Pad a partial batch [n <= batch][K][nb] to the plan's batch (the padding slices are ignored)."""
        n = y.shape[0]
        if n > self.batch:
            raise ValueError(f"at most {self.batch} slices per call")
        if n < self.batch:
            y = torch.cat([y, y[:1].expand(self.batch - n, -1, -1)])
        return y.contiguous(), n

    def correct(self, y, out=None, ax=None, res=None):
        """FBP + U-Net for y [n <= batch][K][nb]; returns (x_hat [n], residual per slice [n])."""
        yf, n = self._full(y)
        x0 = self.fbp(yf)
        xh = self.net.forward(x0, out=out if out is not None and n == self.batch else None)
        ax = api.forward_project(self.plan, xh, out=ax)
        r = api.slice_residual(self.plan, ax, yf, out=res)
        return xh[:n], r[:n]

    def calibrate(self, y_val, quantile: float = 0.95, factor: float = 1.5) -> float:
        """Data-consistency threshold: factor x the quantile of the validation residuals."""
        rs = [self.correct(y_val[i:i + self.batch])[1] for i in range(0, y_val.shape[0], self.batch)]
        self.dc_threshold = factor * float(np.quantile(torch.cat(rs).cpu().numpy(), quantile))
        return self.dc_threshold

    def tv(self, y):
        """TV reconstruction (eq. (3); FISTA or Chambolle-Pock) of the slices in y [n][K][nb]."""
        n = y.shape[0]
        plan = self._tv_plans.get(n)
        if plan is None:
            plan = self._tv_plans[n] = api.Plan(self.geo, n_slices=n)
        x = api.reconstruct_slices(plan, sino=y.contiguous(), method=self.tv_method, lam=self.tv_lambda,
                                   n_iter=self.tv_iters, op_norm=self.op_norm, n_inner=self.tv_inner,
                                   tv_mu=self.tv_mu)
        self.op_norm = plan.last_op_norm
        return x

    def reconstruct(self, y):
        """Corrected FBP of y [n <= batch][K][nb], with the TV mode for slices failing the data-consistency
        check.  Returns (x [n][n_y][n_x], fallback mask as a numpy bool array)."""
        xh, r = self.correct(y)
        mask = np.zeros(y.shape[0], dtype=bool)
        if self.dc_threshold is not None:
            mask = (r > self.dc_threshold).cpu().numpy()
            if mask.any():
                idx = torch.as_tensor(np.nonzero(mask)[0], device=y.device)
                xh[idx] = self.tv(y[idx])
        return xh, mask

    def reconstruct_all(self, y):
        """reconstruct() over y [n][K][nb] in batches; returns (x [n], fallback mask [n])."""
        xs, ms = [], []
        for i in range(0, y.shape[0], self.batch):
            x, m = self.reconstruct(y[i:i + self.batch])
            xs.append(x.clone())
            ms.append(m)
        return torch.cat(xs), np.concatenate(ms)
