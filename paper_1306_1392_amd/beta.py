"""Choice of the TV weight beta of eq. (3) without ground truth (section 3.1).

The paper evaluates two estimators after reconstructing a slice at several
beta values:
  * cross-validation: reconstruct without one projection, then measure the
    squared distance between the reconstruction's projection at that angle and
    the excluded data (averaged here over several excluded projections);
  * the decoherence estimator E_cohe = cos(I(beta) - I(0+), I(beta)), whose
    absolute value is smallest near the best beta.
Every reconstruction, projection and reduction runs in the HIP library; this
module only sequences the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


def _drop(geo: api.Geometry, k: int) -> api.Geometry:
    keep = np.arange(geo.n_angles) != k
    shifts = None if geo.axis_shift is None else np.asarray(geo.axis_shift)[keep]
    return api.Geometry(geo.n_x, geo.n_y, geo.n_det, np.asarray(geo.angles)[keep], geo.axis_pos, axis_shift=shifts,
                        scan=geo.scan, pixel_size=geo.pixel_size, ha_overlap=geo.ha_overlap)


def select_beta(geo: api.Geometry, y, betas, *, excluded=None, beta0: float | None = None,
                method: int = api.FISTA, n_iter: int = 200, n_inner: int = 10):
    """Estimator curves over `betas` for the slices y [S][K][n_det] (device float32).

    Returns a dict with, per beta (arrays [len(betas)][S]): 'cv' (mean squared distance over the
    excluded projections), 'e_cohe' (cosine against the reconstruction at beta0, default
    betas.min() / 100), and the full-data reconstructions 'x' [len(betas)][S][n_y][n_x]."""
    betas = np.asarray(betas, dtype=np.float64)
    S = y.shape[0]
    if excluded is None:
        excluded = np.linspace(0, geo.n_angles - 1, 4).round().astype(int)[:-1] + geo.n_angles // 8
    full = api.Plan(geo, n_slices=S)
    kw = dict(method=method, n_iter=n_iter, n_inner=n_inner)
    x0 = api.reconstruct_slices(full, sino=y, lam=float(beta0 if beta0 is not None else betas.min() / 100), **kw)
    op_norm = full.last_op_norm
    xs, ec = [], []
    for b in betas:
        x = api.reconstruct_slices(full, sino=y, lam=float(b), op_norm=op_norm, **kw)
        xs.append(x)
        ec.append(api.decoherence(full, x, x0).cpu().numpy())
    # the library averages over the excluded projections: weight 1/count, accumulated after the first
    cv = torch.zeros((len(betas), S), device=y.device, dtype=torch.float32)
    wgt = 1.0 / len(excluded)
    for n, k in enumerate(excluded):
        part = _drop(geo, int(k))
        plan_k = api.Plan(part, n_slices=S)
        keep = torch.as_tensor(np.nonzero(np.arange(geo.n_angles) != k)[0], device=y.device)
        yk = y.index_select(1, keep).contiguous()
        nk = 0.0
        for i, b in enumerate(betas):
            xk = api.reconstruct_slices(plan_k, sino=yk, lam=float(b), op_norm=nk, **kw)
            nk = plan_k.last_op_norm
            api.cv_error(full, xk, y, int(k), out=cv[i], weight=wgt, accumulate=n > 0)
    return {"betas": betas, "cv": cv.cpu().numpy().astype(np.float64), "e_cohe": np.array(ec), "x": torch.stack(xs),
            "excluded": np.asarray(excluded)}
