"""The workloads, as seeded recipes.

Seeds follow np.random.SeedSequence([workload, stream, index]); stream 0 is
the generic stream, 1 the test stream, 2 the validation stream.

* single_slice: 256^2 image, 256 bins, 180 angles over [0, pi), axis 127.5,
  10 ellipses, exact sinogram + Gaussian noise with sd 1 % of its maximum.
* batched_raw: R slices of N^2 (default 64 x 2048^2), N bins, 1800 angles
  over [0, pi), axis offset +3.5 bins from the detector centre, 20 ellipses
  per slice, raw uint16 radiographs with two flats and a dark.
* tv_sparse: 1024^2, 1024 bins, 128 angles over [0, pi), 10 ellipses,
  Poisson data at 1e4 photons per bin.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .phantom import rng_for, random_ellipses, ellipse_sinogram, ellipse_raster
from .acquisition import raw_acquisition, poisson_sinogram


def uniform_angles(K: int, span: float = math.pi) -> np.ndarray:
    return np.arange(K, dtype=np.float64) * (span / K)


def cfg_single_slice(index: int = 0, N: int = 256, K: int = 180, noise_frac: float = 0.01,
                     n_ell: int = 10, device="cpu"):
    """Returns dict(sino [K][N] f32, angles, axis, ell, truth [N][N] f64)."""
    rng = rng_for(1, 0, index)
    ell = random_ellipses(rng, n_ell)
    ang = uniform_angles(K)
    axis = (N - 1) / 2.0
    p = ellipse_sinogram(ell, ang, N, axis, N, device=device)
    if noise_frac > 0:
        nz = torch.as_tensor(rng.standard_normal(p.shape), device=device)
        p = p + noise_frac * float(p.max()) * nz
    return dict(sino=p.float(), angles=ang, axis=axis, ell=ell, N=N, K=K,
                truth=None if N > 1024 else ellipse_raster(ell, N, device=device))


def cfg_batched_raw(R: int = 64, N: int = 2048, K: int = 1800, n_ell: int = 20, axis_offset: float = 3.5,
                    index: int = 0, device="cpu", noise: bool = True):
    """Raw radiograph stack for R slices. Returns dict(raw, flats, flat_pos, dark, kappa, angles, axis, ells)."""
    ang = uniform_angles(K)
    axis = (N - 1) / 2.0 + axis_offset
    ells = []
    p = torch.empty(R, K, N, device=device, dtype=torch.float64)
    for r in range(R):
        ell = random_ellipses(rng_for(2, 0, index * 100000 + r), n_ell)
        ells.append(ell)
        p[r] = ellipse_sinogram(ell, ang, N, axis, N, device=device)
    raw, flats, flat_pos, dark, kap = raw_acquisition(p, seed=2_000_000 + index, noise=noise)
    del p
    return dict(raw=raw, flats=flats, flat_pos=flat_pos, dark=dark, kappa=kap, angles=ang,
                axis=axis, ells=ells, N=N, K=K, R=R)


def cfg_tv_sparse(N: int = 1024, K: int = 128, n_ell: int = 10, index: int = 0, photons: float = 1e4,
                  device="cpu"):
    """Poisson sparse-angle sinogram. Returns dict(y [K][N] f32, kappa, angles, axis, ell, truth)."""
    rng = rng_for(3, 0, index)
    ell = random_ellipses(rng, n_ell)
    ang = uniform_angles(K)
    axis = (N - 1) / 2.0
    p = ellipse_sinogram(ell, ang, N, axis, N, device=device)
    y, kap = poisson_sinogram(p, seed=3_000_000 + index, photons=photons)
    return dict(y=y, kappa=kap, angles=ang, axis=axis, ell=ell, N=N, K=K,
                truth=None if N > 1024 else ellipse_raster(ell, N, device=device) * kap)
