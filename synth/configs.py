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

from .phantom import rng_for, random_ellipses, ellipse_sinogram, ellipse_raster, perlin_texture_torch
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


def cfg_uneven(n_slices: int = 500, index: int = 0, n_ell: int = 10, device="cpu", sizes=(512, 1024, 2048),
               k_range=(90, 3600)):
    """Uneven batch: N ~ U{sizes}, K ~ U{k_range}; half of the slices are 360 degree
    half-acquisition scans with the axis delta ~ U[16, 64] bins from a detector edge
    (nb = ceil(N/2) + delta + 1; right or left edge with equal probability), the others
    180 degree full-detector scans; per-projection axis shifts ~ N(0, 0.5^2).
    Returns dict(specs=[dict(N, K, nb, axis, scan, angles, shifts)], sinos=[tensor [K][nb] f32])."""
    rng = rng_for(5, 0, index)
    specs, sinos = [], []
    for i in range(n_slices):
        N = int(rng.choice(sizes))
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        half = i % 2 == 1
        shifts = rng.normal(0.0, 0.5, K)
        if half:
            delta = float(rng.uniform(16, 64))
            nb = int(math.ceil(N / 2)) + int(math.ceil(delta)) + 1
            right = bool(rng.integers(0, 2))
            axis = nb - 1 - delta if right else delta
            ang = uniform_angles(K, 2 * math.pi)
            scan = 2
        else:
            nb = N
            axis = (N - 1) / 2.0 + float(rng.uniform(-4, 4))
            ang = uniform_angles(K)
            scan = 0
        ell = random_ellipses(rng, n_ell, rmax=0.9)
        p = ellipse_sinogram(ell, ang, nb, axis, N, shifts=shifts, device=device).float()
        specs.append(dict(N=N, K=K, nb=nb, axis=axis, scan=scan, angles=ang, shifts=shifts, ell=ell))
        sinos.append(p)
    return dict(specs=specs, sinos=sinos)


def cfg_learned(indices, stream: int, project, N: int = 512, K: int = 90, n_ell: int = 10, photons: float = 1e4,
                device="cpu"):
    """Sparse-angle learned-corrector data: phantom = ellipses + a Perlin texture of
    amplitude 0.2 rho inside the ellipses; sinogram = exact ellipse projections + the
    projection of the texture rasterised at 2N x 2N (pixel 0.5 bin, so the data are not
    made with the reconstruction grid) through ``project(texture [1][2N][2N]) -> [1][K][N]``;
    Poisson counts at ``photons`` per bin, per-slice kappa.  Seeds [4, stream, index].
    Returns (y [B][K][N] f32 line integrals, truth [B][N][N] f32 in the units of y, angles, axis)."""
    ang = uniform_angles(K)
    axis = (N - 1) / 2.0
    ys, truths = [], []
    for i in indices:
        rng = rng_for(4, stream, int(i))
        ell = random_ellipses(rng, n_ell)
        dens_hi = ellipse_raster(ell, 2 * N, sub=2, device=device).float()
        tex = 0.2 * perlin_texture_torch(rng, 2 * N, device=device) * dens_hi
        p = ellipse_sinogram(ell, ang, N, axis, N, device=device).float() + project(tex[None].contiguous())[0]
        truth = ellipse_raster(ell, N, device=device).float() + tex.reshape(N, 2, N, 2).mean(dim=(1, 3))
        y, kap = poisson_sinogram(p, seed=4_000_000 + 1_000_000 * stream + int(i), photons=photons)
        ys.append(y)
        truths.append(truth * kap)
    return torch.stack(ys), torch.stack(truths), ang, axis
