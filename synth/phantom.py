"""Ellipse phantoms, their exact parallel-beam projections and rasters.

Units.  Phantoms live in normalised coordinates, field of view [-1, 1]^2.  An
image of N x N pixels of size ``s`` detector bins maps normalised length 1 to
``s * N / 2`` bins.  Line integrals are returned in bin units, so a filtered
backprojection of them returns the density ``rho`` itself.

Geometry convention (parallel beam, section 2.1 of the paper): pixel (ix, iy)
has centre x = ix - (n_x-1)/2, y = iy - (n_y-1)/2 (pixel units, +y = increasing
row index); at projection k with angle theta_k the point (x, y) lands on
detector coordinate t = s*(x cos theta_k + y sin theta_k) + c + sigma_k, where
detector bin j has its centre at coordinate j.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def rng_for(*key: int) -> np.random.Generator:
    """Seeded generator for the input stream identified by ``key``."""
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def random_ellipses(rng: np.random.Generator, n: int, axes=(0.05, 0.4), rho=(0.0, 1.0),
                    rmax: float = 0.95) -> np.ndarray:
    """``n`` random ellipses as rows (x0, y0, a, b, phi, rho).

    Semi-axes U[axes], orientation U[0, pi), density U[rho].  The centre is
    drawn uniformly in the unit disc and rejected until the whole ellipse stays
    inside the disc of radius ``rmax`` (|centre| <= rmax - max(a, b)), so no
    projection is truncated by the field of view.
    """
    out = np.zeros((n, 6), dtype=np.float64)
    for e in range(n):
        a, b = rng.uniform(axes[0], axes[1], size=2)
        phi = rng.uniform(0.0, math.pi)
        dens = rng.uniform(rho[0], rho[1])
        lim = rmax - max(a, b)
        while True:
            x0, y0 = rng.uniform(-1.0, 1.0, size=2)
            if x0 * x0 + y0 * y0 <= lim * lim:
                break
        out[e] = (x0, y0, a, b, phi, dens)
    return out


def disc_params(radius: float, rho: float = 1.0, x0: float = 0.0, y0: float = 0.0) -> np.ndarray:
    """A single disc as an ellipse row."""
    return np.array([[x0, y0, radius, radius, 0.0, rho]], dtype=np.float64)


def ellipse_sinogram(ell: np.ndarray, angles, n_det: int, axis: float, n_pix: int,
                     pixel_size: float = 1.0, shifts=None, device="cpu",
                     dtype=torch.float64) -> torch.Tensor:
    """Exact line integrals of a sum of ellipses, point-sampled at bin centres.

    Returns a [K][n_det] tensor.  For one ellipse (Kak & Slaney, ch. 3) the
    projection at angle theta and signed distance u is
    2 rho a b sqrt(m^2 - tau^2) / m^2 for |tau| <= m, with
    m^2 = a^2 cos^2(theta - phi) + b^2 sin^2(theta - phi) and
    tau = u - x0 cos theta - y0 sin theta.  Densities add where ellipses overlap.
    """
    th = torch.as_tensor(np.asarray(angles, dtype=np.float64), device=device, dtype=dtype)
    K = th.shape[0]
    sh = torch.zeros(K, device=device, dtype=dtype) if shifts is None else \
        torch.as_tensor(np.asarray(shifts, dtype=np.float64), device=device, dtype=dtype)
    scale = pixel_size * n_pix / 2.0                       # bins per unit normalised length
    j = torch.arange(n_det, device=device, dtype=dtype)
    u = (j[None, :] - axis - sh[:, None]) / scale            # [K][n_det], normalised
    ct, st = torch.cos(th)[:, None], torch.sin(th)[:, None]
    p = torch.zeros(K, n_det, device=device, dtype=dtype)
    for x0, y0, a, b, phi, rho in np.asarray(ell, dtype=np.float64):
        m2 = (a * torch.cos(th - phi)) ** 2 + (b * torch.sin(th - phi)) ** 2
        tau = u - x0 * ct - y0 * st
        r2 = m2[:, None] - tau * tau
        p += torch.where(r2 > 0, 2.0 * rho * a * b * torch.sqrt(torch.clamp(r2, min=0.0)) / m2[:, None],
                         torch.zeros((), device=device, dtype=dtype))
    return p * scale


def ellipse_raster(ell: np.ndarray, n_pix: int, sub: int = 4, device="cpu",
                   dtype=torch.float64) -> torch.Tensor:
    """Ground-truth image [n_pix][n_pix]: ellipse indicators averaged over sub x sub samples."""
    h = 2.0 / n_pix
    idx = torch.arange(n_pix, device=device, dtype=dtype)
    offs = (torch.arange(sub, device=device, dtype=dtype) + 0.5) / sub - 0.5
    coord = ((idx[:, None] - (n_pix - 1) / 2.0) + offs[None, :]) * h     # [n][sub]
    X = coord[None, None, :, :]     # x varies along ix (last dims: ix, sx)
    Y = coord[:, :, None, None]     # y varies along iy
    img = torch.zeros(n_pix, sub, n_pix, sub, device=device, dtype=dtype)
    for x0, y0, a, b, phi, rho in np.asarray(ell, dtype=np.float64):
        c, s = math.cos(phi), math.sin(phi)
        dx, dy = X - x0, Y - y0
        xr = dx * c + dy * s
        yr = -dx * s + dy * c
        img += rho * ((xr / a) ** 2 + (yr / b) ** 2 <= 1.0).to(dtype)
    return img.mean(dim=(1, 3))


def _perlin_octave(perm: np.ndarray, grads: np.ndarray, n_pix: int, freq: int) -> np.ndarray:
    """One octave of 2-D gradient noise with the quintic fade of Perlin (2002)."""
    xs = (np.arange(n_pix) + 0.5) * freq / n_pix
    xi = np.floor(xs).astype(np.int64)
    xf = xs - xi
    X0, Y0 = np.meshgrid(xi, xi, indexing="xy")
    FX, FY = np.meshgrid(xf, xf, indexing="xy")

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def corner(ox, oy):
        hsh = perm[(perm[(X0 + ox) & 255] + Y0 + oy) & 255] & 7
        g = grads[hsh]
        return g[..., 0] * (FX - ox) + g[..., 1] * (FY - oy)

    u, v = fade(FX), fade(FY)
    n00, n10, n01, n11 = corner(0, 0), corner(1, 0), corner(0, 1), corner(1, 1)
    nx0 = n00 + u * (n10 - n00)
    nx1 = n01 + u * (n11 - n01)
    return nx0 + v * (nx1 - nx0)


def perlin_texture(rng: np.random.Generator, n_pix: int, octaves: int = 3, base_freq: int = 8) -> np.ndarray:
    """Seeded gradient-noise texture in about [-1, 1], ``octaves`` octaves of doubling frequency."""
    perm = rng.permutation(256).astype(np.int64)
    grads = np.array([[1, 1], [-1, 1], [1, -1], [-1, -1], [1, 0], [-1, 0], [0, 1], [0, -1]],
                     dtype=np.float64)
    out = np.zeros((n_pix, n_pix))
    amp, tot = 1.0, 0.0
    for o in range(octaves):
        out += amp * _perlin_octave(perm, grads, n_pix, base_freq << o)
        tot += amp
        amp *= 0.5
    return out / tot


def perlin_texture_torch(rng: np.random.Generator, n_pix: int, octaves: int = 3, base_freq: int = 8,
                         device="cpu") -> torch.Tensor:
    """Device version of perlin_texture (same lattice, fade and gradient set), float32 [n][n]."""
    perm = torch.as_tensor(rng.permutation(256).astype(np.int64), device=device)
    grads = torch.tensor([[1, 1], [-1, 1], [1, -1], [-1, -1], [1, 0], [-1, 0], [0, 1], [0, -1]],
                         dtype=torch.float32, device=device)
    out = torch.zeros(n_pix, n_pix, device=device)
    amp, tot = 1.0, 0.0
    for o in range(octaves):
        freq = base_freq << o
        xs = (torch.arange(n_pix, device=device, dtype=torch.float32) + 0.5) * freq / n_pix
        xi = torch.floor(xs).to(torch.int64)
        xf = xs - xi
        X0, Y0 = xi[None, :].expand(n_pix, n_pix), xi[:, None].expand(n_pix, n_pix)
        FX, FY = xf[None, :].expand(n_pix, n_pix), xf[:, None].expand(n_pix, n_pix)

        def corner(ox, oy):
            h = perm[(perm[(X0 + ox) & 255] + Y0 + oy) & 255] & 7
            g = grads[h]
            return g[..., 0] * (FX - ox) + g[..., 1] * (FY - oy)

        def fade(t):
            return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

        u, v = fade(FX), fade(FY)
        n00, n10, n01, n11 = corner(0, 0), corner(1, 0), corner(0, 1), corner(1, 1)
        nx0 = n00 + u * (n10 - n00)
        nx1 = n01 + u * (n11 - n01)
        out += amp * (nx0 + v * (nx1 - nx0))
        tot += amp
        amp *= 0.5
    return out / tot
