"""Simulated detector data: raw uint16 radiographs with flats and dark, and
photon-counting sinograms.

The paper's processing pipe (section 2.3) starts from radiographs, a dark
image and flat fields taken at several times.  This module produces such data
from exact line integrals so that the reconstruction can be checked end to end.
It only models the acquisition (Beer-Lambert attenuation plus photon noise); it
does not normalise anything.
"""
from __future__ import annotations

import numpy as np
import torch


def kappa_for(p: torch.Tensor, max_att: float = 3.0) -> float:
    """Scale of the line integrals so that transmission stays >= exp(-max_att)."""
    pm = float(p.max())
    return 1.0 if pm <= 0 else min(1.0, max_att / pm)


def raw_acquisition(p: torch.Tensor, seed: int, flat_range=(30000.0, 40000.0), dark_mean=100.0,
                    dark_sd=5.0, noise: bool = True, rounding: bool = True):
    """Radiographs of a stack of sinograms ``p`` [R][K][nb] (line integrals, bin units).

    Two flats F0, F1 ~ U[flat_range] per detector pixel, acquired before the
    first and after the last projection; the beam drifts linearly between
    them.  Dark ~ N(dark_mean, dark_sd^2) per pixel.  Each slice's integrals are
    scaled by its own kappa (transmission >= 5 %).  Counts are
    D + Poisson((F_k - D) exp(-kappa p)), rounded and clipped to uint16.

    Returns (raw [K][R][nb] uint16, flats [2][R][nb] f32, flat_pos [2] f64,
    dark [R][nb] f32, kappa [R] f64).  With ``noise=False, rounding=False`` the
    raw stack is returned as float64 (the noise-free model itself).
    """
    R, K, nb = p.shape
    dev = p.device
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    f0 = torch.empty(R, nb, device=dev, dtype=torch.float64).uniform_(flat_range[0], flat_range[1], generator=g)
    f1 = torch.empty(R, nb, device=dev, dtype=torch.float64).uniform_(flat_range[0], flat_range[1], generator=g)
    dark = dark_mean + dark_sd * torch.randn(R, nb, device=dev, dtype=torch.float64, generator=g)
    # the method receives float32 flats and dark: synthesise from exactly those values
    f0 = f0.float().double()
    f1 = f1.float().double()
    dark = dark.float().double()
    kap = torch.tensor([kappa_for(p[r]) for r in range(R)], device=dev, dtype=torch.float64)
    flat_pos = np.array([0.0, float(K - 1)])
    raw = torch.empty(K, R, nb, device=dev, dtype=torch.uint16 if rounding else torch.float64)
    for k in range(K):
        a = k / (K - 1) if K > 1 else 0.0
        fk = (1.0 - a) * f0 + a * f1
        mean = (fk - dark) * torch.exp(-kap[:, None] * p[:, k, :])
        cnt = torch.poisson(mean, generator=g) if noise else mean
        val = dark + cnt
        if rounding:
            raw[k] = torch.clamp(torch.round(val), 0, 65535).to(torch.int32).to(torch.uint16)
        else:
            raw[k] = val
    flats = torch.stack([f0, f1]).float()
    return raw, flats, flat_pos, dark.float(), kap.cpu().numpy()


def poisson_sinogram(p: torch.Tensor, seed: int, photons: float = 1e4, kappa: float | None = None):
    """Photon-counting data: n ~ Poisson(photons exp(-kappa p)), y = -ln(max(n, 1) / photons).

    Returns (y float32 same shape as p, kappa).
    """
    dev = p.device
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    kap = kappa_for(p) if kappa is None else kappa
    n = torch.poisson(photons * torch.exp(-kap * p.double()), generator=g)
    y = -torch.log(torch.clamp(n, min=1.0) / photons)
    return y.float(), kap
