"""Seeded stand-in dictionary for the overlapping-patch prior (the paper's learned basis is not
available): an input like the phantoms, shared by the oracle's tests and the GPU runs."""
from __future__ import annotations

import numpy as np


def dct_dictionary(m: int, extra: int = 0, seed: int = 0) -> np.ndarray:
    """[m*m + extra][m*m]: the m*m separable DCT-II atoms (unit norm, row-major patches) followed by
    `extra` seeded random unit-norm atoms (over-complete when extra > 0)."""
    k = np.arange(m)
    C = np.cos(np.pi * (k[None, :] + 0.5) * k[:, None] / m)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    atoms = np.einsum("ai,bj->abij", C, C).reshape(m * m, m * m)
    if extra:
        R = np.random.default_rng(seed).standard_normal((extra, m * m))
        atoms = np.vstack([atoms, R / np.linalg.norm(R, axis=1, keepdims=True)])
    return atoms
