"""Oracle (test infrastructure only) of the overlapping-patch dictionary prior of
section 3.2: plain FP64 NumPy, written from eqs. (4)-(9), for small images.

Patches.  m x m patches whose top-left corners r_p lie on a grid of step
`stride` along each axis (the last corner is moved to N - m so the patches
cover the image); patch index p = row-corner index * (number of column
corners) + column-corner index.  Centre C_p = r_p + (m - 1)/2.  The core of a
patch (eq. (6)) is the set of pixels whose L1-nearest centre is C_p, ties going
to the lowest patch index; the cores partition the image (eq. (5)).

Unknowns.  W [N_p][N_c]: the coefficients of every patch on the dictionary
D [N_c][m*m] (row k = atom phi_k, row-major over the patch).  The patch
images are X = W D [N_p][m*m]; the solution image x takes every pixel from
its core patch (eq. (7)).

Functional (eq. (8)):
    F(W) = |y - Pi x|^2 + rho sum_p sum_{i in patch p} (x_i - X_p(i - r_p))^2 + beta |W|_1
with Pi the projector A = s^2 B^T (tomography) or the identity (denoising).
Gradient of the smooth part (eq. (9)), with R = Pi^T (Pi x - y) + rho S,
S_i = sum_{p covering i} (x_i - X_p(i - r_p)):
    dF/dW = 2 [core_patches(R) + rho (X - patches(x))] D^T
FISTA (Beck & Teboulle) on W with step 1/L and soft threshold beta/L, from W = 0.
"""
from __future__ import annotations

import math

import numpy as np


def corners(n: int, m: int, stride: int) -> np.ndarray:
    c = list(range(0, n - m + 1, stride))
    if c[-1] != n - m:
        c.append(n - m)
    return np.asarray(c, dtype=np.int64)


class PatchGrid:
    """Patch corners, centres and the core map of an n_y x n_x image."""

    def __init__(self, n_y: int, n_x: int, m: int, stride: int):
        self.n_y, self.n_x, self.m, self.stride = n_y, n_x, m, stride
        self.cy, self.cx = corners(n_y, m, stride), corners(n_x, m, stride)
        self.n_p = len(self.cy) * len(self.cx)
        ry = np.repeat(self.cy, len(self.cx))
        rx = np.tile(self.cx, len(self.cy))
        self.r = np.stack([ry, rx], 1)                      # [N_p][2] corners (row, col)
        cen = self.r + (m - 1) / 2.0
        iy, ix = np.mgrid[0:n_y, 0:n_x]
        # eq. (6): L1-nearest centre, first index on ties (argmin returns the first minimum)
        d = np.abs(iy[..., None] - cen[:, 0]) + np.abs(ix[..., None] - cen[:, 1])
        self.core = np.argmin(d, axis=-1)                   # [n_y][n_x] patch index of each pixel's core

    def patches(self, x: np.ndarray) -> np.ndarray:
        """[N_p][m*m]: the m x m window of x under every patch."""
        m = self.m
        return np.stack([x[ry:ry + m, rx:rx + m].ravel() for ry, rx in self.r])

    def scatter_add(self, P: np.ndarray) -> np.ndarray:
        """Image with sum over patches of P_p placed at the patch (adjoint of patches())."""
        m = self.m
        out = np.zeros((self.n_y, self.n_x))
        for (ry, rx), v in zip(self.r, P):
            out[ry:ry + m, rx:rx + m] += v.reshape(m, m)
        return out

    def assemble(self, X: np.ndarray) -> np.ndarray:
        """eq. (7): every pixel from its core patch's image."""
        m = self.m
        iy, ix = np.mgrid[0:self.n_y, 0:self.n_x]
        p = self.core
        ly, lx = iy - self.r[p, 0], ix - self.r[p, 1]
        return X[p, ly * m + lx]

    def core_patches(self, R: np.ndarray) -> np.ndarray:
        """[N_p][m*m]: R on the core pixels of each patch, 0 on the rest of the patch."""
        m = self.m
        out = np.zeros((self.n_p, m * m))
        for p, (ry, rx) in enumerate(self.r):
            win = R[ry:ry + m, rx:rx + m]
            mask = self.core[ry:ry + m, rx:rx + m] == p
            out[p] = np.where(mask, win, 0.0).ravel()
        return out


class PatchProblem:
    """eq. (8) for one slice.  project / backproject: the projector pair (None = identity)."""

    def __init__(self, grid: PatchGrid, D: np.ndarray, y: np.ndarray, rho: float, beta: float,
                 project=None, backproject=None):
        self.g, self.D, self.y = grid, np.asarray(D, dtype=np.float64), np.asarray(y, dtype=np.float64)
        self.rho, self.beta = rho, beta
        self.P = project or (lambda x: x)
        self.PT = backproject or (lambda r: r)

    def images(self, W):
        X = W @ self.D
        return X, self.g.assemble(X)

    def smooth(self, W) -> float:
        X, x = self.images(W)
        r = self.P(x) - self.y
        sim = self.g.patches(x) - X
        return float(np.sum(r * r) + self.rho * np.sum(sim * sim))

    def energy(self, W) -> float:
        return self.smooth(W) + self.beta * float(np.abs(W).sum())

    def grad(self, W) -> np.ndarray:
        """eq. (9)."""
        X, x = self.images(W)
        S = self.g.scatter_add(self.g.patches(x) - X)       # sum over covering patches of (x_i - X_p)
        R = self.PT(self.P(x) - self.y) + self.rho * S
        G = self.g.core_patches(R) + self.rho * (X - self.g.patches(x))
        return 2.0 * G @ self.D.T

    def lipschitz(self, n_iter: int = 200, seed: int = 0) -> float:
        """Largest eigenvalue of the (linear) gradient map's Hessian by power iteration."""
        y0, self.y = self.y, np.zeros_like(self.y)
        v = np.random.default_rng(seed).standard_normal((self.g.n_p, self.D.shape[0]))
        lam = 0.0
        for _ in range(n_iter):
            v /= np.linalg.norm(v)
            hv = self.grad(v)
            lam = float(np.sum(hv * v))
            v = hv
        self.y = y0
        return lam


def soft(v, t):
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def fista(prob: PatchProblem, n_iter: int, L: float, fast: bool = True, energy: bool = False):
    """ISTA / FISTA on W (step 1/L, shrink beta/L) from W = 0; returns (W, x[, energies])."""
    W = np.zeros((prob.g.n_p, prob.D.shape[0]))
    Z = W.copy()
    t = 1.0
    E = []
    for _ in range(n_iter):
        Wn = soft(Z - prob.grad(Z) / L, prob.beta / L)
        if fast:
            tn = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
            Z = Wn + ((t - 1.0) / tn) * (Wn - W)
            t = tn
        else:
            Z = Wn
        W = Wn
        if energy:
            E.append(prob.energy(W))
    _, x = prob.images(W)
    return (W, x, np.asarray(E)) if energy else (W, x)
