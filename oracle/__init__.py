"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  The reconstruction library never calls it, and it shares no
code with the GPU path (the two are written independently from the paper's
definitions).  Heavy loops are plain C in ``oracle.c`` (double precision,
OpenMP over independent rows / angles); the small layout logic is numpy.

What each function follows:
  normalize            dark/flat correction with time-interpolated flats and
                       -log (section 2.3 processing pipe; Beer-Lambert)
  angle_weights        quadrature weight of each projection (mid-point rule)
  half_acq_layout      360 degree scan with the axis near a detector border,
                       whose usable detector width is doubled (section 2.1)
  ramp_filter / fbp_filter / fbp
                       filtered backprojection (section 2.3, last paragraph):
                       Ram-Lak kernel, direct convolution
  backproject / forward_project
                       pixel-driven backprojection with linear detector
                       interpolation and its exact transpose (section 2.3)
  grad / div / tv      isotropic TV, eq. (2), Chambolle (2004) discretisation
  tv_prox              ROF proximal map by Chambolle's dual projection
  cp_tv / opnorm       eq. (3) solved by Chambolle-Pock with K = [A; mu grad];
                       |K|_2
  backproject_points   the backprojection at chosen pixels only (checks of
                       full-size images)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

SCAN_180, SCAN_360, SCAN_360_HALF = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, strict IEEE: no -ffast-math)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", "-ffp-contract=off", src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        L.or_normalize.argtypes = [i, i, i, P, i, P, P, P, d, P]
        L.or_normalize_hotspot.argtypes = [i, i, i, P, i, P, P, P, d, d, P]
        L.or_ring_filter.argtypes = [i, i, P, P, i]
        L.or_ramp_filter.argtypes = [i, i, P, P, P]
        L.or_angle_weights.argtypes = [i, P, d, d, P]
        L.or_backproject.argtypes = [i, i, i, i, P, d, P, d, P, P]
        L.or_forward_project.argtypes = [i, i, i, i, P, d, P, d, P, P]
        L.or_grad.argtypes = [i, i, P, P, P]
        L.or_div.argtypes = [i, i, P, P, P]
        L.or_tv.argtypes = [i, i, P]
        L.or_tv.restype = d
        L.or_tv_prox.argtypes = [i, i, P, d, i, P]
        L.or_cp_tv.argtypes = [i, i, i, i, i, P, d, P, d, P, d, i, d, d, P, P]
        L.or_opnorm.argtypes = [i, i, i, i, P, d, P, d, P, i, i, d]
        L.or_fista_tv.argtypes = [i, i, i, i, i, i, P, d, P, d, P, d, i, d, i, P, P]
        L.or_opnorm.restype = d
        L.or_num_threads.restype = i
        IP = ctypes.POINTER(ctypes.c_int)
        L.or_backproject_points.argtypes = [i, i, i, i, P, d, P, d, P, i, IP, IP, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    if a is None:
        return None
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().or_num_threads()


@dataclass
class Geom:
    """Parallel-beam geometry of one slice (section 2.1: angles and axis
    displacement may be given per projection; 180 or 360 degree scans)."""
    n_x: int
    n_y: int
    n_det: int
    angles: np.ndarray
    axis: float
    shifts: np.ndarray | None = None
    scan: int = SCAN_180
    pixel_size: float = 1.0
    ha_overlap: float = 0.0
    K: int = field(init=False)

    def __post_init__(self):
        self.angles = np.ascontiguousarray(self.angles, dtype=np.float64)
        self.K = int(self.angles.shape[0])
        if self.shifts is not None:
            self.shifts = np.ascontiguousarray(self.shifts, dtype=np.float64)


# --------------------------------------------------------------------------- a1
def normalize(raw, flats, flat_pos, dark, eps: float = 1e-6) -> np.ndarray:
    """raw [K][R][nb] (counts), flats [F][R][nb], flat_pos [F], dark [R][nb] -> [R][K][nb] f64."""
    raw, flats, dark = _f64(raw), _f64(flats), _f64(dark)
    fp = _f64(np.asarray(flat_pos))
    K, R, nb = raw.shape
    out = np.empty((R, K, nb))
    lib().or_normalize(K, R, nb, _p(raw), flats.shape[0], _p(flats), _p(fp), _p(dark), eps, _p(out))
    return out


def normalize_hotspot(raw, flats, flat_pos, dark, thr: float, eps: float = 1e-6) -> np.ndarray:
    """normalize() with the hot-spot median filter on the flat-field-corrected transmission:
    a pixel exceeding its 3x3 neighbours' median by more than thr takes that median."""
    raw, flats, dark = _f64(raw), _f64(flats), _f64(dark)
    fp = _f64(np.asarray(flat_pos))
    K, R, nb = raw.shape
    out = np.empty((R, K, nb))
    lib().or_normalize_hotspot(K, R, nb, _p(raw), flats.shape[0], _p(flats), _p(fp), _p(dark), eps, thr, _p(out))
    return out


def ring_filter(sino, width: int, obj=None) -> np.ndarray:
    """Ring-artifact filter of each sinogram [S][K][L] (or [K][L]): subtract the high-pass part
    (signal minus its (2 width + 1)-bin moving average) of the angle-averaged signal of
    sino - obj.  Returns a new array."""
    p = np.array(_f64(sino), copy=True)
    squeeze = p.ndim == 2
    if squeeze:
        p = p[None]
    o = None if obj is None else _f64(obj).reshape(p.shape)
    for i in range(p.shape[0]):
        pi = np.ascontiguousarray(p[i])
        oi = None if o is None else np.ascontiguousarray(o[i])
        lib().or_ring_filter(pi.shape[0], pi.shape[1], _p(pi), _p(oi), int(width))
        p[i] = pi
    return p[0] if squeeze else p


def ring_object(sino, g: Geom, threshold: float) -> np.ndarray:
    """Projection A(x [x > threshold]) of the thresholded FBP of sino [K][L] (the strongly absorbing
    part of the object, removed from the data before the ring filter's average)."""
    x = fbp(sino, g)
    return forward_project(np.where(x > threshold, x, 0.0), g)


# --------------------------------------------------------------------------- weights
def angle_weights(g: Geom) -> np.ndarray:
    """Mid-point quadrature weights; full-detector 360 scans count every line twice (factor 1/2)."""
    span = math.pi if g.scan == SCAN_180 else 2.0 * math.pi
    factor = 0.5 if g.scan == SCAN_360 else 1.0
    w = np.empty(g.K)
    lib().or_angle_weights(g.K, _p(g.angles), span, factor, _p(w))
    return w


def half_acq_layout(g: Geom) -> dict:
    """Extended-row layout of a half-acquisition scan.

    delta = distance of the axis to the nearer detector edge.  Axis near the
    right edge: rows are extended to L = floor(2c) + 1 bins (origin kept).
    Axis near bin 0: o = ceil(nb - 1 - 2c) zero bins are prepended, c' = c + o,
    L = nb + o.  With u oriented so that the measured side is u <= delta, the
    weight is 1 for u <= -d_f, (1 - sin(pi u / (2 d_f)))/2 for |u| <= d_f and
    0 beyond, where d_f = ha_overlap (or delta when 0); w(u) + w(-u) = 1.
    """
    nb, c = g.n_det, g.axis
    if g.scan != SCAN_360_HALF:
        return dict(offset=0, L=nb, axis=c, weights=np.ones(nb))
    if c >= 0.5 * (nb - 1):
        o, L, cx, sgn = 0, int(math.floor(2.0 * c)) + 1, c, 1.0
        delta = nb - 1 - c
    else:
        o = int(math.ceil(nb - 1 - 2.0 * c))
        L, cx, sgn = nb + o, c + o, -1.0
        delta = c
    df = g.ha_overlap if g.ha_overlap > 0 else delta
    u = sgn * (np.arange(L, dtype=np.float64) - cx)
    w = np.where(u <= -df, 1.0, np.where(u >= df, 0.0, 0.0))
    if df > 0:
        mid = np.abs(u) < df
        w = np.where(mid, 0.5 * (1.0 - np.sin(np.pi * u / (2.0 * df))), w)
    else:
        w = np.where(u < 0, 1.0, np.where(u == 0, 0.5, 0.0))
    return dict(offset=o, L=L, axis=cx, weights=w)


# --------------------------------------------------------------------------- a2/a3
def ramp_filter(rows, w) -> np.ndarray:
    """Direct Ram-Lak convolution of each row on [0, L), times its weight."""
    rows = _f64(rows)
    sh = rows.shape
    L = sh[-1]
    r2 = rows.reshape(-1, L)
    w = _f64(np.broadcast_to(np.asarray(w, dtype=np.float64), (r2.shape[0],)).copy())
    out = np.empty_like(r2)
    lib().or_ramp_filter(r2.shape[0], L, _p(r2), _p(w), _p(out))
    return out.reshape(sh)


def fbp_filter(sino, g: Geom) -> np.ndarray:
    """sino [S][K][nb] -> filtered [S][K][L] (half-acquisition weighted and extended first)."""
    sino = _f64(sino)
    if sino.ndim == 2:
        sino = sino[None]
    S, K, nb = sino.shape
    lay = half_acq_layout(g)
    ext = np.zeros((S, K, lay["L"]))
    ext[:, :, lay["offset"]:lay["offset"] + nb] = sino
    ext *= lay["weights"][None, None, :]
    w = angle_weights(g)
    return ramp_filter(ext, np.tile(w, S))


# --------------------------------------------------------------------------- a4-a6
def backproject(sino, g: Geom, extended: bool = False) -> np.ndarray:
    """B = hat-weight backprojection.  sino [S][K][L] -> img [S][n_y][n_x].
    extended=True reads rows in the half-acquisition extended layout."""
    sino = _f64(sino)
    squeeze = sino.ndim == 2
    if squeeze:
        sino = sino[None]
    S, K, L = sino.shape
    axis = half_acq_layout(g)["axis"] if extended else g.axis
    out = np.empty((S, g.n_y, g.n_x))
    for i in range(S):
        si = np.ascontiguousarray(sino[i])
        oi = np.empty((g.n_y, g.n_x))
        lib().or_backproject(g.n_x, g.n_y, K, L, _p(g.angles), axis, _p(g.shifts), g.pixel_size, _p(si), _p(oi))
        out[i] = oi
    return out[0] if squeeze else out


def backproject_points(sino, g: Geom, ix, iy, extended: bool = False) -> np.ndarray:
    """B at the pixels (ix[i], iy[i]) of one slice; sino [K][L]."""
    sino = np.ascontiguousarray(_f64(sino))
    K, L = sino.shape
    axis = half_acq_layout(g)["axis"] if extended else g.axis
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    out = np.empty(ix.shape[0])
    IP = ctypes.POINTER(ctypes.c_int)
    lib().or_backproject_points(g.n_x, g.n_y, K, L, _p(g.angles), axis, _p(g.shifts), g.pixel_size, _p(sino),
                                int(ix.shape[0]), ix.ctypes.data_as(IP), iy.ctypes.data_as(IP), _p(out))
    return out


def forward_project(img, g: Geom) -> np.ndarray:
    """A = s^2 B^T.  img [S][n_y][n_x] -> sino [S][K][n_det]."""
    img = _f64(img)
    squeeze = img.ndim == 2
    if squeeze:
        img = img[None]
    S = img.shape[0]
    out = np.empty((S, g.K, g.n_det))
    for i in range(S):
        ii = np.ascontiguousarray(img[i])
        oi = np.empty((g.K, g.n_det))
        lib().or_forward_project(g.n_x, g.n_y, g.K, g.n_det, _p(g.angles), g.axis, _p(g.shifts), g.pixel_size,
                                 _p(ii), _p(oi))
        out[i] = oi
    return out[0] if squeeze else out


def fbp(sino, g: Geom) -> np.ndarray:
    """Filtered backprojection of line integrals [S][K][nb] -> [S][n_y][n_x] ([K][nb] -> [n_y][n_x])."""
    out = backproject(fbp_filter(sino, g), g, extended=True)
    return out[0] if np.ndim(sino) == 2 else out


def fbp_raw(raw, flats, flat_pos, dark, g: Geom, eps: float = 1e-6) -> np.ndarray:
    """The FBP pipeline from raw radiographs: normalise -> weight/extend -> filter -> backproject."""
    return fbp(normalize(raw, flats, flat_pos, dark, eps), g)


# --------------------------------------------------------------------------- a7-a9
def grad(x):
    x = _f64(x)
    ny, nx = x.shape
    g1, g2 = np.empty_like(x), np.empty_like(x)
    lib().or_grad(ny, nx, _p(x), _p(g1), _p(g2))
    return g1, g2


def div(q1, q2):
    q1, q2 = _f64(q1), _f64(q2)
    ny, nx = q1.shape
    d = np.empty_like(q1)
    lib().or_div(ny, nx, _p(q1), _p(q2), _p(d))
    return d


def tv(x) -> float:
    x = _f64(x)
    return lib().or_tv(x.shape[0], x.shape[1], _p(x))


def tv_prox(g, lam: float, n_inner: int) -> np.ndarray:
    """ROF prox of each slice of g ([n_y][n_x] or [S][n_y][n_x])."""
    g = _f64(g)
    squeeze = g.ndim == 2
    if squeeze:
        g = g[None]
    out = np.empty_like(g)
    for i in range(g.shape[0]):
        gi = np.ascontiguousarray(g[i])
        oi = np.empty_like(gi)
        lib().or_tv_prox(gi.shape[0], gi.shape[1], _p(gi), lam, n_inner, _p(oi))
        out[i] = oi
    return out[0] if squeeze else out


def cp_tv(y, g: Geom | None, lam: float, n_iter: int, op_norm: float, energy: bool = False,
          identity_shape=None, mu: float = 1.0):
    """Chambolle-Pock iterate after n_iter iterations (and the energy trace), K = [A; mu grad],
    tau = sigma = 1/op_norm (op_norm >= |K|).  g=None with identity_shape=(n_y, n_x) replaces A by
    the identity."""
    y = _f64(y)
    E = np.empty(max(n_iter, 1)) if energy else None
    if g is None:
        ny, nx = identity_shape
        x = np.empty((ny, nx))
        lib().or_cp_tv(1, nx, ny, 0, 0, None, 0.0, None, 1.0, _p(y), lam, n_iter, op_norm, mu, _p(x), _p(E))
    else:
        x = np.empty((g.n_y, g.n_x))
        lib().or_cp_tv(0, g.n_x, g.n_y, g.K, g.n_det, _p(g.angles), g.axis, _p(g.shifts), g.pixel_size,
                       _p(y), lam, n_iter, op_norm, mu, _p(x), _p(E))
    return (x, E[:n_iter]) if energy else x


def opnorm(g: Geom, x0, n_iter: int = 200, with_grad: bool = True, mu: float = 1.0) -> float:
    """|[A; mu grad]|_2 (with_grad) or |A|_2 by power iteration from x0."""
    x0 = _f64(x0)
    return lib().or_opnorm(g.n_x, g.n_y, g.K, g.n_det, _p(g.angles), g.axis, _p(g.shifts), g.pixel_size,
                           _p(x0), n_iter, int(bool(with_grad)), float(mu))


def fista_tv(y, g: Geom | None, lam: float, n_iter: int, lipschitz: float, n_inner: int, fast: bool = True,
             energy: bool = False, identity_shape=None):
    """ISTA (fast=False) or FISTA iterate x_{n_iter} for eq. (3), step 1/lipschitz, inner ROF prox of
    n_inner dual iterations (and the energy trace).  g=None with identity_shape replaces A by the identity."""
    y = _f64(y)
    E = np.empty(max(n_iter, 1)) if energy else None
    if g is None:
        ny, nx = identity_shape
        x = np.empty((ny, nx))
        lib().or_fista_tv(int(fast), 1, nx, ny, 0, 0, None, 0.0, None, 1.0, _p(y), lam, n_iter, lipschitz,
                          n_inner, _p(x), _p(E))
    else:
        x = np.empty((g.n_y, g.n_x))
        lib().or_fista_tv(int(fast), 0, g.n_x, g.n_y, g.K, g.n_det, _p(g.angles), g.axis, _p(g.shifts),
                          g.pixel_size, _p(y), lam, n_iter, lipschitz, n_inner, _p(x), _p(E))
    return (x, E[:n_iter]) if energy else x


# --------------------------------------------------------------------------- beta selection (section 3.1)
def drop_angle(g: Geom, k: int) -> Geom:
    """The geometry with projection k removed (the leave-one-angle-out reconstruction)."""
    keep = np.arange(g.K) != k
    return Geom(g.n_x, g.n_y, g.n_det, g.angles[keep], g.axis,
                None if g.shifts is None else g.shifts[keep], g.scan, g.pixel_size, g.ha_overlap)


def cv_error(x, y, g: Geom, k: int) -> float:
    """Cross-validation estimator of section 3.1 for one excluded projection k: the squared distance
    |(A x)_k - y_k|^2 between the projection at angle k of a reconstruction x (made without
    projection k) and the measured row y_k.  x [n_y][n_x]; y [K][n_det] (the full data)."""
    one = Geom(g.n_x, g.n_y, g.n_det, g.angles[k:k + 1], g.axis,
               None if g.shifts is None else g.shifts[k:k + 1], g.scan, g.pixel_size, g.ha_overlap)
    row = forward_project(x, one)[0]
    d = row - _f64(y)[k]
    return float(np.dot(d, d))


def e_cohe(x_beta, x_zero) -> float:
    """Decoherence estimator of section 3.1: the cosine between I(beta) - I(0+) and I(beta)."""
    a = _f64(x_beta).ravel()
    d = a - _f64(x_zero).ravel()
    return float(np.dot(d, a) / (np.linalg.norm(d) * np.linalg.norm(a)))
