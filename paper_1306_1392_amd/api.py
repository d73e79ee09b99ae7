"""Python binding of the C ABI: the same entry points, taking torch CUDA tensors as
device buffers.  Every computation runs in the HIP library; this module only
checks shapes and passes pointers and the current stream."""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check, SCAN_180, SCAN_360, SCAN_360_HALF, FBP, TV_CP, ISTA, FISTA  # noqa: F401


@dataclass
class Geometry:
    """Parallel-beam geometry of a slice family (angles in radians, axis in bin coordinates)."""
    n_x: int
    n_y: int
    n_det: int
    angles: np.ndarray
    axis_pos: float
    axis_shift: np.ndarray | None = None
    scan: int = SCAN_180
    pixel_size: float = 1.0
    ha_overlap: float = 0.0

    def __post_init__(self):
        self.angles = np.ascontiguousarray(self.angles, dtype=np.float64)
        if self.axis_shift is not None:
            self.axis_shift = np.ascontiguousarray(self.axis_shift, dtype=np.float64)

    @property
    def n_angles(self) -> int:
        return int(self.angles.shape[0])

    def _c(self) -> _lib.Geom:
        g = _lib.Geom()
        g.n_x, g.n_y, g.n_det, g.n_angles = self.n_x, self.n_y, self.n_det, self.n_angles
        g.angles = self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g.axis_pos = float(self.axis_pos)
        g.axis_shift = (self.axis_shift.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                        if self.axis_shift is not None else None)
        g.scan = int(self.scan)
        g.pixel_size = float(self.pixel_size)
        g.ha_overlap = float(self.ha_overlap)
        return g


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensors only")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Immutable reconstruction plan (FP64 angle tables, weights, filter spectra, work lists)."""

    def __init__(self, geoms, n_slices: int = 1, slice_geom=None):
        if isinstance(geoms, Geometry):
            geoms = [geoms]
        self.geoms = list(geoms)
        arr = (_lib.Geom * len(self.geoms))(*[g._c() for g in self.geoms])
        sg = None
        if slice_geom is not None:
            sg_np = np.ascontiguousarray(slice_geom, dtype=np.int32)
            n_slices = int(sg_np.shape[0])
            sg = sg_np.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.n_slices = int(n_slices)
        self.slice_geom = None if slice_geom is None else np.asarray(slice_geom, dtype=np.int32)
        h = ctypes.c_void_p()
        self._L = _lib.lib()
        check(self._L.pyhst_plan_create(arr, len(self.geoms), sg, self.n_slices, ctypes.byref(h)),
              "pyhst_plan_create")
        self.handle = h
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(self._L.pyhst_plan_sizes(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "pyhst_plan_sizes")
        self.sino_elems, self.filt_elems, self.img_elems = a.value, b.value, c.value
        self.uniform = self.slice_geom is None or len(set(self.slice_geom.tolist())) == 1
        # the geometry every slice of a uniform plan uses (slice_geom may name any one of geoms)
        self.geom0 = self.geoms[int(self.slice_geom[0]) if self.slice_geom is not None else 0]

    def slice_info(self, i: int) -> _lib.SliceInfo:
        si = _lib.SliceInfo()
        check(self._L.pyhst_plan_slice_info(self.handle, i, ctypes.byref(si)), "pyhst_plan_slice_info")
        return si

    def set_tiles(self, bp_tile: int = -1, persistent: bool = False):
        check(self._L.pyhst_plan_set_tiles(self.handle, int(bp_tile), int(bool(persistent))), "pyhst_plan_set_tiles")

    def get_tiles(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(self._L.pyhst_plan_get_tiles(self.handle, ctypes.byref(a), ctypes.byref(b)), "pyhst_plan_get_tiles")
        return a.value, bool(b.value)

    def set_fp_kernel(self, kind: int = 0):
        """Forward-projector kernel: FP_AUTO, FP_BLOCKS, FP_STAGED or FP_LINES."""
        check(self._L.pyhst_plan_set_fp_kernel(self.handle, int(kind)), "pyhst_plan_set_fp_kernel")

    def set_bp_slices(self, per_workgroup: int = 0):
        """Slices per backprojector workgroup: 0 automatic, 1 or 2."""
        check(self._L.pyhst_plan_set_bp_slices(self.handle, int(per_workgroup)), "pyhst_plan_set_bp_slices")

    def get_fp_kernel(self) -> int:
        k = ctypes.c_int32()
        check(self._L.pyhst_plan_get_fp_kernel(self.handle, ctypes.byref(k)), "pyhst_plan_get_fp_kernel")
        return k.value

    # shapes of the packed buffers of a uniform plan
    def sino_shape(self):
        g = self.geom0
        return (self.n_slices, g.n_angles, g.n_det) if self.uniform else (self.sino_elems,)

    def filt_shape(self):
        g = self.geom0
        return (self.n_slices, g.n_angles, self.slice_info(0).filt_len) if self.uniform else (self.filt_elems,)

    def img_shape(self):
        g = self.geom0
        return (self.n_slices, g.n_y, g.n_x) if self.uniform else (self.img_elems,)

    def autotune(self, filt, img, reps: int = 3, stream=None) -> float:
        """Pick the fastest backprojector tile / scheduling for this plan on these buffers."""
        _need(filt, self.filt_elems, "filt")
        _need(img, self.img_elems, "img")
        ms = ctypes.c_float()
        check(self._L.pyhst_plan_autotune(self.handle, _ptr(filt), _ptr(img), int(reps), ctypes.byref(ms),
                                          _stream(stream)), "pyhst_plan_autotune")
        return ms.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._L.pyhst_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _need(t: torch.Tensor, n: int, name: str, dtype=torch.float32):
    if t is None:
        raise ValueError(f"{name}: missing")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")


def _need_raw(plan: Plan, raw, flats, flat_pos, dark, rows: int | None = None):
    """Raw radiographs [K][rows][n_det] uint16, flats [n_flats][rows][n_det] and dark [rows][n_det] float32
    (rows = the plan's slices unless halo rows are given)."""
    g = plan.geom0
    rows = plan.n_slices if rows is None else rows
    nf = int(np.asarray(flat_pos).shape[0])
    _need(raw, g.n_angles * rows * g.n_det, "raw", torch.uint16)
    _need(flats, nf * rows * g.n_det, "flats")
    _need(dark, rows * g.n_det, "dark")


def pyhst_normalize(plan: Plan, raw, flats, flat_pos, dark, eps: float = 1e-6, out=None, stream=None):
    """uint16 radiographs [K][R][nb] -> -log sinograms [R][K][nb]."""
    if out is None:
        out = torch.empty(plan.sino_shape(), device=raw.device, dtype=torch.float32)
    _need(out, plan.sino_elems, "sino")
    _need_raw(plan, raw, flats, flat_pos, dark)
    fp = np.ascontiguousarray(flat_pos, dtype=np.float64)
    check(_lib.lib().pyhst_normalize(plan.handle, _ptr(raw), _ptr(flats),
                                     fp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(fp.shape[0]),
                                     _ptr(dark), float(eps), _ptr(out), _stream(stream)), "pyhst_normalize")
    return out


normalize = pyhst_normalize


def fbp_filter(plan: Plan, sino, out=None, stream=None):
    if out is None:
        out = torch.empty(plan.filt_shape(), device=sino.device, dtype=torch.float32)
    _need(sino, plan.sino_elems, "sino")
    _need(out, plan.filt_elems, "filt")
    check(_lib.lib().fbp_filter(plan.handle, _ptr(sino), _ptr(out), _stream(stream)), "fbp_filter")
    return out


def backproject(plan: Plan, sino, filtered_layout: int = 0, out=None, alpha: float = 1.0, beta: float = 0.0,
                stream=None):
    if out is None:
        out = torch.empty(plan.img_shape(), device=sino.device, dtype=torch.float32)
    _need(sino, plan.filt_elems if filtered_layout else plan.sino_elems, "sino")
    _need(out, plan.img_elems, "img")
    check(_lib.lib().backproject(plan.handle, _ptr(sino), int(filtered_layout), _ptr(out), float(alpha), float(beta),
                                 _stream(stream)), "backproject")
    return out


def forward_project(plan: Plan, img, out=None, alpha: float = 1.0, stream=None):
    """sino = alpha * A img (alpha = 1/s^2 gives B^T, the adjoint of backproject)."""
    if out is None:
        out = torch.empty(plan.sino_shape(), device=img.device, dtype=torch.float32)
    _need(img, plan.img_elems, "img")
    _need(out, plan.sino_elems, "sino")
    check(_lib.lib().forward_project(plan.handle, _ptr(img), _ptr(out), float(alpha), _stream(stream)),
          "forward_project")
    return out


def opnorm(plan: Plan, with_grad: bool, mu: float = 1.0, stream=None) -> float:
    """|[A; mu grad]| (with_grad) or |A| of the plan's batch by power iteration (x 1.02), the op_norm the
    iterative methods take.  Synchronises the stream."""
    L = _lib.lib()
    nb = ctypes.c_size_t()
    check(L.pyhst_opnorm(plan.handle, int(bool(with_grad)), float(mu), None, ctypes.byref(nb), None,
                         _stream(stream)), "pyhst_opnorm(query)")
    work = torch.empty(max(nb.value, 1), device="cuda", dtype=torch.uint8)
    nb.value = work.numel()
    v = ctypes.c_double()
    check(L.pyhst_opnorm(plan.handle, int(bool(with_grad)), float(mu), _ptr(work), ctypes.byref(nb), ctypes.byref(v),
                         _stream(stream)), "pyhst_opnorm")
    return v.value


def balanced_mu(plan: Plan, stream=None) -> float:
    """mu = |A| / |grad| with |grad| = 2 sqrt(2) (its bound on any image): the gradient-block scale that
    balances Chambolle-Pock's two dual blocks."""
    return opnorm(plan, False, stream=stream) / 1.02 / (2.0 * math.sqrt(2.0))


def tv_prox(x, lam: float, n_inner: int, out=None, work=None, stream=None):
    """ROF prox of each slice of x ([S][ny][nx] or [ny][nx])."""
    xs = x if x.dim() == 3 else x[None]
    S, ny, nx = xs.shape
    if out is None:
        out = torch.empty_like(x)
    _need(x, S * ny * nx, "x")
    _need(out, S * ny * nx, "out")
    if work is None:
        work = torch.empty(4 * S * ny * nx, device=x.device, dtype=torch.float32)
    _need(work, work.numel(), "work")
    check(_lib.lib().tv_prox(S, ny, nx, _ptr(x), _ptr(out), float(lam), int(n_inner), _ptr(work), work.numel(),
                             _stream(stream)), "tv_prox")
    return out


def _set_pre(a, hot_threshold, ring_width, ring_object_threshold):
    """Optional preprocessing (section 2.3): hot-spot filter threshold (None = off), ring filter half-width
    (0 = off) and the threshold of the object removed before the ring filter's average (None = off)."""
    a.hot_spot = int(hot_threshold is not None)
    a.hot_threshold = float(hot_threshold) if hot_threshold is not None else 0.0
    a.ring_width = int(ring_width)
    a.ring_object = int(ring_object_threshold is not None)
    a.ring_threshold = float(ring_object_threshold) if ring_object_threshold is not None else 0.0


def normalize_hotspot(plan: Plan, raw, flats, flat_pos, dark, threshold: float, eps: float = 1e-6, out=None,
                      halo=(0, 0), stream=None):
    """normalize() with the hot-spot median filter (section 2.3) on the flat-field-corrected data.
    halo = (rows before, rows after) present in raw/flats/dark only as neighbours (0 or 1 each)."""
    h0, h1 = int(halo[0]), int(halo[1])
    _need_raw(plan, raw, flats, flat_pos, dark, plan.n_slices + h0 + h1)
    fp = np.ascontiguousarray(flat_pos, dtype=np.float64)
    if out is None:
        out = torch.empty(plan.sino_shape(), device=raw.device, dtype=torch.float32)
    _need(out, plan.sino_elems, "out")
    check(_lib.lib().pyhst_normalize_hotspot(plan.handle, _ptr(raw), _ptr(flats),
                                             fp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(fp.shape[0]),
                                             _ptr(dark), float(eps), float(threshold), h0, h1, _ptr(out),
                                             _stream(stream)),
          "pyhst_normalize_hotspot")
    return out


def ring_filter(plan: Plan, sino, width: int, obj=None, work=None, stream=None):
    """Ring-artifact filter (section 2.3) of the sinograms, in place; returns sino."""
    _need(sino, plan.sino_elems, "sino")
    if obj is not None:
        _need(obj, plan.sino_elems, "obj")
    n = 2 * plan.n_slices * plan.geom0.n_det
    if work is None:
        work = torch.empty(n, device=sino.device, dtype=torch.float64)
    check(_lib.lib().pyhst_ring_filter(plan.handle, _ptr(sino), int(width), _ptr(obj), _ptr(work), work.numel(),
                                       _stream(stream)), "pyhst_ring_filter")
    return sino


def reconstruct_slices(plan: Plan, *, raw=None, sino=None, flats=None, flat_pos=None, dark=None, eps: float = 1e-6,
                       method: int = FBP, lam: float = 0.0, n_iter: int = 0, op_norm: float = 0.0,
                       n_inner: int = 20, energy: bool = False, out=None, work=None, use_graph: bool = False,
                       hot_threshold: float | None = None, ring_width: int = 0,
                       ring_object_threshold: float | None = None, tv_mu: float = 1.0, halo=(0, 0), stream=None,
                       no_alloc: bool = False):
    """Returns out (and the energy trace as a numpy array when energy=True).  op_norm is |[A; tv_mu grad]| for
    TV_CP and |A| for ISTA/FISTA; <= 0: computed first by opnorm() (a separate, synchronising call), then
    available as plan.last_op_norm.  halo: raw rows before / after the plan's (hot-spot filter only).
    no_alloc: call reconstruct_slices_static (scratch from the library's per-device array, at most
    PYHST_STATIC_SCRATCH_BYTES; work and use_graph are not used)."""
    iterative = method in (TV_CP, ISTA, FISTA)
    if raw is not None:
        if flat_pos is None:
            raise ValueError("raw input needs flat_pos")
        _need_raw(plan, raw, flats, flat_pos, dark, plan.n_slices + int(halo[0]) + int(halo[1]))
    if sino is not None:
        _need(sino, plan.sino_elems, "sino")
    if iterative and not op_norm > 0.0:
        op_norm = opnorm(plan, method == TV_CP, tv_mu, stream=stream)
    a = _lib.ReconArgs()
    a.raw = _ptr(raw)
    a.sino = _ptr(sino)
    a.flats = _ptr(flats)
    fp = None
    if flat_pos is not None:
        fp = np.ascontiguousarray(flat_pos, dtype=np.float64)
        a.flat_pos = fp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        a.n_flats = int(fp.shape[0])
    a.dark = _ptr(dark)
    a.eps = float(eps)
    a.method = int(method)
    a.lambda_ = float(lam)
    a.n_iter = int(n_iter)
    a.op_norm = float(op_norm)
    a.tv_mu = float(tv_mu)
    a.use_graph = int(bool(use_graph))
    a.n_inner = int(n_inner)
    a.hot_halo_lo, a.hot_halo_hi = int(halo[0]), int(halo[1])
    _set_pre(a, hot_threshold, ring_width, ring_object_threshold)
    dev = (raw if raw is not None else sino).device
    E = None
    if energy and iterative:
        E = torch.zeros(max(n_iter, 1), device=dev, dtype=torch.float32)
        a.energy = _ptr(E)
    L = _lib.lib()
    if no_alloc:
        if out is None:
            out = torch.empty(plan.img_shape(), device=dev, dtype=torch.float32)
        _need(out, plan.img_elems, "out")
        a.out = _ptr(out)
        check(L.reconstruct_slices_static(plan.handle, ctypes.byref(a), _stream(stream)), "reconstruct_slices_static")
        return _finish(plan, a, out, E, energy, n_iter, stream)
    # size query
    a.out = None
    check(L.reconstruct_slices(plan.handle, ctypes.byref(a), _stream(stream)), "reconstruct_slices(query)")
    need = a.work_bytes
    if work is None or work.numel() * work.element_size() < need:
        work = torch.empty(max(need, 1), device=dev, dtype=torch.uint8)
    if out is None:
        out = torch.empty(plan.img_shape(), device=dev, dtype=torch.float32)
    _need(out, plan.img_elems, "out")
    a.out = _ptr(out)
    a.work = _ptr(work)
    a.work_bytes = work.numel() * work.element_size()
    check(L.reconstruct_slices(plan.handle, ctypes.byref(a), _stream(stream)), "reconstruct_slices")
    return _finish(plan, a, out, E, energy, n_iter, stream)


def _finish(plan, a, out, E, energy, n_iter, stream):
    plan.last_op_norm = a.op_norm
    if not energy:
        return out
    if E is None:
        return out, np.zeros(0, dtype=np.float32)
    (torch.cuda.current_stream() if stream is None else stream).synchronize()
    e = E[:n_iter].cpu().numpy()
    if not np.all(np.isfinite(e)):
        raise FloatingPointError("reconstruct_slices: non-finite energy")
    return out, e


def slice_residual(plan: Plan, ax, y, out=None, stream=None):
    """|ax - y| / |y| per slice (device float [n_slices])."""
    _need(ax, plan.sino_elems, "ax")
    _need(y, plan.sino_elems, "y")
    if out is None:
        out = torch.empty(plan.n_slices, device=ax.device, dtype=torch.float32)
    check(_lib.lib().pyhst_slice_residual(plan.handle, _ptr(ax), _ptr(y), _ptr(out), _stream(stream)),
          "pyhst_slice_residual")
    return out


def cv_error(plan: Plan, x, y, k: int, row=None, out=None, weight: float = 1.0, accumulate: bool = False,
             stream=None):
    """Cross-validation estimator weight * |(A x)_k - y_k|^2 per slice (device float [n_slices]), added to
    out when accumulate; plan is the full-data plan, x a reconstruction made without projection k."""
    _need(x, plan.img_elems, "x")
    _need(y, plan.sino_elems, "y")
    nb = plan.geom0.n_det
    if row is None:
        row = torch.empty(plan.n_slices * nb, device=x.device, dtype=torch.float32)
    _need(row, plan.n_slices * nb, "row")
    if out is None:
        if accumulate:
            raise ValueError("cv_error: accumulate needs out")
        out = torch.empty(plan.n_slices, device=x.device, dtype=torch.float32)
    _need(out, plan.n_slices, "out")
    check(_lib.lib().pyhst_cv_error(plan.handle, _ptr(x), _ptr(y), int(k), _ptr(row), _ptr(out), float(weight),
                                    int(bool(accumulate)), _stream(stream)), "pyhst_cv_error")
    return out


def decoherence(plan: Plan, x_beta, x_zero, out=None, stream=None):
    """Decoherence estimator cos(x_beta - x_zero, x_beta) per slice (device float [n_slices])."""
    _need(x_beta, plan.img_elems, "x_beta")
    _need(x_zero, plan.img_elems, "x_zero")
    if out is None:
        out = torch.empty(plan.n_slices, device=x_beta.device, dtype=torch.float32)
    check(_lib.lib().pyhst_decoherence(plan.handle, _ptr(x_beta), _ptr(x_zero), _ptr(out), _stream(stream)),
          "pyhst_decoherence")
    return out


def _patch_args(plan: Plan, y, dictionary, m, stride, rho, beta, n_iter, fast, identity, lipschitz):
    if y is not None:
        _need(y, plan.img_elems if identity else plan.sino_elems, "y")
    if dictionary.dtype != torch.float32 or not dictionary.is_contiguous() or dictionary.dim() != 2 \
            or dictionary.shape[1] != m * m:
        raise ValueError("dictionary must be a contiguous float32 [n_atoms][m*m] tensor")
    a = _lib.PatchArgs()
    a.y, a.dict = _ptr(y), _ptr(dictionary)
    a.m, a.stride, a.n_atoms = int(m), int(stride), int(dictionary.shape[0])
    a.rho, a.beta, a.n_iter, a.fast, a.identity = float(rho), float(beta), int(n_iter), int(fast), int(identity)
    a.lipschitz = float(lipschitz)
    a.w = None
    check(_lib.lib().pyhst_patch_fista(plan.handle, ctypes.byref(a), None), "pyhst_patch_fista(query)")
    return a


def patch_lipschitz(plan: Plan, dictionary, m: int, stride: int, rho: float, identity: bool = False,
                    stream=None) -> float:
    """Lipschitz constant (x 1.02) of eq. (9)'s gradient map by power iteration; synchronises the stream."""
    a = _patch_args(plan, None, dictionary, m, stride, rho, 0.0, 0, True, identity, 0.0)
    work = torch.empty(max(a.work_bytes, 1), device=dictionary.device, dtype=torch.uint8)
    a.work, a.work_bytes = _ptr(work), work.numel()
    check(_lib.lib().pyhst_patch_lipschitz(plan.handle, ctypes.byref(a), _stream(stream)), "pyhst_patch_lipschitz")
    return a.lipschitz


def patch_fista(plan: Plan, y, dictionary, m: int, stride: int, rho: float, beta: float, n_iter: int,
                fast: bool = True, identity: bool = False, lipschitz: float = 0.0, energy: bool = False,
                out=None, w=None, work=None, stream=None):
    """Overlapping-patch dictionary prior (section 3.2) by ISTA/FISTA on the patch coefficients.
    y: sinograms (or images when identity=True); dictionary [n_atoms][m*m] float32 on the device.
    Returns (image, coefficients [n_slices][n_patches][n_atoms]) and the energy trace when asked;
    lipschitz <= 0: estimated first by patch_lipschitz() (a separate, synchronising call); the value used
    is left in plan.last_lipschitz."""
    if not lipschitz > 0.0:
        lipschitz = patch_lipschitz(plan, dictionary, m, stride, rho, identity, stream=stream)
    a = _patch_args(plan, y, dictionary, m, stride, rho, beta, n_iter, fast, identity, lipschitz)
    dev = y.device
    if work is None or work.numel() < a.work_bytes:
        work = torch.empty(max(a.work_bytes, 1), device=dev, dtype=torch.uint8)
    W = torch.empty((plan.n_slices, a.n_patches, a.n_atoms), device=dev, dtype=torch.float32) if w is None else w
    _need(W, plan.n_slices * a.n_patches * a.n_atoms, "w")
    out = torch.empty(plan.img_shape(), device=dev, dtype=torch.float32) if out is None else out
    _need(out, plan.img_elems, "out")
    E = None
    if energy:
        E = torch.zeros(max(n_iter, 1), device=dev, dtype=torch.float32)
        a.energy = _ptr(E)
    a.w, a.out, a.work, a.work_bytes = _ptr(W), _ptr(out), _ptr(work), work.numel()
    check(_lib.lib().pyhst_patch_fista(plan.handle, ctypes.byref(a), _stream(stream)), "pyhst_patch_fista")
    plan.last_lipschitz = a.lipschitz
    if not energy:
        return out, W
    (torch.cuda.current_stream() if stream is None else stream).synchronize()
    e = E[:n_iter].cpu().numpy()
    if not np.all(np.isfinite(e)):
        raise FloatingPointError("patch_fista: non-finite energy")
    return out, W, e


def work_bytes(plan: Plan, **kw) -> int:
    a = _lib.ReconArgs()
    a.raw = _ptr(kw.get("raw"))
    a.sino = _ptr(kw.get("sino"))
    a.method = int(kw.get("method", FBP))
    a.n_iter = int(kw.get("n_iter", 0))
    if kw.get("energy"):
        a.energy = ctypes.c_void_p(1)   # only its presence matters to the size query
    _set_pre(a, kw.get("hot_threshold"), kw.get("ring_width", 0), kw.get("ring_object_threshold"))
    a.out = None
    check(_lib.lib().reconstruct_slices(plan.handle, ctypes.byref(a), None), "reconstruct_slices(query)")
    return a.work_bytes


def uniform_angles(K: int, span: float = math.pi) -> np.ndarray:
    return np.arange(K, dtype=np.float64) * (span / K)
