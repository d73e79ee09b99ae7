"""ctypes declarations of the C ABI in include/pyhst.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpyhst.so")

c_int32, c_int64, c_double, c_float, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                         ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t)

OK, EARG, EGEOM, ENOMEM, EHIP, ENUM = 0, -1, -2, -3, -4, -5
SCAN_180, SCAN_360, SCAN_360_HALF = 0, 1, 2
FBP, TV_CP, ISTA, FISTA = 0, 1, 2, 3
FP_AUTO, FP_BLOCKS, FP_STAGED, FP_LINES = 0, 1, 2, 3

EXPORTS = ["pyhst_plan_create", "pyhst_plan_destroy", "pyhst_plan_slice_info", "pyhst_plan_sizes",
           "pyhst_plan_set_tiles", "pyhst_plan_get_tiles", "pyhst_plan_set_fp_kernel", "pyhst_plan_get_fp_kernel", "pyhst_plan_set_bp_slices", "pyhst_normalize", "fbp_filter", "backproject",
           "forward_project", "tv_prox", "reconstruct_slices", "pyhst_microbench", "pyhst_strerror",
           "pyhst_last_error", "pyhst_unet_create", "pyhst_unet_destroy", "pyhst_unet_num_params",
           "pyhst_unet_set_params", "pyhst_unet_get_params", "pyhst_unet_get_grads", "pyhst_unet_forward",
           "pyhst_unet_backward", "pyhst_unet_adam", "pyhst_unet_train_step", "pyhst_plan_autotune", "pyhst_slice_residual", "pyhst_unet_tensor",
           "pyhst_cv_error", "pyhst_decoherence", "pyhst_normalize_hotspot", "pyhst_ring_filter",
           "pyhst_patch_fista", "pyhst_patch_lipschitz", "pyhst_opnorm", "pyhst_unet_set_scale",
           "pyhst_unet_get_scale", "reconstruct_slices_static"]


class Geom(ctypes.Structure):
    _fields_ = [("n_x", c_int32), ("n_y", c_int32), ("n_det", c_int32), ("n_angles", c_int32),
                ("angles", ctypes.POINTER(c_double)), ("axis_pos", c_double),
                ("axis_shift", ctypes.POINTER(c_double)), ("scan", c_int32), ("pixel_size", c_double),
                ("ha_overlap", c_double)]


class SliceInfo(ctypes.Structure):
    _fields_ = [("n_x", c_int32), ("n_y", c_int32), ("n_det", c_int32), ("n_angles", c_int32),
                ("filt_len", c_int32), ("filt_pad", c_int32), ("filt_axis", c_double),
                ("sino_offset", c_int64), ("filt_offset", c_int64), ("img_offset", c_int64)]


class ReconArgs(ctypes.Structure):
    _fields_ = [("raw", c_void_p), ("sino", c_void_p), ("flats", c_void_p), ("flat_pos", ctypes.POINTER(c_double)),
                ("n_flats", c_int32), ("dark", c_void_p), ("eps", c_float), ("method", c_int32),
                ("lambda_", c_float), ("n_iter", c_int32), ("op_norm", c_double),
                ("energy", c_void_p), ("out", c_void_p), ("work", c_void_p),
                ("work_bytes", c_size_t), ("use_graph", c_int32), ("n_inner", c_int32),
                ("hot_spot", c_int32), ("hot_threshold", c_float), ("ring_width", c_int32),
                ("ring_object", c_int32), ("ring_threshold", c_float), ("tv_mu", c_double),
                ("hot_halo_lo", c_int32), ("hot_halo_hi", c_int32)]


class PatchArgs(ctypes.Structure):
    _fields_ = [("y", c_void_p), ("dict", c_void_p), ("m", c_int32), ("stride", c_int32), ("n_atoms", c_int32),
                ("rho", c_float), ("beta", c_float), ("n_iter", c_int32), ("fast", c_int32), ("identity", c_int32),
                ("lipschitz", c_double), ("w", c_void_p), ("out", c_void_p), ("energy", c_void_p),
                ("work", c_void_p), ("work_bytes", c_size_t), ("n_patches", c_int32)]


_lib = None


def lib(path: str = LIB_PATH):
    """Load libpyhst.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    P = c_void_p
    L.pyhst_plan_create.argtypes = [ctypes.POINTER(Geom), c_int32, ctypes.POINTER(c_int32), c_int32,
                                    ctypes.POINTER(c_void_p)]
    L.pyhst_plan_destroy.argtypes = [P]
    L.pyhst_plan_slice_info.argtypes = [P, c_int32, ctypes.POINTER(SliceInfo)]
    L.pyhst_plan_sizes.argtypes = [P, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)]
    L.pyhst_plan_set_tiles.argtypes = [P, c_int32, c_int32]
    L.pyhst_plan_get_tiles.argtypes = [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]
    L.pyhst_plan_set_fp_kernel.argtypes = [P, c_int32]
    L.pyhst_plan_get_fp_kernel.argtypes = [P, ctypes.POINTER(c_int32)]
    L.pyhst_plan_set_bp_slices.argtypes = [P, c_int32]
    L.pyhst_normalize.argtypes = [P, P, P, ctypes.POINTER(c_double), c_int32, P, c_float, P, P]
    L.fbp_filter.argtypes = [P, P, P, P]
    L.backproject.argtypes = [P, P, c_int32, P, c_float, c_float, P]
    L.forward_project.argtypes = [P, P, P, c_float, P]
    L.tv_prox.argtypes = [c_int32, c_int32, c_int32, P, P, c_float, c_int32, P, c_size_t, P]
    L.reconstruct_slices.argtypes = [P, ctypes.POINTER(ReconArgs), P]
    L.reconstruct_slices_static.argtypes = [P, ctypes.POINTER(ReconArgs), P]
    L.pyhst_microbench.argtypes = [c_int32, c_int32, c_int32, P, P]
    L.pyhst_unet_create.argtypes = [c_int32, c_int32, c_int32, c_int32, c_int32, ctypes.POINTER(c_void_p)]
    L.pyhst_unet_destroy.argtypes = [P]
    L.pyhst_unet_num_params.argtypes = [P, ctypes.POINTER(c_int64)]
    L.pyhst_unet_set_params.argtypes = [P, P, P]
    L.pyhst_unet_get_params.argtypes = [P, P, P]
    L.pyhst_unet_get_grads.argtypes = [P, P, P]
    L.pyhst_unet_forward.argtypes = [P, P, c_int32, P, P]
    L.pyhst_unet_backward.argtypes = [P, P, P, c_int32, P, P]
    L.pyhst_unet_adam.argtypes = [P, c_float, c_float, c_float, c_float, P]
    L.pyhst_unet_train_step.argtypes = [P, P, P, c_int32, c_float, P, P]
    L.pyhst_plan_autotune.argtypes = [P, P, P, c_int32, ctypes.POINTER(c_float), P]
    L.pyhst_slice_residual.argtypes = [P, P, P, P, P]
    L.pyhst_cv_error.argtypes = [P, P, P, c_int32, P, P, c_float, c_int32, P]
    L.pyhst_normalize_hotspot.argtypes = [P, P, P, ctypes.POINTER(c_double), c_int32, P, c_float, c_float, c_int32,
                                          c_int32, P, P]
    L.pyhst_ring_filter.argtypes = [P, P, c_int32, P, P, c_size_t, P]
    L.pyhst_patch_fista.argtypes = [P, ctypes.POINTER(PatchArgs), P]
    L.pyhst_patch_lipschitz.argtypes = [P, ctypes.POINTER(PatchArgs), P]
    L.pyhst_opnorm.argtypes = [P, c_int32, c_double, P, ctypes.POINTER(c_size_t), ctypes.POINTER(c_double), P]
    L.pyhst_unet_set_scale.argtypes = [P, c_float]
    L.pyhst_unet_get_scale.argtypes = [P, ctypes.POINTER(c_float)]
    L.pyhst_decoherence.argtypes = [P, P, P, P, P]
    L.pyhst_unet_tensor.argtypes = [P, c_int32, c_int32, c_int32, P, c_int64, P]
    L.pyhst_strerror.argtypes = [c_int32]
    L.pyhst_strerror.restype = ctypes.c_char_p
    L.pyhst_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("pyhst_strerror", "pyhst_last_error"):
            getattr(L, name).restype = c_int32
    _lib = L
    return L


class PyhstError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        msg = L.pyhst_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.pyhst_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def check(code: int, where: str):
    if code != OK:
        raise PyhstError(code, where)
