"""MI355X (gfx950) reconstruction path of PyHST2 (Mirone et al., NIM B):
parallel-beam FBP (normalise + -log, ramp filter, pixel-driven backprojection),
the matched projector pair, the TV-regularised mode (Chambolle-Pock, ISTA,
FISTA) and the estimators for its weight, as hand-written HIP kernels behind
the C ABI of include/pyhst.h.

PyTorch provides device memory and streams only; every step of the path runs
in the HIP library, which must be built (no CPU fallback exists)."""
from ._lib import lib, PyhstError, SCAN_180, SCAN_360, SCAN_360_HALF, FBP, TV_CP, ISTA, FISTA  # noqa: F401
from ._lib import FP_AUTO, FP_BLOCKS, FP_STAGED, FP_LINES  # noqa: F401
from .api import (  # noqa: F401
    Geometry, Plan, pyhst_normalize, normalize, fbp_filter, backproject, forward_project, tv_prox,
    reconstruct_slices, work_bytes, uniform_angles, slice_residual, cv_error, decoherence,
    normalize_hotspot, ring_filter, patch_fista, patch_lipschitz, opnorm, balanced_mu,
)
