"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only *generates* data (phantoms, their exact line integrals and
simulated detector counts).  It holds none of the reconstruction method's
arithmetic: no normalisation, filtering, projection, backprojection or TV.
"""
from .phantom import (  # noqa: F401
    rng_for,
    random_ellipses,
    ellipse_sinogram,
    ellipse_raster,
    disc_params,
    perlin_texture,
)
from .acquisition import (  # noqa: F401
    raw_acquisition,
    poisson_sinogram,
    kappa_for,
)
from .configs import (  # noqa: F401
    uniform_angles,
    cfg_single_slice,
    cfg_batched_raw,
    cfg_tv_sparse,
    cfg_uneven,
    cfg_learned,
)
from .dictionary import dct_dictionary  # noqa: F401,E402
