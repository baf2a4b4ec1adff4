"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This package holds input generation only: random phantoms (ellipses and
ellipsoids, rasterised by sub-pixel averaging), angle sets and measurement
noise.  It contains none of the projector's arithmetic, so that the FP64
oracle and the HIP path can both consume the same inputs without sharing
any code that could hide a common mistake.
"""

from .phantoms import (  # noqa: F401
    SEED_ROOT,
    rng_for,
    ellipse_params,
    rasterize_ellipses,
    ellipse_phantom,
    ellipsoid_params,
    rasterize_ellipsoids,
    ellipsoid_volume,
    add_cracks,
    gaussian_blob,
    uniform_angles,
    sparse_angles,
    limited_view_angles,
    uneven_stack,
    poisson_log_data,
    gaussian_noise,
)
