"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds *no* arithmetic of the method: it only draws media,
right-hand sides and random-init weights from fixed seeds, describes the
workload configurations, and packs weights into the self-describing blob the
C library reads.  Both sides of every parity check receive the same arrays
from here and compute everything else on their own.

Workloads (the paper's datasets are not available; these synthetic media stand
in for them with the same shapes and value ranges):

* ``bump64``      -- 64^2 interior, 8-cell PML, Gaussian-bump speed, 3 levels.
* ``grf1024``     -- 1024^2 interior, 16-cell PML, Gaussian random field speed
                     in [1.5, 4.5] (stands in for the high-contrast 2D benchmark
                     of Sec. 4.1), 6 levels.
* ``ellipses64``  -- 64 independent 2D problems of uneven side, high-contrast
                     ellipses, 5 levels (batched form).
* ``layered192``  -- 192^3 interior, 12-cell PML, layered medium with a
                     spherical inclusion (stands in for the 3D benchmark of
                     Sec. 4.1), 5 levels.
* ``serve``       -- Poisson request trace over 16 cached media.
"""
from .configs import Config, CONFIGS, level_sides, ext_side
from .media import (medium_bump, medium_grf, medium_ellipses, medium_layered_sphere,
                    omega_for_ppw, point_source, gaussian_source, random_rhs, make_problem)
from .weights import make_weights, pack_blob, weight_names
from .classical import shifted_laplacian
from .workloads import make_batch, serve_media, serve_trace

__all__ = [
    "shifted_laplacian", "make_batch", "serve_media", "serve_trace",
    "Config", "CONFIGS", "level_sides", "ext_side",
    "medium_bump", "medium_grf", "medium_ellipses", "medium_layered_sphere",
    "omega_for_ppw", "point_source", "gaussian_source", "random_rhs", "make_problem",
    "make_weights", "pack_blob", "weight_names",
]
