"""MI355X-native hot path of majorization-minimization LiDAR bundle adjustment.

Thin Python binding of ``libba`` (the HIP/gfx950 library behind
``include/ba.h``): argument marshalling only.  PyTorch provides device memory
and streams; every step of the path runs in the library's kernels.  The
library must have been built (``python -m paper_2608_14266_amd.build``); this
module raises if it is missing.
"""
from __future__ import annotations

from ._lib import (  # noqa: F401
    MODE_COUPLED,
    MODE_EXACT,
    MODE_MM,
    PREC_F32,
    PREC_F64,
    BAError,
    Problem,
    Server,
    VoxelMap,
    autotune,
    build_clusters,
    build_clusters_from_sums,
    eval_residual_grad_hessian,
    iterate,
    lib_path,
    load,
    profile_enable,
    profile_query,
    profile_reset,
    problem_get_tuning,
    problem_set_tuning,
    request_footprint,
    solve_increment,
    solve_increment_noalloc,
    solve_increment_workspace,
    voxelize,
    voxelize_host,
)
from .tuning import tuned  # noqa: F401,E402
