"""MI355X (gfx950) implementation of the differentiable CT projector hot path
of the PYRO-NN update (arXiv 2511.08427): ray-driven forward projection A,
its exact adjoint A^T and the voxel-driven distance-weighted back-projection,
for 2-D parallel/fan and 3-D cone beams given by per-view projection
matrices.  The operators live in libpyronn_mi.so (C ABI, include/pyronn_mi.h);
this package marshals torch tensors into it.
"""
from . import _native
from .geometry import (
    Geometry,
    calibrated_geometry,
    circular_vectors,
    cone_geometry,
    cone_matrices,
    decompose_cone_matrix,
    detector_pose,
    fan_geometry,
    fan_matrices,
    parallel2d_matrices,
    parallel3d_matrices,
    parallel_geometry,
    trajectory_vectors,
)
from .ops import (
    AdjointProjection,
    BackProjection,
    BatchPlan,
    ConeBackProjection3D,
    ConeProjection3D,
    FanBackProjection2D,
    FanProjection2D,
    ParallelBackProjection2D,
    ParallelProjection2D,
    Projection,
    adjoint,
    adjoint_batched,
    adjoint_noalloc,
    backproject,
    backproject_batched,
    backproject_sampled,
    detector_jitter,
    fbp,
    fbp_filter,
    forward,
    forward_batched,
    forward_sampled,
    gantry_blur,
    gaussian_noise_,
    ring_artifacts_,
    splat,
    SplatProjection,
    unrolled_gd,
)

PnError = _native.PnError
LIB_PATH = _native.LIB_PATH


def version() -> str:
    return _native.lib.pn_version().decode()


def release_caches():
    _native.check(_native.lib.pn_release_caches(), "pn_release_caches")
