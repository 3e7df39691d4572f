"""Seeded synthetic inputs for the CT projector workloads.

This module generates what both sides of a parity check consume: random
ellipse/ellipsoid phantoms, smooth analytic balls, random draws that perturb
a trajectory, Poisson count draws, and the named workload configurations
(shapes, spacings, distances, view counts, seeds).  It holds none of the
projector arithmetic: no projection matrices, rays, interpolation or
back-projection.  The FP64 oracle and the GPU path each compose geometry
from the plain parameters given here with their own code.

Conventions used for the rasterised phantoms (world units are mm):
  * the volume array is ``[nz, ny, nx]`` (2-D images are ``[1, ny, nx]``);
  * voxel ``(i, j, k)`` has its centre at ``o + (i*sx, j*sy, k*sz)`` with
    ``o = -((n - 1) / 2) * s`` per axis, i.e. the volume is centred on the
    world origin (the isocentre);
  * phantoms are point-sampled at voxel centres and ellipses are additive.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Ellipsoid",
    "voxel_centres",
    "ellipse_phantom_2d",
    "ellipsoid_phantom_3d",
    "smooth_ball_volume",
    "perturbation_draws",
    "poisson_counts",
    "batched_problem_list",
    "CONFIGS",
]


@dataclass
class Ellipsoid:
    """One additive ellipse (2-D, ``axes`` has 2 entries) or ellipsoid (3-D).

    ``rotation`` maps body coordinates to world coordinates (columns are the
    body axes in world (x, y[, z]) order); ``centre`` and ``axes`` are in mm.
    """

    centre: np.ndarray
    axes: np.ndarray
    rotation: np.ndarray
    density: float


def voxel_centres(shape, spacing, origin=None):
    """World coordinates of voxel centres along each axis.

    ``shape``/``spacing``/``origin`` are in (z, y, x) order; returns the three
    1-D coordinate vectors (z, y, x).  A ``None`` origin centres the grid.
    """
    out = []
    for a in range(3):
        n, s = int(shape[a]), float(spacing[a])
        o = -0.5 * (n - 1) * s if origin is None else float(origin[a])
        out.append(o + s * np.arange(n, dtype=np.float64))
    return out


def _quat_to_matrix(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def _rasterise(shape, spacing, ellipsoids, dim):
    zc, yc, xc = voxel_centres(shape, spacing)
    vol = np.zeros(tuple(int(n) for n in shape), dtype=np.float64)
    for e in ellipsoids:
        # bounding box of the ellipsoid in world coordinates, per axis
        half = np.abs(e.rotation) @ e.axes
        sel = []
        coords = [xc, yc, zc][:dim]
        for a in range(dim):
            lo, hi = e.centre[a] - half[a], e.centre[a] + half[a]
            idx = np.nonzero((coords[a] >= lo) & (coords[a] <= hi))[0]
            sel.append(idx)
        if any(len(ix) == 0 for ix in sel):
            continue
        if dim == 2:
            X, Y = np.meshgrid(xc[sel[0]], yc[sel[1]], indexing="xy")
            rel = np.stack([X - e.centre[0], Y - e.centre[1]], axis=-1)
            body = rel @ e.rotation  # world -> body: R^T r, done row-wise
            inside = (body[..., 0] / e.axes[0]) ** 2 + (body[..., 1] / e.axes[1]) ** 2 <= 1.0
            vol[0, sel[1][0] : sel[1][-1] + 1, sel[0][0] : sel[0][-1] + 1] += e.density * inside
        else:
            Z, Y, X = np.meshgrid(zc[sel[2]], yc[sel[1]], xc[sel[0]], indexing="ij")
            rel = np.stack([X - e.centre[0], Y - e.centre[1], Z - e.centre[2]], axis=-1)
            body = rel @ e.rotation
            q = sum((body[..., a] / e.axes[a]) ** 2 for a in range(3))
            vol[
                sel[2][0] : sel[2][-1] + 1,
                sel[1][0] : sel[1][-1] + 1,
                sel[0][0] : sel[0][-1] + 1,
            ] += e.density * (q <= 1.0)
    return vol


def ellipse_phantom_2d(seed, shape=(64, 64), spacing=(1.0, 1.0), n_ellipses=10):
    """Random additive ellipses on a ``[1, ny, nx]`` grid.

    Per ellipse the draws are, in order: centre ~ U[-0.8, 0.8]^2, semi-axes
    ~ U[0.05, 0.5]^2, angle ~ U[0, pi), density ~ U[0, 1].  Normalised
    coordinates are scaled by the half-extent n*s/2 of each axis.
    Returns ``(image, ellipses)`` with the image in float64.
    """
    ny, nx = int(shape[0]), int(shape[1])
    sy, sx = float(spacing[0]), float(spacing[1])
    half = np.array([nx * sx / 2, ny * sy / 2])
    rng = np.random.default_rng(seed)
    ells = []
    for _ in range(n_ellipses):
        c = rng.uniform(-0.8, 0.8, 2) * half
        ax = rng.uniform(0.05, 0.5, 2) * half
        th = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.0, 1.0)
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        ells.append(Ellipsoid(c, ax, R, float(rho)))
    img = _rasterise((1, ny, nx), (1.0, sy, sx), ells, 2)
    return img, ells


def ellipsoid_phantom_3d(seed, shape=(256, 256, 256), spacing=(0.5, 0.5, 0.5), n_ellipsoids=12):
    """Random additive ellipsoids on a ``[nz, ny, nx]`` grid.

    Per ellipsoid the draws are, in order: centre ~ U[-0.8, 0.8]^3 (x, y, z),
    semi-axes ~ U[0.05, 0.5]^3, rotation = normalised quaternion of four
    N(0, 1) draws, density ~ U[0, 1].  Returns ``(volume, ellipsoids)``.
    """
    nz, ny, nx = (int(n) for n in shape)
    sz, sy, sx = (float(s) for s in spacing)
    half = np.array([nx * sx / 2, ny * sy / 2, nz * sz / 2])
    rng = np.random.default_rng(seed)
    ells = []
    for _ in range(n_ellipsoids):
        c = rng.uniform(-0.8, 0.8, 3) * half
        ax = rng.uniform(0.05, 0.5, 3) * half
        R = _quat_to_matrix(rng.standard_normal(4))
        rho = rng.uniform(0.0, 1.0)
        ells.append(Ellipsoid(c, ax, R, float(rho)))
    vol = _rasterise((nz, ny, nx), (sz, sy, sx), ells, 3)
    return vol, ells


def smooth_ball_volume(shape, spacing, centre_xyz, radius, rho=1.0):
    """Point samples of rho*(1 - r^2/R^2) inside a ball (0 outside).

    ``shape``/``spacing`` in (z, y, x) order, ``centre_xyz`` in world (x, y, z).
    For a 2-D grid pass ``shape=(1, ny, nx)``; the ball is then a disc in
    the z = 0 plane.
    """
    zc, yc, xc = voxel_centres(shape, spacing)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    cx, cy = centre_xyz[0], centre_xyz[1]
    cz = centre_xyz[2] if len(centre_xyz) > 2 else 0.0
    r2 = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2
    return np.where(r2 < radius * radius, rho * (1.0 - r2 / (radius * radius)), 0.0)


def perturbation_draws(seed, n_views, sigma_mm=0.5, sigma_deg=0.5):
    """I.i.d. Gaussian perturbations for a 'perturbed circular' trajectory.

    Returns ``dS`` (n_views, 3) and ``dC`` (n_views, 3) in mm, added to the
    source and detector centre, and ``dphi`` (n_views,) in radians, an
    in-plane rotation of the detector axes.  Draw order: dS, dC, dphi.
    """
    rng = np.random.default_rng(seed)
    dS = rng.normal(0.0, sigma_mm, (n_views, 3))
    dC = rng.normal(0.0, sigma_mm, (n_views, 3))
    dphi = rng.normal(0.0, math.radians(sigma_deg), n_views)
    return {"dS": dS, "dC": dC, "dphi": dphi}


def poisson_counts(rate, seed):
    """Poisson photon counts with the given (non-negative) rate array."""
    rng = np.random.default_rng(seed)
    return rng.poisson(np.asarray(rate, dtype=np.float64)).astype(np.float64)


def batched_problem_list(seed=4, n_problems=32):
    """The uneven batched cone-beam workload: a seeded list of problems.

    Per problem p (draw order: size index, view count, detector index):
    a cubic volume n in {64, 96, ..., 256} with spacing 128/n mm, N_v in
    {90, ..., 720}, a square detector d in {128, 192, ..., 512} with pixel
    512/d mm, SID 750 mm, SDD 1200 mm.  Trajectory kinds cycle perturbed
    circular, helical (pitch 0.5), sinusoidal.  Phantom seed is 400 + p and
    the perturbation seed 500 + p.
    """
    rng = np.random.default_rng(seed)
    sizes = list(range(64, 257, 32))
    dets = list(range(128, 513, 64))
    kinds = ["perturbed", "helical", "sinusoidal"]
    probs = []
    for p in range(n_problems):
        n = sizes[int(rng.integers(0, len(sizes)))]
        nv = int(rng.integers(90, 721))
        d = dets[int(rng.integers(0, len(dets)))]
        probs.append(
            dict(
                vol_shape=(n, n, n),
                vol_spacing=(128.0 / n,) * 3,
                n_views=nv,
                det_shape=(d, d),
                det_spacing=(512.0 / d, 512.0 / d),
                sid=750.0,
                sdd=1200.0,
                angular_range=2 * math.pi,
                trajectory=kinds[p % 3],
                pitch=0.5,
                phantom_seed=400 + p,
                perturb_seed=500 + p,
                n_ellipsoids=12,
            )
        )
    return probs


CONFIGS = {
    # 2-D parallel beam, 64^2 image of 10 ellipses, 90 angles over 180 deg
    "parallel2d_64": dict(
        ndim=2, beam="parallel", batch=1, vol_shape=(1, 64, 64), vol_spacing=(1.0, 1.0, 1.0),
        n_views=90, angular_range=math.pi, det_shape=(1, 95), det_spacing=(1.0, 1.0),
        phantom="ellipses", n_ellipses=10, seeds=[1],
    ),
    # 2-D fan beam, batch of 16 512^2 images, 720 views over 360 deg
    "fan2d_512x16": dict(
        ndim=2, beam="fan", batch=16, vol_shape=(1, 512, 512), vol_spacing=(0.5, 0.5, 0.5),
        n_views=720, angular_range=2 * math.pi, det_shape=(1, 1024), det_spacing=(0.5, 0.5),
        sid=1000.0, sdd=1500.0, phantom="ellipses", n_ellipses=10, seeds=list(range(2, 18)),
        fd_target_seed=18, fd_direction_seed=19,
    ),
    # 3-D circular cone beam, 256^3 volume of 12 ellipsoids, 360 views
    "cone3d_256": dict(
        ndim=3, beam="cone", batch=1, vol_shape=(256, 256, 256), vol_spacing=(0.5, 0.5, 0.5),
        n_views=360, angular_range=2 * math.pi, det_shape=(512, 512), det_spacing=(1.0, 1.0),
        sid=750.0, sdd=1200.0, phantom="ellipsoids", n_ellipsoids=12, seeds=[3],
    ),
    # 3-D cone beam 512^3, 720 views, reduced-precision storage + unrolled loop
    "cone3d_512": dict(
        ndim=3, beam="cone", batch=1, vol_shape=(512, 512, 512), vol_spacing=(0.25, 0.25, 0.25),
        n_views=720, angular_range=2 * math.pi, det_shape=(1024, 1024), det_spacing=(0.5, 0.5),
        sid=750.0, sdd=1200.0, phantom="ellipsoids", n_ellipsoids=12, seeds=[5],
        poisson_seed=55, I0=1e5, unrolled_steps=10,
    ),
}
