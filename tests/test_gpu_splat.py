"""GPU parity of the splat projector pn_splat (the transpose of the
voxel-driven back-projection) against the FP64 oracle, its transposition
against pn_backproject, the autograd pair it completes, and its behaviour
for reduced-precision storage, high dynamic range and non-finite input.
The kernel adds per-block partial sums to the sinogram with float atomics,
so results are compared within FP32 rounding, not bitwise.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from test_gpu_parity import make_case

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = 1e-2


def _say(msg):
    print(f"[gpu-splat] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_08427_amd as pn

    return pn


def rel(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    return float(np.linalg.norm((g - o).ravel()) / max(np.linalg.norm(o.ravel()), 1e-300))


def f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


CASES = ["parallel2d_64", "fan2d_ragged", "cone3d_ragged", "cone3d_anisotropic", "cone3d_perturbed",
         "cone3d_helical", "cone3d_parallel_beam", "cone3d_long_x"]


@pytest.mark.parametrize("name", CASES)
def test_splat_matches_oracle(pn, name):
    _say(f"case {name}")
    gp, go, vols = make_case(pn, name)
    x = f32(np.stack(vols))
    y = pn.splat(torch.from_numpy(x).float().cuda(), gp)
    torch.cuda.synchronize()
    g = y.double().cpu().numpy()
    for b in range(x.shape[0]):
        ref = O.splat(x[b], go)
        assert rel(g[b], ref) <= TOL32, (name, b, rel(g[b], ref))


@pytest.mark.parametrize("name", ["fan2d_ragged", "cone3d_ragged", "cone3d_perturbed"])
def test_splat_is_the_transpose_of_backproject_gpu(pn, name):
    """<pn_backproject(q), x> = <q, pn_splat(x)> with FP64 host sums."""
    _say(f"dot {name}")
    gp, go, vols = make_case(pn, name)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(gp.vol_shape).astype(np.float32)
    q = rng.standard_normal(gp.sino_shape()).astype(np.float32)
    bq = pn.backproject(torch.from_numpy(q).cuda(), gp).double().cpu().numpy()
    sx = pn.splat(torch.from_numpy(x).cuda(), gp).double().cpu().numpy()
    lhs, rhs = float(np.sum(bq * x)), float(np.sum(q * sx))
    scale = np.linalg.norm(bq) * np.linalg.norm(x)
    assert abs(lhs - rhs) <= 1e-5 * scale, (lhs, rhs)


@pytest.mark.parametrize("pix,sid,sdd,shp,det,tol", [
    # 16^3 blocks project into 19-30 detector columns: some views' rectangles
    # fit the LDS accumulator, the others deposit with float atomics
    (0.65, 750.0, 1200.0, (32, 48, 48), (80, 100), TOL32),
    # magnification 4: nearly every rectangle is too large for the LDS.  A
    # voxel spans 8 pixels, so a pixel takes few taps per view and the FP32
    # rounding of the tap positions does not average out: rounding the
    # projection matrices alone (relative 2^-24) moves the FP64 oracle's
    # result by 6-7e-6 here, and evaluating them in FP32 adds as much again
    (0.5, 120.0, 480.0, (20, 30, 36), (120, 150), 3 * TOL32),
])
def test_splat_lds_and_direct_deposits(pn, pix, sid, sdd, shp, det, tol):
    """Blocks whose detector rectangle exceeds the LDS accumulator take the
    straight float-atomic path; both paths in one call match the oracle and
    the transpose of pn_backproject."""
    _say(f"rectangles pix={pix} sid={sid}")
    sp = (0.5, 0.5, 0.5) if sid > 500 else (1.0, 1.0, 1.0)
    gp = pn.cone_geometry(shp, sp, det, (pix, pix), 24, sid, sdd)
    go = O.circular_cone(shp, sp, det, (pix, pix), 24, 2 * math.pi, sid, sdd)
    rng = np.random.default_rng(12)
    x = f32(W.ellipsoid_phantom_3d(8, shp, sp)[0] + 0.1 * rng.random(shp))
    y = pn.splat(torch.from_numpy(x).float().cuda(), gp).double().cpu().numpy()
    assert rel(y, O.splat(x, go)) <= tol
    q = rng.standard_normal(gp.sino_shape()).astype(np.float32)
    bq = pn.backproject(torch.from_numpy(q).cuda(), gp).double().cpu().numpy()
    lhs, rhs = float(np.sum(bq * x)), float(np.sum(q * y))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(bq) * np.linalg.norm(x), (lhs, rhs)


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
def test_splat_reduced_precision_storage(pn, dt):
    gp, go, vols = make_case(pn, "cone3d_ragged")
    xs = torch.from_numpy(vols[0]).to(dt).cuda()
    ref = O.splat(xs.double().cpu().numpy(), go)
    assert rel(pn.splat(xs, gp).double().cpu().numpy(), ref) <= TOL16
    y32 = pn.splat(xs, gp, out_dtype=torch.float32)
    assert y32.dtype == torch.float32 and rel(y32.double().cpu().numpy(), ref) <= TOL32


def test_splat_high_dynamic_range_and_batch(pn):
    """Hot voxels 1e5 times the rest, and batch items 1e4 apart: each block
    takes its own fixed-point scale."""
    gp, go, vols = make_case(pn, "cone3d_ragged")
    v = vols[0].copy()
    rng = np.random.default_rng(9)
    idx = rng.choice(np.flatnonzero(v > 0.1), 15, replace=False)
    v.flat[idx] *= 1e5
    x = f32(np.stack([v, 1e-4 * vols[0][::-1].copy()]))
    y = pn.splat(torch.from_numpy(x).float().cuda(), gp).double().cpu().numpy()
    for b in range(2):
        assert rel(y[b], O.splat(x[b], go)) <= TOL32, b


def test_splat_non_finite_stays_in_its_item(pn):
    gp, go, vols = make_case(pn, "cone3d_ragged")
    x = f32(np.stack([vols[0], 0.5 * vols[0]]))
    x[0, 10, 12, 11] = np.nan
    y = pn.splat(torch.from_numpy(x).float().cuda(), gp).double().cpu().numpy()
    ref0 = O.splat(x[0], go)
    assert np.all(np.isnan(y[0][np.isnan(ref0)])) and np.isfinite(y[0]).mean() > 0.5
    assert np.all(np.isfinite(y[1])) and rel(y[1], O.splat(x[1], go)) <= TOL32


def test_backprojection_layer_gradient(pn):
    """The back-projection layers are differentiable: the gradient of
    L(q) = 0.5 |B q - x|^2 is B^T (B q - x), checked against the oracle's
    splat of the oracle's residual, and by a central difference (exact for a
    quadratic up to rounding)."""
    gp, go, vols = make_case(pn, "fan2d_ragged")
    x = torch.from_numpy(vols[0]).float().cuda()
    q0 = O.forward(vols[0], go)
    q = torch.from_numpy(q0).float().cuda().requires_grad_(True)
    layer = pn.FanBackProjection2D(gp)
    loss = 0.5 * (layer(q) - x).square().sum()
    loss.backward()
    resid = O.backproject(f32(q0), go) - f32(vols[0])
    assert rel(q.grad.double().cpu().numpy(), O.splat(resid, go)) <= 1e-4
    d = torch.from_numpy(np.random.default_rng(3).standard_normal(q0.shape)).float().cuda()
    eps = 1e-3 * float(q.norm() / d.norm())

    def L(t):
        r = (pn.backproject(t, gp).double() - x.double())
        return 0.5 * float((r * r).sum())

    with torch.no_grad():
        fd = (L(q + eps * d) - L(q - eps * d)) / (2 * eps)
    an = float((q.grad.double() * d.double()).sum())
    assert abs(fd - an) <= 2e-3 * abs(an), (fd, an)


def test_splat_full_size_cone256_sampled_views(pn):
    """cone3d_256 (256^3 phantom, 360 views, 512^2 detector): four whole
    views of the GPU splat against the oracle's splat of those views."""
    cfg = W.CONFIGS["cone3d_256"]
    shp, sp, det, ds = cfg["vol_shape"], cfg["vol_spacing"], cfg["det_shape"], cfg["det_spacing"]
    gp = pn.cone_geometry(shp, sp, det, ds, cfg["n_views"], cfg["sid"], cfg["sdd"])
    go = O.circular_cone(shp, sp, det, ds, cfg["n_views"], cfg["angular_range"], cfg["sid"], cfg["sdd"])
    vol = W.ellipsoid_phantom_3d(cfg["seeds"][0], shp, sp, cfg["n_ellipsoids"])[0]
    _say("full size: GPU splat")
    y = pn.splat(torch.from_numpy(vol).float().cuda(), gp)
    torch.cuda.synchronize()
    views = [0, 45, 181, 299]
    sub = dict(go)
    sub["P"] = np.ascontiguousarray(go["P"][views])
    _say("full size: oracle splat of 4 views")
    ref = O.splat(f32(vol), sub)
    assert rel(y[views].double().cpu().numpy(), ref) <= TOL32
