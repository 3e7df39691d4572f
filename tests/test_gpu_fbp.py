"""GPU parity of the filtered back-projection (pn_filter, then pn_backproject)
against the FP64 oracle.

The filter is a linear convolution of each cosine-weighted detector row with
the discrete Ram-Lak or Shepp-Logan kernel, scaled by pi / N / a.  The
kernel computes it as a Toeplitz product on the matrix cores, FP32
operands and accumulators (nu multiply-adds per output with
|g[k]| <= 1/4 and sum_k |g[k]| < 1), so the expected FP32 rounding error of
an output is ~sqrt(nu) * 6e-8 * ||row||; the bar is relative L2 <= 1e-5 on
the whole filtered sinogram, as for the projectors.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = 1e-2


def _say(msg):
    print(f"[gpu-fbp] {msg}", flush=True)
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


def cpu(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


def make_case(pn, name):
    """(product geometry, oracle geometry, pixel pitch at the axis, volumes)."""
    if name == "parallel2d_95":
        gp = pn.parallel_geometry((64, 64), (1.0, 1.0), 95, 0.8, 90)
        go = O.parallel_2d((64, 64), (1.0, 1.0), 95, 0.8, 90, math.pi)
        return gp, go, 0.8, [W.ellipse_phantom_2d(1)[0]]
    if name == "fan2d_ragged":
        gp = pn.fan_geometry((100, 90), (0.5, 0.5), 150, 0.5, 96, 1000.0, 1500.0)
        go = O.circular_fan((100, 90), (0.5, 0.5), 150, 0.5, 96, 2 * math.pi, 1000.0, 1500.0)
        return gp, go, 0.5 * 1000.0 / 1500.0, [W.ellipse_phantom_2d(s, (100, 90), (0.5, 0.5))[0] for s in (2, 3)]
    if name == "cone3d_ragged":
        shp, sp, det, ds = (36, 44, 40), (0.5, 0.5, 0.5), (37, 45), (1.0, 1.1)
        gp = pn.cone_geometry(shp, sp, det, ds, 30, 750.0, 1200.0)
        go = O.circular_cone(shp, sp, det, ds, 30, 2 * math.pi, 750.0, 1200.0)
        return gp, go, 1.1 * 750.0 / 1200.0, [W.ellipsoid_phantom_3d(3, shp, sp)[0]]
    if name == "cone3d_wide_rows":
        # 1024 columns (the filter's maximum), a few rows
        shp, sp, det, ds = (24, 40, 40), (1.0, 1.0, 1.0), (6, 1024), (1.0, 0.1)
        gp = pn.cone_geometry(shp, sp, det, ds, 7, 300.0, 600.0)
        go = O.circular_cone(shp, sp, det, ds, 7, 2 * math.pi, 300.0, 600.0)
        return gp, go, 0.1 * 300.0 / 600.0, [W.ellipsoid_phantom_3d(5, shp, sp)[0]]
    raise KeyError(name)


@pytest.mark.parametrize("kind", ["ram-lak", "shepp-logan"])
@pytest.mark.parametrize("name", ["parallel2d_95", "fan2d_ragged", "cone3d_ragged", "cone3d_wide_rows"])
def test_filter_and_fbp_fp32(pn, name, kind):
    _say(f"case {name} {kind}: oracle sinogram")
    gp, go, pitch, vols = make_case(pn, name)
    sino = np.stack([O.forward(v, go) for v in vols])
    s32 = sino.astype(np.float32).astype(np.float64)
    _say(f"case {name} {kind}: filter {gp.sino_shape(len(vols))}")
    q = pn.fbp_filter(gpu(s32), gp, kind)
    torch.cuda.synchronize()
    ref_q = np.stack([O.fbp_filter(s, go, pitch, kind) for s in s32])
    assert rel(cpu(q), ref_q) <= TOL32, rel(cpu(q), ref_q)
    _say(f"case {name} {kind}: fbp")
    rec = pn.fbp(gpu(s32), gp, kind)
    torch.cuda.synchronize()
    ref_rec = np.stack([O.fbp(s, go, pitch, kind) for s in s32])
    assert rel(cpu(rec), ref_rec) <= TOL32, rel(cpu(rec), ref_rec)
    # the product FBP is exactly the back-projection of the product filter
    assert torch.equal(rec, pn.backproject(q, gp))


def test_filter_parallel_matches_direct_convolution(pn):
    """A random row set against the textbook linear convolution written as a
    sum (no FFT), in FP64: catches a reversed or shifted kernel."""
    gp = pn.parallel_geometry((8, 8), (1.0, 1.0), 77, 1.0, 3)
    go = O.parallel_2d((8, 8), (1.0, 1.0), 77, 1.0, 3, math.pi)
    rng = np.random.default_rng(5)
    p = rng.standard_normal((3, 1, 77)).astype(np.float32).astype(np.float64)
    q = cpu(pn.fbp_filter(gpu(p), gp, "shepp-logan"))
    n = np.arange(77)
    ref = np.empty_like(p)
    for v in range(3):
        for i in range(77):
            k = i - n
            ref[v, 0, i] = np.sum(-2.0 / (math.pi ** 2 * (4.0 * k * k - 1.0)) * p[v, 0]) * math.pi / 3
    assert rel(q, ref) <= TOL32
    assert rel(q, O.fbp_filter(p, go, 1.0, "shepp-logan")) <= TOL32


@pytest.mark.parametrize("kind", ["ram-lak", "shepp-logan"])
@pytest.mark.parametrize("nu", [16, 33, 128, 129, 511, 512, 513, 1000])
def test_filter_tile_edges_random_rows(pn, kind, nu):
    """Rows of white noise (no smoothness to hide a wrong tap) against the
    textbook linear convolution in FP64, for widths around the kernel's
    16-column blocks and 256-column wave tiles, across two 512-column
    workgroups, and a batch of 2 x 37 rows (partial 64-row workgroups)."""
    views = 37
    gp = pn.parallel_geometry((8, 8), (1.0, 1.0), nu, 1.0, views)
    rng = np.random.default_rng(nu)
    pb = rng.standard_normal((2, views, 1, nu)).astype(np.float32).astype(np.float64)
    qb = cpu(pn.fbp_filter(gpu(pb), gp, kind))
    assert rel(qb[1], cpu(pn.fbp_filter(gpu(pb[1]), gp, kind))) == 0.0  # batch items are independent rows
    p, q = pb[0], qb[0]
    k = np.arange(-nu + 1, nu)
    ak = np.abs(k).astype(np.float64)
    if kind == "ram-lak":
        g = np.where(ak == 0, 0.25, np.where(ak % 2 == 1, -1.0 / (math.pi ** 2 * np.maximum(ak, 1) ** 2), 0.0))
    else:
        g = -2.0 / (math.pi ** 2 * (4.0 * ak * ak - 1.0))
    G = g[(np.arange(nu)[:, None] - np.arange(nu)[None, :]) + nu - 1]   # G[n][m] = g[n - m]
    ref = (p[:, 0, :] @ G.T * (math.pi / views))[:, None, :]
    assert rel(q, ref) <= TOL32, (kind, nu, rel(q, ref))


def test_filter_edge_cases(pn):
    gp = pn.parallel_geometry((16, 16), (1.0, 1.0), 9, 1.0, 5)
    # empty batch, one column, the column limit
    pn.fbp_filter(torch.zeros((0, 5, 1, 9), device="cuda"), gp)
    g1 = pn.parallel_geometry((16, 16), (1.0, 1.0), 1, 2.0, 4)
    x = torch.full((4, 1, 1), 3.0, device="cuda")
    # one column: only g[0] = 1/4 contributes
    assert torch.allclose(pn.fbp_filter(x, g1), torch.full_like(x, 3.0 * 0.25 * math.pi / 4 / 2.0))
    gbig = pn.parallel_geometry((16, 16), (1.0, 1.0), 1025, 1.0, 2)
    with pytest.raises(RuntimeError, match="at most 1024"):
        pn.fbp_filter(torch.zeros((2, 1, 1025), device="cuda"), gbig)
    with pytest.raises(ValueError):
        pn.fbp_filter(torch.zeros((5, 1, 9), device="cuda"), gp, "hann")
    # divergent beams without source distances are refused
    gf = pn.fan_geometry((16, 16), (1.0, 1.0), 9, 1.0, 5, 100.0, 200.0)
    bad = pn.Geometry(2, "fan", gf.vol_shape, gf.vol_spacing, gf.det_shape, gf.matrices, gf.det_spacing)
    with pytest.raises(RuntimeError, match="sid > 0"):
        pn.fbp_filter(torch.zeros((5, 1, 9), device="cuda"), bad)


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
def test_filter_reduced_precision_storage(pn, dt):
    gp, go, pitch, vols = make_case(pn, "fan2d_ragged")
    sino = np.stack([O.forward(v, go) for v in vols[:1]])
    s16 = gpu(sino, dt)
    q = pn.fbp_filter(s16, gp)
    assert q.dtype == dt
    ref = O.fbp_filter(cpu(s16)[0], go, pitch)
    assert rel(cpu(q)[0], ref) <= TOL16


def test_full_size_cone256_filter_sampled(pn):
    cfg = W.CONFIGS["cone3d_256"]
    shp, sp, det, ds = cfg["vol_shape"], cfg["vol_spacing"], cfg["det_shape"], cfg["det_spacing"]
    gp = pn.cone_geometry(shp, sp, det, ds, cfg["n_views"], cfg["sid"], cfg["sdd"])
    go = O.circular_cone(shp, sp, det, ds, cfg["n_views"], cfg["angular_range"], cfg["sid"], cfg["sdd"])
    pitch = ds[1] * cfg["sid"] / cfg["sdd"]
    _say("full-size cone 256^3 x 360: forward + filter")
    vol = W.ellipsoid_phantom_3d(cfg["seeds"][0], shp, sp, cfg["n_ellipsoids"])[0]
    y = pn.forward(gpu(vol), gp)
    q = pn.fbp_filter(y, gp)
    torch.cuda.synchronize()
    views = np.array([0, 77, 181, 359])
    sub = dict(go)
    sub["P"] = go["P"][views]
    # the oracle takes N from the matrices it is given: rescale pi / 4 to pi / 360
    ref = O.fbp_filter(cpu(y[views]), sub, pitch) * (len(views) / cfg["n_views"])
    assert rel(cpu(q[views]), ref) <= TOL32
    _say("full-size cone 256^3 x 360: fdk")
    rec = pn.fbp(y, gp)
    assert torch.equal(rec, pn.backproject(q, gp))


@pytest.mark.parametrize("kind", ["ram-lak", "shepp-logan"])
def test_fdk_reconstructs_ball_gpu(pn, kind):
    """GPU FDK of a centred ball of radius 10 mm from its exact cone-beam line
    integrals (2 sqrt(R^2 - dist^2), dist = distance of the ray to the
    centre): the central slices are 1 inside and 0 outside up to
    discretisation, a closed-form check independent of the oracle's FBP."""
    nz, n, R, nvr, nuc, dd, sid, sdd, nviews = 48, 64, 10.0, 64, 96, 0.75, 400.0, 600.0, 120
    gp = pn.cone_geometry((nz, n, n), (0.5, 0.5, 0.5), (nvr, nuc), (dd, dd), nviews, sid, sdd)
    sino = np.zeros((nviews, nvr, nuc))
    uu, vv = np.meshgrid(np.arange(nuc, dtype=np.float64), np.arange(nvr, dtype=np.float64))
    pix = np.stack([uu.ravel(), vv.ravel(), np.ones(uu.size)])
    for k in range(nviews):
        Q = gp.matrices[k][:, :3]
        S = -np.linalg.solve(Q, gp.matrices[k][:, 3])
        d = np.linalg.solve(Q, pix)
        dist = np.linalg.norm(np.cross(S[None, :], d.T), axis=1) / np.linalg.norm(d, axis=0)
        sino[k] = np.where(dist < R, 2 * np.sqrt(np.maximum(R * R - dist ** 2, 0.0)), 0.0).reshape(nvr, nuc)
    rec = cpu(pn.fbp(gpu(sino), gp, kind))
    sl = rec[nz // 2 - 1:nz // 2 + 1].mean(axis=0)
    c = (np.arange(n) - (n - 1) / 2) * 0.5
    yy, xx = np.meshgrid(c, c, indexing="ij")
    r = np.hypot(xx, yy)
    inside, outside = sl[r < R - 2].mean(), np.abs(sl[(r > R + 2) & (r < c[-1])]).mean()
    assert abs(inside - 1.0) < 0.01 and outside < 0.01, (inside, outside)
