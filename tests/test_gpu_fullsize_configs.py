"""GPU parity at the full sizes of the 2-D fan batch, the 32-problem uneven
batched list and the 512^3 cone problem (through the C ABI), on outputs the
FP64 oracle computes one at a time: sampled rays, sampled voxels of the
voxel-driven back-projection, and whole 16^3 (2-D: 32^2) blocks of the
adjoint.  Plus the finite-difference gradient check on the whole fan batch.

* fan2d_512x16: 16 images of 512^2 at 0.5 mm, 720 views over 360 deg,
  1024 bins at 0.5 mm, SID 1000, SDD 1500 (phantom seeds 2..17);
* batched list: 32 problems from seed 4 (64^3..256^3, 90..720 views,
  128^2..512^2 detectors; perturbed circular, helical, sinusoidal), run
  through the batched entry points;
* cone3d_512: 512^3 at 0.25 mm, 720 views, 1024^2 at 0.5 mm, SID 750,
  SDD 1200, in FP32, BF16 and FP16 storage (FP32 accumulation).

Tolerances: rel-L2 <= 1e-5 for FP32 storage, <= 1e-2 for 16-bit storage
(against the FP64 oracle of the unrounded phantom).
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
    print(f"[gpu-fullsize] {msg}", flush=True)
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


def take(t, *idx):
    """Elements of a device tensor at host index arrays, as FP64 numpy."""
    ii = tuple(torch.from_numpy(np.asarray(i, dtype=np.int64)).to(t.device) for i in idx)
    return t[ii].double().cpu().numpy()


# ------------------------------------------------------ 2-D fan batch ----


@pytest.fixture(scope="module")
def fan16(pn):
    cfg = W.CONFIGS["fan2d_512x16"]
    shp, sp = cfg["vol_shape"][1:], cfg["vol_spacing"][1:]
    nu, du = cfg["det_shape"][1], cfg["det_spacing"][1]
    gp = pn.fan_geometry(shp, sp, nu, du, cfg["n_views"], cfg["sid"], cfg["sdd"], cfg["angular_range"])
    go = O.circular_fan(shp, sp, nu, du, cfg["n_views"], cfg["angular_range"], cfg["sid"], cfg["sdd"])
    imgs = np.stack([W.ellipse_phantom_2d(s, shp, sp, cfg["n_ellipses"])[0] for s in cfg["seeds"]])
    return cfg, gp, go, imgs


@pytest.mark.timeout(600)
def test_fan_batch_full_size_sampled(pn, fan16):
    cfg, gp, go, imgs = fan16
    B, nv, nu = imgs.shape[0], cfg["n_views"], cfg["det_shape"][1]
    _say("fan 16 x 512^2 x 720 x 1024: forward")
    x = torch.from_numpy(imgs).float().cuda()
    y = pn.forward(x, gp)
    assert tuple(y.shape) == (B, nv, 1, nu)
    rng = np.random.default_rng(21)
    for b in range(B):
        view, col = rng.integers(0, nv, 400), rng.integers(0, nu, 400)
        ref = O.forward_rays(imgs[b], go, view, np.zeros(400, np.int64), col)
        assert rel(take(y, np.full(400, b), view, np.zeros(400, np.int64), col), ref) <= TOL32, f"item {b}"
    _say("fan batch: back-projection and adjoint")
    bp = pn.backproject(y, gp)
    at = pn.adjoint(y, gp)
    torch.cuda.synchronize()
    for b in (0, 7, 15):
        yb = y[b].double().cpu().numpy()
        i, j = rng.integers(0, 512, 600), rng.integers(0, 512, 600)
        refb = O.backproject_voxels(yb, go, i, j, np.zeros(600, np.int64))
        assert rel(take(bp, np.full(600, b), np.zeros(600, np.int64), j, i), refb) <= TOL32, f"item {b}"
        for box in ((240, 272, 240, 272, 0, 1), (0, 32, 480, 512, 0, 1)):
            refa = O.adjoint(yb, go, box=box)
            got = at[b, 0, box[2]:box[3], box[0]:box[1]].double().cpu().numpy()
            assert rel(got, refa[0]) <= TOL32, f"item {b} box {box}"


@pytest.mark.timeout(600)
def test_fan_batch_full_size_finite_difference(pn, fan16):
    """L(x) = 1/2 ||A x - y||^2 over the whole batch; the central difference
    along a smooth direction equals <A^T (A x - y), v> up to rounding (the
    step |A x - y| / |A v| keeps the FP32 rounding of L small against the
    difference)."""
    cfg, gp, go, imgs = fan16
    _say("fan batch: autograd finite differences")
    shp, sp = cfg["vol_shape"][1:], cfg["vol_spacing"][1:]
    target = np.stack([W.ellipse_phantom_2d(cfg["fd_target_seed"], shp, sp)[0]] * imgs.shape[0])
    y = pn.forward(torch.from_numpy(target).float().cuda(), gp).detach()
    x = torch.from_numpy(imgs).float().cuda().requires_grad_(True)
    loss = 0.5 * ((pn.Projection.apply(x, gp) - y) ** 2).sum()
    loss.backward()
    ph = lambda s: W.ellipse_phantom_2d(s, shp, sp)[0]
    v = torch.from_numpy(np.stack([ph(100 + 2 * b) - ph(101 + 2 * b) for b in range(imgs.shape[0])])).float().cuda()
    with torch.no_grad():
        res = (pn.forward(x.detach(), gp) - y).double()
        av = pn.forward(v, gp).double()
    eps = float(res.norm()) / float(av.norm())

    def L(z):
        r = (pn.forward(z, gp) - y).double()
        return 0.5 * float((r * r).sum())

    fd = (L(x.detach() + eps * v) - L(x.detach() - eps * v)) / (2 * eps)
    an = float((x.grad.double() * v.double()).sum())
    assert abs(fd - an) <= 1e-4 * abs(an)


# ------------------------------------------------- 32-problem list -------


def _batched_problem(pn, p):
    n = p["vol_shape"]
    draws = W.perturbation_draws(p["perturb_seed"], p["n_views"]) if p["trajectory"] == "perturbed" else None
    gp = pn.cone_geometry(n, p["vol_spacing"], p["det_shape"], p["det_spacing"], p["n_views"], p["sid"], p["sdd"],
                          p["angular_range"], p["trajectory"], p["pitch"], draws)
    S, C, eu, ev = O.trajectory_vectors(p["trajectory"], p["n_views"], p["angular_range"], p["sid"], p["sdd"],
                                        p["det_shape"], p["det_spacing"], n, p["vol_spacing"], p["pitch"], draws)
    Po = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], p["det_shape"]) for k in range(p["n_views"])])
    go = O.cone_geometry(n, p["vol_spacing"], p["det_shape"], p["det_spacing"], Po)
    vol = W.ellipsoid_phantom_3d(p["phantom_seed"], n, p["vol_spacing"], p["n_ellipsoids"])[0]
    return gp, go, vol


@pytest.mark.timeout(900)
def test_batched_list_32_problems_against_oracle(pn):
    probs = W.batched_problem_list()
    assert len(probs) == 32
    _say("batched list: 32 problems, building")
    built = [_batched_problem(pn, p) for p in probs]
    xs = [(torch.from_numpy(vol).float().cuda(), gp) for gp, _, vol in built]
    _say("batched list: forward, adjoint and back-projection (batched entry points)")
    ys = pn.forward_batched(xs)
    sp = [(y, gp) for y, (_, gp) in zip(ys, xs)]
    ats = pn.adjoint_batched(sp)
    bps = pn.backproject_batched(sp)
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    for i, ((gp, go, vol), p, y, at, bp) in enumerate(zip(built, probs, ys, ats, bps)):
        n, nvw, (rows, cols) = p["vol_shape"][0], p["n_views"], p["det_shape"]
        view, row, col = rng.integers(0, nvw, 300), rng.integers(0, rows, 300), rng.integers(0, cols, 300)
        assert rel(take(y, view, row, col), O.forward_rays(vol, go, view, row, col)) <= TOL32, f"problem {i}: A"
        yc = y.double().cpu().numpy()
        ii, jj, kk = rng.integers(0, n, 300), rng.integers(0, n, 300), rng.integers(0, n, 300)
        refb = O.backproject_voxels(yc, go, ii, jj, kk)
        assert rel(take(bp, kk, jj, ii), refb) <= TOL32, f"problem {i}: BP"
        c0 = int(rng.integers(0, n - 16 + 1))
        box = (c0, c0 + 16, n // 2 - 8, n // 2 + 8, n // 2 - 8, n // 2 + 8)
        refa = O.adjoint(yc, go, box=box)
        got = at[box[4]:box[5], box[2]:box[3], box[0]:box[1]].double().cpu().numpy()
        assert rel(got, refa) <= TOL32, f"problem {i}: AT box {box}"
        del yc
    _say("batched list: all 32 problems match")


# ------------------------------------------------- 512^3 cone ------------


@pytest.fixture(scope="module")
def cone512(pn):
    cfg = W.CONFIGS["cone3d_512"]
    shp, sp, det, ds = cfg["vol_shape"], cfg["vol_spacing"], cfg["det_shape"], cfg["det_spacing"]
    gp = pn.cone_geometry(shp, sp, det, ds, cfg["n_views"], cfg["sid"], cfg["sdd"], cfg["angular_range"])
    go = O.circular_cone(shp, sp, det, ds, cfg["n_views"], cfg["angular_range"], cfg["sid"], cfg["sdd"])
    vol = W.ellipsoid_phantom_3d(cfg["seeds"][0], shp, sp, cfg["n_ellipsoids"])[0]
    return cfg, gp, go, vol


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16, torch.float16])
def test_cone512_full_size_sampled(pn, cone512, dt):
    cfg, gp, go, vol = cone512
    tol = TOL32 if dt == torch.float32 else TOL16
    name = str(dt).split(".")[-1]
    nvw, (rows, cols) = cfg["n_views"], cfg["det_shape"]
    _say(f"cone 512^3 x 720 x 1024^2 ({name}): forward")
    x = torch.from_numpy(vol).to(torch.float32).cuda().to(dt)
    y = pn.forward(x, gp)
    assert y.dtype == dt
    rng = np.random.default_rng(512)
    view, row, col = rng.integers(0, nvw, 2000), rng.integers(0, rows, 2000), rng.integers(0, cols, 2000)
    assert rel(take(y, view, row, col), O.forward_rays(vol, go, view, row, col)) <= tol
    _say(f"cone 512^3 ({name}): back-projection (FP32 output)")
    bp = pn.backproject(y, gp, out_dtype=torch.float32)
    i, j, k = rng.integers(0, 512, 800), rng.integers(0, 512, 800), rng.integers(0, 512, 800)
    y32 = pn.forward(torch.from_numpy(vol).float().cuda(), gp) if dt != torch.float32 else y
    yc = y32.double().cpu().numpy()
    del y32
    refb = O.backproject_voxels(yc, go, i, j, k)
    assert rel(take(bp, k, j, i), refb) <= tol
    del bp
    _say(f"cone 512^3 ({name}): adjoint (FP32 output), two 16^3 blocks")
    at = pn.adjoint(y, gp, out_dtype=torch.float32)
    torch.cuda.synchronize()
    for box in ((248, 264, 248, 264, 248, 264), (40, 56, 300, 316, 100, 116)):
        refa = O.adjoint(yc, go, box=box)
        got = at[box[4]:box[5], box[2]:box[3], box[0]:box[1]].double().cpu().numpy()
        assert rel(got, refa) <= tol, f"box {box}"
