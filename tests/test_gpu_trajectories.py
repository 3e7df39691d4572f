"""GPU parity (through the C ABI) on the trajectory tooling: a moved and
turned detector panel, a three-turn helical orbit around a long object, and
calibrated pinhole matrices K[R|t] used as they are (paper Sec. 2.4,
arbitrary source and detector positions and orientations; Sec. 2.1,
calibrated matrices).  A, A^T and the voxel-driven BP against the FP64
oracle at rel-L2 <= 1e-5, plus the dot test for A^T.
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


def _say(msg):
    print(f"[gpu-trajectories] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_08427_amd as pn

    return pn


def rel(g, o):
    g, o = np.asarray(g, np.float64), np.asarray(o, np.float64)
    return float(np.linalg.norm((g - o).ravel()) / np.linalg.norm(o.ravel()))


def _look_at(eye, target, up=(0.0, 0.0, 1.0)):
    z = np.asarray(target, float) - np.asarray(eye, float)
    z /= np.linalg.norm(z)
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    return np.stack([x, np.cross(z, x), z])


def case(pn, name):
    if name == "tilted_offset_panel":
        shp, sp, det, ds, nv = (36, 40, 44), (0.5, 0.5, 0.5), (48, 56), (1.0, 1.0), 24
        off, tilt = (6.0, -4.0), (0.2, 0.15, -0.25)
        gp = pn.cone_geometry(shp, sp, det, ds, nv, 750.0, 1200.0, det_offset=off, det_tilt=tilt)
        vec = O.detector_pose(*O.circular_cone_vectors(nv, 2 * math.pi, 750.0, 1200.0, ds), off, tilt)
        Po = np.stack([O.cone_matrix(*(a[k] for a in vec), det) for k in range(nv)])
        return gp, O.cone_geometry(shp, sp, det, ds, Po), W.ellipsoid_phantom_3d(71, shp, sp, 8)[0]
    if name == "helical_three_turns_long_object":
        shp, sp, det, ds, nv = (96, 32, 32), (0.5, 0.5, 0.5), (24, 48), (1.0, 1.0), 120
        rng = 3 * 2 * math.pi
        gp = pn.cone_geometry(shp, sp, det, ds, nv, 750.0, 1200.0, rng, "helical", 0.8)
        S, C, eu, ev = O.trajectory_vectors("helical", nv, rng, 750.0, 1200.0, det, ds, shp, sp, 0.8)
        Po = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], det) for k in range(nv)])
        return gp, O.cone_geometry(shp, sp, det, ds, Po), W.ellipsoid_phantom_3d(72, shp, sp, 10)[0]
    if name == "calibrated_pinhole":
        shp, sp, det = (30, 34, 32), (0.6, 0.6, 0.6), (44, 52)
        rng = np.random.default_rng(73)
        Ps = []
        for k in range(18):
            a = 2 * math.pi * k / 18 + rng.normal(0, 0.02)
            eye = [800.0 * math.cos(a), 800.0 * math.sin(a), rng.normal(0, 15.0)]
            R = _look_at(eye, rng.normal(0, 2.0, 3))
            c, s = math.cos(rng.normal(0, 0.05)), math.sin(rng.normal(0, 0.05))
            R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]]) @ R       # roll about the viewing axis
            K = np.array([[1250.0 / 0.9, 0.0, 25.5 + rng.normal()], [0.0, 1250.0 / 0.9, 21.5 + rng.normal()],
                          [0.0, 0.0, 1.0]])
            Ps.append(K @ np.hstack([R, (-R @ np.asarray(eye))[:, None]]))
        P = np.stack(Ps)
        gp = pn.calibrated_geometry(P, shp, sp, det, (0.9, 0.9))
        return gp, O.cone_geometry(shp, sp, det, (0.9, 0.9), P), W.ellipsoid_phantom_3d(74, shp, sp, 8)[0]
    raise KeyError(name)


@pytest.mark.parametrize("name", ["tilted_offset_panel", "helical_three_turns_long_object", "calibrated_pinhole"])
def test_trajectory_tooling_parity(pn, name):
    _say(name)
    gp, go, vol = case(pn, name)
    y = pn.forward(torch.from_numpy(vol).float().cuda(), gp)
    yc = y.cpu().double().numpy()
    ref = O.forward(vol, go)
    assert np.linalg.norm(ref) > 0
    assert rel(yc, ref) <= TOL32
    assert rel(pn.adjoint(y, gp).cpu().numpy(), O.adjoint(yc, go)) <= TOL32
    assert rel(pn.backproject(y, gp).cpu().numpy(), O.backproject(yc, go)) <= TOL32
    rs = np.random.default_rng(5)
    xr = torch.from_numpy(rs.random(gp.vol_shape)).float().cuda()
    qr = torch.from_numpy(rs.random(gp.sino_shape())).float().cuda()
    lhs = float((pn.forward(xr, gp).double() * qr.double()).sum())
    rhs = float((xr.double() * pn.adjoint(qr, gp).double()).sum())
    assert abs(lhs - rhs) <= TOL32 * abs(lhs)
