"""Trajectory tooling of the product binding (CPU, host logic only): moved
and turned panels, multi-turn helical orbits, calibrated matrices and their
decomposition (paper Sec. 2.4, arbitrary source and detector positions and
orientations; Sec. 2.1, calibrated matrices of real systems).

The binding's panel pose (Rodrigues rotations about the panel's moving
axes) and the oracle's (a product of axis rotation matrices) are separate
implementations of the same definition; they must agree, and so must the
matrices the native library composes from them and the oracle's.
"""
import math

import numpy as np
import pytest

import oracle as O

SID, SDD = 700.0, 1100.0


@pytest.fixture(scope="module")
def pn():
    import paper_2511_08427_amd as pn

    return pn


def _same_up_to_scale(P, Q):
    P, Q = np.asarray(P).reshape(-1, 12), np.asarray(Q).reshape(-1, 12)
    for a, b in zip(P, Q):
        s = np.dot(a, b) / np.dot(b, b)
        assert np.linalg.norm(a - s * b) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("offset,tilt", [((4.0, -2.5), (0.3, 0.0, 0.0)), ((0.0, 0.0), (0.0, 0.2, -0.35)),
                                         ((-11.0, 6.0), (-0.4, 0.25, 0.15))])
def test_panel_pose_matches_oracle(pn, offset, tilt):
    args = (12, 2 * math.pi, SID, SDD, (0.9, 0.7))
    S, C, eu, ev = pn.circular_vectors(*args)
    got = pn.detector_pose(S, C, eu, ev, offset, tilt)
    ref = O.detector_pose(*O.circular_cone_vectors(*args), offset, tilt)
    for g, r in zip(got, ref):
        assert np.abs(g - r).max() < 1e-11
    det = (30, 50)
    gp = pn.cone_geometry((20, 22, 24), (1.0, 1.0, 1.0), det, (0.9, 0.7), 12, SID, SDD, det_offset=offset,
                          det_tilt=tilt)
    Po = np.stack([O.cone_matrix(*(a[k] for a in ref), det) for k in range(12)])
    _same_up_to_scale(gp.matrices, Po)


def test_multi_turn_helical_matches_oracle(pn):
    args = ("helical", 90, 3 * 2 * math.pi, SID, SDD, (24, 40), (1.0, 1.0), (80, 32, 32), (1.0, 1.0, 1.0), 0.7)
    for g, r in zip(pn.trajectory_vectors(*args), O.trajectory_vectors(*args)):
        assert np.abs(g - r).max() < 1e-9


@pytest.mark.parametrize("scale", [1.0, -2.5, 1e-3])
def test_decompose_inverts_composition(pn, scale):
    det, ds = (28, 36), (0.8, 1.1)
    S, C, eu, ev = pn.circular_vectors(7, 2 * math.pi, SID, SDD, ds)
    S, C, eu, ev = pn.detector_pose(S + [0.0, 0.0, 3.0], C, eu, ev, (2.0, -1.0), (0.1, -0.2, 0.3))
    P = pn.cone_matrices(S, C, eu, ev, det)
    for k in range(7):
        got = pn.decompose_cone_matrix(scale * P[k], det, ds)
        for g, r in zip(got, (S[k], C[k], eu[k], ev[k])):
            assert np.abs(g - r).max() <= 1e-9 * max(1.0, np.abs(r).max())


def _pinhole(f_px, cu, cv, R, t):
    """K [R | t]: a textbook pinhole camera in pixel units (u = col, v = row)."""
    K = np.array([[f_px, 0.0, cu], [0.0, f_px, cv], [0.0, 0.0, 1.0]])
    return K @ np.hstack([R, np.asarray(t, float)[:, None]])


def _look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    z = np.asarray(target, float) - np.asarray(eye, float)
    z /= np.linalg.norm(z)
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return R, -R @ np.asarray(eye, float)


def test_calibrated_matrices_validated(pn):
    """Pinhole matrices K[R|t] of a camera looking at the volume are
    accepted as they are; the library refuses non-finite entries, a singular
    3x3 block, a source inside the volume and a volume partly behind the
    source."""
    shp, sp, det = (24, 26, 28), (1.0, 1.0, 1.0), (40, 48)
    Ps = []
    for k in range(5):
        a = 0.6 * k
        R, t = _look_at([SID * math.cos(a), SID * math.sin(a), 30.0 * math.sin(2 * a)])
        Ps.append(_pinhole(SDD / 0.9, 23.5, 19.5, R, t))
    g = pn.calibrated_geometry(np.stack(Ps), shp, sp, det)
    assert g.n_views == 5
    bad = np.stack(Ps).copy()
    bad[2, 1, 1] = np.nan
    with pytest.raises(pn.PnError):
        pn.calibrated_geometry(bad, shp, sp, det)
    bad = np.stack(Ps).copy()
    bad[1, 2, :3] = 0.0
    with pytest.raises(pn.PnError):
        pn.calibrated_geometry(bad, shp, sp, det)
    R, t = _look_at([3.0, 2.0, 1.0], target=(50.0, 0.0, 0.0))
    with pytest.raises(pn.PnError):
        pn.calibrated_geometry(_pinhole(500.0, 23.5, 19.5, R, t)[None], shp, sp, det)
    # a source above the volume looking along +x: its principal plane x = 0
    # cuts the volume, so part of it lies behind the source (a matrix and its
    # negative project alike, so only a sign change of W across the volume
    # can tell "behind")
    R, t = _look_at([0.0, 0.0, 100.0], target=(1000.0, 0.0, 100.0))
    with pytest.raises(pn.PnError):
        pn.calibrated_geometry(_pinhole(500.0, 23.5, 19.5, R, t)[None], shp, sp, det)


def test_decompose_pinhole_source(pn):
    """The source found by decomposing a pinhole matrix is the camera centre,
    and the panel's axes are orthogonal for a square-pixel K."""
    eye = np.array([SID * 0.6, -SID * 0.8, 40.0])
    R, t = _look_at(eye)
    P = _pinhole(SDD / 0.5, 31.5, 27.5, R, t)
    S, C, eu, ev = pn.decompose_cone_matrix(P, (56, 64), (0.5, 0.5))
    assert np.abs(S - eye).max() < 1e-9
    assert abs(np.dot(eu, ev)) < 1e-9 and abs(np.linalg.norm(eu) - 0.5) < 1e-12
    assert abs(np.linalg.norm(C - S) - SDD) < 1e-6
