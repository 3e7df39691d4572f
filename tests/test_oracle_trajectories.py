"""Pins of the oracle's trajectory tooling (CPU): moved and turned detector
panels and multi-turn helical orbits (paper Sec. 2.4, arbitrary source and
detector positions and orientations), checked against closed forms of the
central projection that do not go through the oracle's composition code.

Geometry of view 0 of the circular orbit: source S = (SID, 0, 0), central
ray along -x, panel centre at distance SDD from the source, u_hat = +y,
v_hat = +z, n_hat = u_hat x v_hat = +x (towards the source).
"""
import math

import numpy as np
import pytest

import oracle as O

SID, SDD = 600.0, 1000.0
DET = (40, 64)          # rows, cols
DS = (0.8, 0.6)         # row, column spacing (mm)


def _proj(P, X):
    U = P @ np.append(X, 1.0)
    return U[0] / U[2], U[1] / U[2]


def _view0(offset=(0.0, 0.0), tilt=(0.0, 0.0, 0.0)):
    S, C, eu, ev = O.circular_cone_vectors(1, 2 * math.pi, SID, SDD, DS)
    S, C, eu, ev = O.detector_pose(S, C, eu, ev, offset, tilt)
    return O.cone_matrix(S[0], C[0], eu[0], ev[0], DET)


CU, CV = 0.5 * (DET[1] - 1), 0.5 * (DET[0] - 1)


def test_offset_panel_moves_the_isocentre_image():
    """A panel shifted by (o_u, o_v) mm within its plane sees the isocentre
    at ((cols-1)/2 - o_u/du, (rows-1)/2 - o_v/dv)."""
    for ou, ov in ((12.5, 0.0), (0.0, -7.25), (-30.0, 18.0)):
        u, v = _proj(_view0((ou, ov)), np.zeros(3))
        assert abs(u - (CU - ou / DS[1])) < 1e-9 and abs(v - (CV - ov / DS[0])) < 1e-9


@pytest.mark.parametrize("gamma", [0.3, -0.45])
def test_panel_turned_about_v(gamma):
    """Turned by gamma about its v axis (through its centre), the panel maps
    a point seen at angle theta from the central ray (in the central plane)
    to u_mm = SDD (cos g tan(theta + g) - sin g); the isocentre stays at the
    centre pixel."""
    P = _view0(tilt=(0.0, 0.0, gamma))
    u, v = _proj(P, np.zeros(3))
    assert abs(u - CU) < 1e-9 and abs(v - CV) < 1e-9
    for L in (-40.0, 15.0, 55.0):
        theta = math.atan2(L, SID)
        u_mm = SDD * (math.cos(gamma) * math.tan(theta + gamma) - math.sin(gamma))
        u, v = _proj(P, np.array([0.0, L, 0.0]))
        assert abs(u - (CU + u_mm / DS[1])) < 1e-9 and abs(v - CV) < 1e-9


@pytest.mark.parametrize("alpha", [0.25, -0.4])
def test_panel_turned_about_u(alpha):
    """Turned by alpha about its u axis, v_mm = SDD (cos a tan(phi - a) +
    sin a) for a point at elevation phi above the central ray."""
    P = _view0(tilt=(0.0, alpha, 0.0))
    for H in (-30.0, 10.0, 45.0):
        phi = math.atan2(H, SID)
        v_mm = SDD * (math.cos(alpha) * math.tan(phi - alpha) + math.sin(alpha))
        u, v = _proj(P, np.array([0.0, 0.0, H]))
        assert abs(v - (CV + v_mm / DS[0])) < 1e-9 and abs(u - CU) < 1e-9


def test_panel_rolled_about_its_normal():
    """Rolled by phi about its normal, a point imaged at panel offsets
    (a, b) mm is imaged at (a cos phi + b sin phi, -a sin phi + b cos phi)."""
    phi = 0.37
    P0, P1 = _view0(), _view0(tilt=(phi, 0.0, 0.0))
    for X in (np.array([5.0, 20.0, -12.0]), np.array([-15.0, -33.0, 25.0])):
        u0, v0 = _proj(P0, X)
        a, b = (u0 - CU) * DS[1], (v0 - CV) * DS[0]
        u1, v1 = _proj(P1, X)
        assert abs((u1 - CU) * DS[1] - (a * math.cos(phi) + b * math.sin(phi))) < 1e-9
        assert abs((v1 - CV) * DS[0] - (-a * math.sin(phi) + b * math.cos(phi))) < 1e-9


def test_pose_keeps_pitch_and_orthogonality():
    S, C, eu, ev = O.circular_cone_vectors(5, 2 * math.pi, SID, SDD, DS)
    _, _, eu2, ev2 = O.detector_pose(S, C, eu, ev, (3.0, -2.0), (0.2, -0.3, 0.4))
    assert np.allclose(np.linalg.norm(eu2, axis=1), DS[1]) and np.allclose(np.linalg.norm(ev2, axis=1), DS[0])
    assert np.abs(np.sum(eu2 * ev2, axis=1)).max() < 1e-12


def test_multi_turn_helical_source_heights():
    """T turns: the source, read from each matrix as its null vector (SVD,
    not the composition), rises linearly by h per turn, centred on z = 0."""
    turns, per_turn = 3, 40
    n = turns * per_turn
    det, ds = (32, 48), (1.0, 1.0)
    S, C, eu, ev = O.trajectory_vectors("helical", n, 2 * math.pi * turns, SID, SDD, det, ds, (64, 48, 48),
                                        (1.0, 1.0, 1.0), pitch=0.8)
    h = 0.8 * det[0] * ds[0] * SID / SDD
    z = []
    for k in range(n):
        P = O.cone_matrix(S[k], C[k], eu[k], ev[k], det)
        w = np.linalg.svd(P)[2][-1]
        z.append(w[2] / w[3])
    z = np.array(z)
    beta = np.arange(n) * (2 * math.pi * turns / n)
    assert np.abs(z - h * (beta / (2 * math.pi) - 0.5 * turns)).max() < 1e-9
    assert abs((z[per_turn] - z[0]) - h) < 1e-9 and abs(z[0] + 1.5 * h) < 1e-9
