"""Acquisition geometry: volume/detector description plus one projection
matrix per view (PYRO-NN update, Listing 1 parameters and Sec. 2.4
"Flexible Trajectory Modeling").

Trajectories are described by per-view vectors -- source position S (or ray
direction for parallel beams), detector centre C and the world steps e_u /
e_v between neighbouring pixel centres -- and turned into projection
matrices by the native library (pn_*_matrices, FP64).  A circular orbit is
composed view by view at beta_k = k * range / N about +z (the paper rotates
incrementally; composing each view directly gives the same matrices up to
rounding).  Arbitrary matrices, e.g. calibrated ones, can be passed to
``Geometry`` directly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import _native as N

_BEAMS = {"parallel": N.PN_PARALLEL, "fan": N.PN_FAN, "cone": N.PN_CONE}


@dataclass
class Geometry:
    """A CT geometry.

    vol_shape/vol_spacing/vol_origin are in array order (z, y, x); 2-D
    geometries use vol_shape (1, ny, nx).  det_shape is (rows, cols); 2-D
    uses (1, cols).  ``matrices`` has shape (n_views, 3, 4) for 3-D and
    (n_views, 2, 3) for 2-D.  A NaN origin entry centres that axis.
    """

    ndim: int
    beam: str
    vol_shape: tuple
    vol_spacing: tuple
    det_shape: tuple
    matrices: np.ndarray
    det_spacing: tuple = (1.0, 1.0)
    vol_origin: tuple = (math.nan, math.nan, math.nan)
    sid: float = 0.0
    sdd: float = 0.0
    _c: object = field(default=None, init=False, repr=False, compare=False)

    def __post_init__(self):
        psh = (3, 4) if self.ndim == 3 else (2, 3)
        self.matrices = np.ascontiguousarray(np.asarray(self.matrices, dtype=np.float64).reshape((-1,) + psh))
        self.vol_shape = tuple(int(v) for v in self.vol_shape)
        self.det_shape = tuple(int(v) for v in self.det_shape)
        self.vol_spacing = tuple(float(v) for v in self.vol_spacing)
        self.det_spacing = tuple(float(v) for v in self.det_spacing)
        self.vol_origin = tuple(float(v) for v in self.vol_origin)
        if self.beam not in _BEAMS:
            raise ValueError(f"unknown beam {self.beam!r}")

    @property
    def n_views(self) -> int:
        return int(self.matrices.shape[0])

    def sino_shape(self, batch=None):
        s = (self.n_views,) + tuple(self.det_shape)
        return s if batch is None else (batch,) + s

    def vol_tensor_shape(self, batch=None):
        return tuple(self.vol_shape) if batch is None else (batch,) + tuple(self.vol_shape)

    def c_struct(self) -> N.PnGeometry:
        """The pn_geometry struct (kept alive with this object)."""
        if self._c is None:
            g = N.PnGeometry()
            g.ndim = self.ndim
            g.beam = _BEAMS[self.beam]
            for a in range(3):
                g.vol_shape[a] = self.vol_shape[a]
                g.vol_spacing[a] = self.vol_spacing[a]
                g.vol_origin[a] = self.vol_origin[a]
            for a in range(2):
                g.det_shape[a] = self.det_shape[a]
                g.det_spacing[a] = self.det_spacing[a]
            g.sid = self.sid
            g.sdd = self.sdd
            g.n_views = self.n_views
            g.proj = N.dptr(self.matrices)
            self._c = g
        return self._c

    def check(self):
        """Validates the geometry on the host (raises PnError)."""
        N.check(N.lib.pn_check_geometry(self.c_struct()), "pn_check_geometry")
        return self


# ----------------------------------------------------- matrix builders ---


def cone_matrices(S, C, eu, ev, det_shape):
    S, C, eu, ev = (np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3)) for a in (S, C, eu, ev))
    n = S.shape[0]
    P = np.zeros((n, 3, 4))
    N.check(N.lib.pn_cone_matrices(n, N.dptr(S), N.dptr(C), N.dptr(eu), N.dptr(ev), int(det_shape[0]),
                                   int(det_shape[1]), N.dptr(P)), "pn_cone_matrices")
    return P


def fan_matrices(S, C, eu, n_cols):
    S, C, eu = (np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 2)) for a in (S, C, eu))
    n = S.shape[0]
    P = np.zeros((n, 2, 3))
    N.check(N.lib.pn_fan_matrices(n, N.dptr(S), N.dptr(C), N.dptr(eu), int(n_cols), N.dptr(P)), "pn_fan_matrices")
    return P


def parallel2d_matrices(direction, C, eu, n_cols):
    d, C, eu = (np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 2)) for a in (direction, C, eu))
    n = d.shape[0]
    P = np.zeros((n, 2, 3))
    N.check(N.lib.pn_parallel2d_matrices(n, N.dptr(d), N.dptr(C), N.dptr(eu), int(n_cols), N.dptr(P)),
            "pn_parallel2d_matrices")
    return P


def parallel3d_matrices(direction, C, eu, ev, det_shape):
    d, C, eu, ev = (np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3)) for a in (direction, C, eu, ev))
    n = d.shape[0]
    P = np.zeros((n, 3, 4))
    N.check(N.lib.pn_parallel3d_matrices(n, N.dptr(d), N.dptr(C), N.dptr(eu), N.dptr(ev), int(det_shape[0]),
                                         int(det_shape[1]), N.dptr(P)), "pn_parallel3d_matrices")
    return P


# --------------------------------------------------------- trajectories --


def _angles(n_views, angular_range):
    return np.arange(n_views, dtype=np.float64) * (float(angular_range) / n_views)


def circular_vectors(n_views, angular_range, sid, sdd, det_spacing):
    """Circular orbit about +z: S = SID (cos b, sin b, 0), detector centre
    C = -(SDD - SID)(cos b, sin b, 0), e_u = du (-sin b, cos b, 0),
    e_v = dv (0, 0, 1).  det_spacing = (dv, du)."""
    dv, du = det_spacing
    b = _angles(n_views, angular_range)
    cb, sb, z = np.cos(b), np.sin(b), np.zeros(n_views)
    S = np.stack([sid * cb, sid * sb, z], 1)
    C = np.stack([-(sdd - sid) * cb, -(sdd - sid) * sb, z], 1)
    eu = np.stack([-du * sb, du * cb, z], 1)
    ev = np.stack([z, z, np.full(n_views, float(dv))], 1)
    return S, C, eu, ev


def trajectory_vectors(kind, n_views, angular_range, sid, sdd, det_shape, det_spacing, vol_shape, vol_spacing,
                       pitch=0.5, draws=None):
    """Vectors of a circular ('circular'), helical, sinusoidal or perturbed
    circular trajectory.

    helical: source and detector rise by h = pitch * rows * dv * SID/SDD per
    turn over angular_range / 2pi turns (several for long objects), centred
    on z = 0: S_z = h (beta - angular_range / 2) / 2pi; sinusoidal:
    S_z = (nz sz / 4) sin(2 beta),
    detector following; perturbed: circular plus ``draws`` = {dS, dC (mm),
    dphi (rad, in-panel rotation of e_u/e_v)}.
    """
    S, C, eu, ev = circular_vectors(n_views, angular_range, sid, sdd, det_spacing)
    b = _angles(n_views, angular_range)
    if kind == "circular":
        pass
    elif kind == "helical":
        # feed h per turn over angular_range / 2pi turns, centred on z = 0
        h = pitch * det_shape[0] * det_spacing[0] * sid / sdd
        dz = h * (b - 0.5 * float(angular_range)) / (2 * math.pi)
        S[:, 2] += dz
        C[:, 2] += dz
    elif kind == "sinusoidal":
        dz = vol_shape[0] * vol_spacing[0] / 4.0 * np.sin(2 * b)
        S[:, 2] += dz
        C[:, 2] += dz
    elif kind == "perturbed":
        S = S + np.asarray(draws["dS"])
        C = C + np.asarray(draws["dC"])
        nu_ = np.linalg.norm(eu, axis=1, keepdims=True)
        nv_ = np.linalg.norm(ev, axis=1, keepdims=True)
        uh, vh = eu / nu_, ev / nv_
        c, s = np.cos(draws["dphi"])[:, None], np.sin(draws["dphi"])[:, None]
        eu, ev = nu_ * (c * uh + s * vh), nv_ * (c * vh - s * uh)
    else:
        raise ValueError(f"unknown trajectory kind {kind!r}")
    return S, C, eu, ev


def _rotate(v, axis, angle):
    """Rodrigues rotation of the rows of v about the unit rows of axis."""
    c, s = math.cos(angle), math.sin(angle)
    k = axis
    return v * c + np.cross(k, v) * s + k * np.sum(k * v, axis=1, keepdims=True) * (1.0 - c)


def detector_pose(S, C, eu, ev, offset=(0.0, 0.0), tilt=(0.0, 0.0, 0.0)):
    """Moves each flat panel within its plane and turns it about its centre
    (Sec. 2.4: arbitrary detector positions and orientations).

    offset (o_u, o_v): mm along the panel's unit axes u_hat, v_hat.
    tilt (roll, tilt_u, tilt_v), rad: the panel turns by `roll` about its
    normal n_hat = u_hat x v_hat, then by `tilt_u` about its (new) u axis,
    then by `tilt_v` about its (new) v axis, all through the shifted centre;
    the pixel pitches stay.  Vectors of shape (n_views, 3).
    """
    S, C, eu, ev = (np.array(a, dtype=np.float64, ndmin=2) for a in (S, C, eu, ev))
    du = np.linalg.norm(eu, axis=1, keepdims=True)
    dv = np.linalg.norm(ev, axis=1, keepdims=True)
    u, v = eu / du, ev / dv
    C = C + float(offset[0]) * u + float(offset[1]) * v
    n = np.cross(u, v)
    roll, tu, tv = (float(a) for a in tilt)
    u, v = _rotate(u, n, roll), _rotate(v, n, roll)
    v, n = _rotate(v, u, tu), _rotate(n, u, tu)
    u = _rotate(u, v, tv)
    return S, C, du * u, dv * v


def cone_geometry(vol_shape, vol_spacing, det_shape, det_spacing, n_views, sid, sdd,
                  angular_range=2 * math.pi, trajectory="circular", pitch=0.5, draws=None,
                  vol_origin=(math.nan,) * 3, det_offset=(0.0, 0.0), det_tilt=(0.0, 0.0, 0.0)) -> Geometry:
    """3-D cone beam on a generated trajectory (Listing 1: GeometryCone3D +
    circular_trajectory_3d), optionally with the panel moved by det_offset
    and turned by det_tilt (see detector_pose)."""
    S, C, eu, ev = trajectory_vectors(trajectory, n_views, angular_range, sid, sdd, det_shape, det_spacing,
                                      vol_shape, vol_spacing, pitch, draws)
    if any(det_offset) or any(det_tilt):
        S, C, eu, ev = detector_pose(S, C, eu, ev, det_offset, det_tilt)
    P = cone_matrices(S, C, eu, ev, det_shape)
    return Geometry(3, "cone", vol_shape, vol_spacing, det_shape, P, det_spacing, vol_origin, sid, sdd)


def fan_geometry(img_shape, img_spacing, n_cols, det_spacing, n_views, sid, sdd,
                 angular_range=2 * math.pi) -> Geometry:
    """2-D fan beam with a flat detector on a circular orbit."""
    b = _angles(n_views, angular_range)
    cb, sb = np.cos(b), np.sin(b)
    S = np.stack([sid * cb, sid * sb], 1)
    C = np.stack([-(sdd - sid) * cb, -(sdd - sid) * sb], 1)
    eu = float(det_spacing) * np.stack([-sb, cb], 1)
    P = fan_matrices(S, C, eu, n_cols)
    ny, nx = img_shape
    return Geometry(2, "fan", (1, ny, nx), (1.0,) + tuple(img_spacing), (1, n_cols), P,
                    (1.0, float(det_spacing)), (math.nan,) * 3, sid, sdd)


def parallel_geometry(img_shape, img_spacing, n_cols, det_spacing, n_views, angular_range=math.pi) -> Geometry:
    """2-D parallel beam; view k has rays along (cos t, sin t), t = k*range/N."""
    t = _angles(n_views, angular_range)
    ct, st = np.cos(t), np.sin(t)
    d = np.stack([ct, st], 1)
    eu = float(det_spacing) * np.stack([-st, ct], 1)
    P = parallel2d_matrices(d, np.zeros((n_views, 2)), eu, n_cols)
    ny, nx = img_shape
    return Geometry(2, "parallel", (1, ny, nx), (1.0,) + tuple(img_spacing), (1, n_cols), P,
                    (1.0, float(det_spacing)))


# ------------------------------------------------- calibrated matrices ---


def calibrated_geometry(matrices, vol_shape, vol_spacing, det_shape, det_spacing=(1.0, 1.0),
                        vol_origin=(math.nan,) * 3, beam="cone") -> Geometry:
    """A geometry from measured projection matrices (Sec. 2.1: calibrated
    matrices of a real system), checked by the library before use: finite,
    non-singular, the volume (dilated by a voxel) in front of every source
    and the source outside it (PnError otherwise).  matrices: (n, 3, 4)
    mapping world mm to detector pixel indices (column, row)."""
    ndim = 3 if np.asarray(matrices).shape[-2:] == (3, 4) else 2
    g = Geometry(ndim, beam, vol_shape, vol_spacing, det_shape, matrices, det_spacing, vol_origin)
    N.check(N.lib.pn_check_geometry(g.c_struct()), "pn_check_geometry")
    return g


def decompose_cone_matrix(P, det_shape, det_spacing):
    """Source, detector centre and pixel steps (S, C, e_u, e_v) of a 3x4
    cone-beam matrix, the inverse of cone_matrices for a panel with the given
    pixel pitch (det_spacing = (row, column) mm); the overall scale and sign
    of P do not matter."""
    P = np.asarray(P, dtype=np.float64).reshape(3, 4)
    A = P[:, :3]
    S = -np.linalg.solve(A, P[:, 3])
    Ai = np.linalg.inv(A)               # columns: e_u, e_v, d00 - S, up to one scale
    k = float(det_spacing[1]) / np.linalg.norm(Ai[:, 0])
    if np.dot(Ai[:, 2], -S) < 0:        # the pixel (0, 0) lies beyond the source, not behind it
        k = -k
    eu, ev, d00 = k * Ai[:, 0], k * Ai[:, 1], S + k * Ai[:, 2]
    rows, cols = det_shape
    C = d00 + 0.5 * (cols - 1) * eu + 0.5 * (rows - 1) * ev
    return S, C, eu, ev
