"""FP64 CPU oracle for the CT projector operators -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library: geometry is
composed here with numpy, and the ray loops live in ``oracle.c`` (loaded with
ctypes).

Geometry (PYRO-NN update, Sec. 2.4 "Flexible Trajectory Modeling"): a
projection matrix is built from the source position, the detector position
and the detector's two (scaled) pixel directions, after Graetz's method
cited there.  With pixel (0, 0) at world position d00,

    M = [e_u | e_v | d00 - S],   P = M^-1 [I | -S],

so that pixel (c, r) maps to (U, V, W) = (c, r, 1) and u = U/W, v = V/W.
The 2-D fan-beam analogue drops the v axis; parallel beams replace the
source by a ray direction.  The circular trajectory of Listing 1 places view
k at angle beta_k = k * range / N (counter-clockwise about +z); this oracle
composes each view directly rather than by an incremental rotation.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# The mutation test of the pins (tests/test_oracle_mutations.py) loads a
# deliberately broken build from a temporary directory through this variable.
_LIB_LOAD = os.environ.get("ORACLE_LIB_OVERRIDE") or _LIB_PATH
_lib = None


def build(force=True):
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (-O2, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if _LIB_LOAD == _LIB_PATH and not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_LOAD)
        lib.oracle_ray_taps.restype = ctypes.c_int64
        _lib = lib
    return _lib


_I64P = ctypes.POINTER(ctypes.c_int64)
_F64P = ctypes.POINTER(ctypes.c_double)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_I64P)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_F64P)


def max_threads():
    return int(_load().oracle_max_threads())


# --------------------------------------------------------------- geometry --


def cone_matrix(S, C, eu, ev, det_shape):
    """3x4 matrix of a flat-panel cone-beam view.

    S: source, C: detector centre, eu/ev: world step per column/row (mm),
    det_shape: (rows, cols).  Pixel (c, r) sits at
    C + (c - (cols-1)/2) eu + (r - (rows-1)/2) ev.
    """
    nv, nu = det_shape
    S, C, eu, ev = (np.asarray(a, dtype=np.float64) for a in (S, C, eu, ev))
    d00 = C - 0.5 * (nu - 1) * eu - 0.5 * (nv - 1) * ev
    M = np.column_stack([eu, ev, d00 - S])
    Mi = np.linalg.inv(M)
    return np.hstack([Mi, -(Mi @ S)[:, None]])


def fan_matrix(S, C, eu, n_cols):
    """2x3 matrix of a flat-detector fan-beam view (2-D analogue of cone_matrix)."""
    S, C, eu = (np.asarray(a, dtype=np.float64) for a in (S, C, eu))
    d0 = C - 0.5 * (n_cols - 1) * eu
    M = np.column_stack([eu, d0 - S])
    Mi = np.linalg.inv(M)
    return np.hstack([Mi, -(Mi @ S)[:, None]])


def parallel2d_matrix(direction, C, eu, n_cols):
    """2x3 matrix of a 2-D parallel-beam view: rays along ``direction``,
    detector axis ``eu`` (mm per bin) through the point C (the central bin)."""
    M = np.column_stack([np.asarray(eu, float), np.asarray(direction, float)])
    Mi = np.linalg.inv(M)
    row = np.concatenate([Mi[0], [-(Mi[0] @ np.asarray(C, float)) + 0.5 * (n_cols - 1)]])
    return np.vstack([row, [0.0, 0.0, 1.0]])


def parallel3d_matrix(direction, C, eu, ev, det_shape):
    """3x4 matrix of a 3-D parallel-beam view (last row (0, 0, 0, 1))."""
    nv, nu = det_shape
    M = np.column_stack([np.asarray(eu, float), np.asarray(ev, float), np.asarray(direction, float)])
    Mi = np.linalg.inv(M)
    C = np.asarray(C, float)
    r0 = np.concatenate([Mi[0], [-(Mi[0] @ C) + 0.5 * (nu - 1)]])
    r1 = np.concatenate([Mi[1], [-(Mi[1] @ C) + 0.5 * (nv - 1)]])
    return np.vstack([r0, r1, [0.0, 0.0, 0.0, 1.0]])


def circular_cone_vectors(n_views, angular_range, sid, sdd, det_spacing):
    """Source, detector centre and pixel steps of a circular orbit about +z.

    det_spacing = (row spacing, column spacing) in mm.  Returns four arrays
    of shape (n_views, 3).
    """
    dv, du = det_spacing
    beta = np.arange(n_views, dtype=np.float64) * (angular_range / n_views)
    cb, sb = np.cos(beta), np.sin(beta)
    z = np.zeros_like(beta)
    S = np.stack([sid * cb, sid * sb, z], axis=1)
    C = np.stack([-(sdd - sid) * cb, -(sdd - sid) * sb, z], axis=1)
    eu = np.stack([-du * sb, du * cb, z], axis=1)
    ev = np.stack([z, z, dv + z], axis=1)
    return S, C, eu, ev


def cone_geometry(vol_shape, vol_spacing, det_shape, det_spacing, P, origin=None, parallel=False):
    """Oracle geometry dict for a 3-D problem.

    vol_shape/vol_spacing/origin in (z, y, x) order (as the array axes);
    det_shape = (rows, cols); P has shape (n_views, 3, 4).
    """
    nz, ny, nx = (int(v) for v in vol_shape)
    sz, sy, sx = (float(v) for v in vol_spacing)
    if origin is None:
        origin = (-0.5 * (nz - 1) * sz, -0.5 * (ny - 1) * sy, -0.5 * (nx - 1) * sx)
    return dict(
        dims=3,
        parallel=bool(parallel),
        n=(nx, ny, nz),
        s=(sx, sy, sz),
        o=(float(origin[2]), float(origin[1]), float(origin[0])),
        P=np.ascontiguousarray(P, dtype=np.float64).reshape(-1, 3, 4),
        det=(int(det_shape[0]), int(det_shape[1])),
    )


def image_geometry(img_shape, img_spacing, n_cols, P, origin=None, parallel=False):
    """Oracle geometry dict for a 2-D problem.

    img_shape/img_spacing/origin in (y, x) order; P has shape (n_views, 2, 3).
    """
    ny, nx = (int(v) for v in img_shape)
    sy, sx = (float(v) for v in img_spacing)
    if origin is None:
        origin = (-0.5 * (ny - 1) * sy, -0.5 * (nx - 1) * sx)
    return dict(
        dims=2,
        parallel=bool(parallel),
        n=(nx, ny, 1),
        s=(sx, sy, 1.0),
        o=(float(origin[1]), float(origin[0]), 0.0),
        P=np.ascontiguousarray(P, dtype=np.float64).reshape(-1, 2, 3),
        det=(1, int(n_cols)),
    )


def circular_cone(vol_shape, vol_spacing, det_shape, det_spacing, n_views, angular_range, sid, sdd):
    S, C, eu, ev = circular_cone_vectors(n_views, angular_range, sid, sdd, det_spacing)
    P = np.stack([cone_matrix(S[k], C[k], eu[k], ev[k], det_shape) for k in range(n_views)])
    return cone_geometry(vol_shape, vol_spacing, det_shape, det_spacing, P)


def circular_fan(img_shape, img_spacing, n_cols, det_spacing, n_views, angular_range, sid, sdd):
    beta = np.arange(n_views, dtype=np.float64) * (angular_range / n_views)
    P = []
    for b in beta:
        c, s = math.cos(b), math.sin(b)
        S = np.array([sid * c, sid * s])
        C = np.array([-(sdd - sid) * c, -(sdd - sid) * s])
        eu = det_spacing * np.array([-s, c])
        P.append(fan_matrix(S, C, eu, n_cols))
    return image_geometry(img_shape, img_spacing, n_cols, np.stack(P))


def parallel_2d(img_shape, img_spacing, n_cols, det_spacing, n_views, angular_range):
    theta = np.arange(n_views, dtype=np.float64) * (angular_range / n_views)
    P = []
    for t in theta:
        c, s = math.cos(t), math.sin(t)
        P.append(parallel2d_matrix([c, s], [0.0, 0.0], det_spacing * np.array([-s, c]), n_cols))
    return image_geometry(img_shape, img_spacing, n_cols, np.stack(P), parallel=True)


def trajectory_vectors(kind, n_views, angular_range, sid, sdd, det_shape, det_spacing, vol_shape,
                       vol_spacing, pitch=0.5, draws=None):
    """Vectors of the non-circular trajectories of the batched workload.

    helical: source and detector rise together, S_z = h (beta/2pi - T/2)
      with h = pitch * rows * row_spacing * SID/SDD (table feed per turn)
      over T = angular_range / 2pi turns (long objects: several turns);
    sinusoidal: S_z = A sin(2 beta), A = nz * sz / 4, detector follows;
    perturbed: circular orbit plus the Gaussian draws ``draws`` (dS, dC in
      mm, dphi in rad rotating the detector axes within the panel).
    """
    S, C, eu, ev = circular_cone_vectors(n_views, angular_range, sid, sdd, det_spacing)
    beta = np.arange(n_views, dtype=np.float64) * (angular_range / n_views)
    if kind == "helical":
        # T = angular_range / 2pi turns; the orbit is centred on z = 0
        h = pitch * det_shape[0] * det_spacing[0] * sid / sdd
        turns = angular_range / (2 * math.pi)
        dz = h * (beta / (2 * math.pi) - 0.5 * turns)
        S[:, 2] += dz
        C[:, 2] += dz
    elif kind == "sinusoidal":
        amp = vol_shape[0] * vol_spacing[0] / 4.0
        dz = amp * np.sin(2 * beta)
        S[:, 2] += dz
        C[:, 2] += dz
    elif kind == "perturbed":
        S = S + draws["dS"]
        C = C + draws["dC"]
        du = np.linalg.norm(eu, axis=1)[:, None]
        dv = np.linalg.norm(ev, axis=1)[:, None]
        uh, vh = eu / du, ev / dv
        cp, sp = np.cos(draws["dphi"])[:, None], np.sin(draws["dphi"])[:, None]
        eu = du * (cp * uh + sp * vh)
        ev = dv * (-sp * uh + cp * vh)
    elif kind != "circular":
        raise ValueError(kind)
    return S, C, eu, ev


def detector_pose(S, C, eu, ev, offset=(0.0, 0.0), tilt=(0.0, 0.0, 0.0)):
    """A flat panel moved within its plane and turned about its centre
    (Sec. 2.4, arbitrary detector positions and orientations).

    offset = (o_u, o_v): mm along the panel's unit axes (u_hat, v_hat);
    tilt = (roll, tilt_u, tilt_v) in rad: the panel frame
    F = [u_hat, v_hat, n_hat] (n_hat = u_hat x v_hat) becomes
    F Rz(roll) Rx(tilt_u) Ry(tilt_v), i.e. the panel turns about its own
    normal, then about its u axis, then about its v axis, all through the
    (shifted) centre.  Pixel pitches are kept.  Arrays of shape (n, 3).
    """
    S, C, eu, ev = (np.array(a, dtype=np.float64, ndmin=2) for a in (S, C, eu, ev))
    du = np.linalg.norm(eu, axis=1)[:, None]
    dv = np.linalg.norm(ev, axis=1)[:, None]
    uh, vh = eu / du, ev / dv
    nh = np.cross(uh, vh)
    C = C + offset[0] * uh + offset[1] * vh
    r, a, b = tilt
    Rz = np.array([[math.cos(r), -math.sin(r), 0.0], [math.sin(r), math.cos(r), 0.0], [0.0, 0.0, 1.0]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, math.cos(a), -math.sin(a)], [0.0, math.sin(a), math.cos(a)]])
    Ry = np.array([[math.cos(b), 0.0, math.sin(b)], [0.0, 1.0, 0.0], [-math.sin(b), 0.0, math.cos(b)]])
    R = Rz @ Rx @ Ry
    F = np.stack([uh, vh, nh], axis=2)          # columns u_hat, v_hat, n_hat per view
    G = F @ R
    return S, C, du * G[:, :, 0], dv * G[:, :, 1]


# -------------------------------------------------------------- operators --


def _geo_args(g):
    n, pn = _i64(np.array(g["n"]))
    s, ps = _f64(np.array(g["s"]))
    o, po = _f64(np.array(g["o"]))
    P, pP = _f64(g["P"])
    keep = (n, s, o, P)
    return keep, pn, ps, po, pP


def forward(vol, g, nthreads=0, weight_bits=0):
    """A vol.  vol: [nz][ny][nx] (2-D: [1][ny][nx]); returns [n_views][rows][cols].

    weight_bits = B > 0: the sampler variant (paper Sec. 2.1, texture versus
    kernel interpolation), whose in-plane interpolation weights are rounded
    to the nearest multiple of 2^-B, ties upward; 0 is A itself."""
    lib = _load()
    keep, pn, ps, po, pP = _geo_args(g)
    nv, nu = g["det"]
    nviews = g["P"].shape[0]
    v, pv = _f64(vol)
    assert v.size == g["n"][0] * g["n"][1] * g["n"][2]
    out = np.zeros((nviews, nv, nu), dtype=np.float64)
    rc = lib.oracle_forward_q(
        ctypes.c_int(g["dims"]), ctypes.c_int(int(g["parallel"])), pn, ps, po, ctypes.c_int64(nviews), pP,
        ctypes.c_int64(nv), ctypes.c_int64(nu), pv, out.ctypes.data_as(_F64P), ctypes.c_int(nthreads),
        ctypes.c_int(int(weight_bits)))
    if rc:
        raise MemoryError("oracle_forward")
    return out


def forward_rays(vol, g, view, row, col, nthreads=0, weight_bits=0):
    """Selected entries of A vol at (view[t], row[t], col[t]) (weight_bits as
    ``forward``)."""
    lib = _load()
    keep, pn, ps, po, pP = _geo_args(g)
    v, pv = _f64(vol)
    vw, pvw = _i64(view)
    rw, prw = _i64(row)
    cl, pcl = _i64(col)
    out = np.zeros(vw.size, dtype=np.float64)
    rc = lib.oracle_forward_rays_q(
        ctypes.c_int(g["dims"]), ctypes.c_int(int(g["parallel"])), pn, ps, po, pP, pv, ctypes.c_int64(vw.size),
        pvw, prw, pcl, out.ctypes.data_as(_F64P), ctypes.c_int(nthreads), ctypes.c_int(int(weight_bits)))
    if rc:
        raise MemoryError("oracle_forward_rays")
    return out


def adjoint(sino, g, box=None, nthreads=0):
    """A^T sino, optionally restricted to box = (i0, i1, j0, j1, k0, k1)."""
    lib = _load()
    keep, pn, ps, po, pP = _geo_args(g)
    nv, nu = g["det"]
    nviews = g["P"].shape[0]
    sn, psn = _f64(sino)
    assert sn.size == nviews * nv * nu
    nx, ny, nz = g["n"]
    if box is None:
        box = (0, nx, 0, ny, 0, nz)
    b, pb = _i64(np.array(box))
    out = np.zeros((b[5] - b[4], b[3] - b[2], b[1] - b[0]), dtype=np.float64)
    rc = lib.oracle_adjoint(
        ctypes.c_int(g["dims"]), ctypes.c_int(int(g["parallel"])), pn, ps, po, ctypes.c_int64(nviews), pP,
        ctypes.c_int64(nv), ctypes.c_int64(nu), psn, pb, out.ctypes.data_as(_F64P), ctypes.c_int(nthreads))
    if rc:
        raise MemoryError("oracle_adjoint")
    return out


def backproject(sino, g, nthreads=0, weight_bits=0):
    """Voxel-driven (W0/W)^2-weighted back-projection; returns [nz][ny][nx].

    weight_bits = B > 0: the sampler variant (paper Sec. 2.1), detector
    interpolation weights rounded to the nearest multiple of 2^-B, ties
    upward; 0 is the back-projection itself."""
    lib = _load()
    keep, pn, ps, po, pP = _geo_args(g)
    nv, nu = g["det"]
    nviews = g["P"].shape[0]
    sn, psn = _f64(sino)
    assert sn.size == nviews * nv * nu
    nx, ny, nz = g["n"]
    out = np.zeros((nz, ny, nx), dtype=np.float64)
    lib.oracle_backproject_q(
        ctypes.c_int(g["dims"]), pn, ps, po, ctypes.c_int64(nviews), pP, ctypes.c_int64(nv),
        ctypes.c_int64(nu), psn, out.ctypes.data_as(_F64P), ctypes.c_int(nthreads), ctypes.c_int(int(weight_bits)))
    return out


def backproject_voxels(sino, g, i, j, k, nthreads=0, weight_bits=0):
    """Back-projection at voxels (i[t], j[t], k[t]) only (weight_bits as
    ``backproject``)."""
    lib = _load()
    keep, pn, ps, po, pP = _geo_args(g)
    nv, nu = g["det"]
    nviews = g["P"].shape[0]
    sn, psn = _f64(sino)
    ii, pi = _i64(i)
    jj, pj = _i64(j)
    kk, pk = _i64(k)
    out = np.zeros(ii.size, dtype=np.float64)
    lib.oracle_backproject_voxels_q(
        ctypes.c_int(g["dims"]), pn, ps, po, ctypes.c_int64(nviews), pP, ctypes.c_int64(nv),
        ctypes.c_int64(nu), psn, ctypes.c_int64(ii.size), pi, pj, pk, out.ctypes.data_as(_F64P),
        ctypes.c_int(nthreads), ctypes.c_int(int(weight_bits)))
    return out


def splat(vol, g, nthreads=0):
    """Transpose of ``backproject``: each voxel's (W0/W)^2-weighted value
    spread over the bilinear taps of its projection; returns
    [n_views][rows][cols]."""
    lib = _load()
    keep, pn, ps, po, pP = _geo_args(g)
    nv, nu = g["det"]
    nviews = g["P"].shape[0]
    v, pv = _f64(vol)
    assert v.size == g["n"][0] * g["n"][1] * g["n"][2]
    out = np.zeros((nviews, nv, nu), dtype=np.float64)
    lib.oracle_splat(
        ctypes.c_int(g["dims"]), pn, ps, po, ctypes.c_int64(nviews), pP, ctypes.c_int64(nv), ctypes.c_int64(nu),
        pv, out.ctypes.data_as(_F64P), ctypes.c_int(nthreads))
    return out


def ray_taps(g, view, row, col):
    """(voxel linear indices, weights*ds) of one ray: a row of the matrix A."""
    lib = _load()
    keep, pn, ps, po, pP = _geo_args(g)
    cap = 4 * max(g["n"]) + 4
    idx = np.zeros(cap, dtype=np.int64)
    w = np.zeros(cap, dtype=np.float64)
    psz = 6 if g["dims"] == 2 else 12
    Pv = np.ascontiguousarray(g["P"][view].reshape(psz))
    cnt = lib.oracle_ray_taps(
        ctypes.c_int(g["dims"]), ctypes.c_int(int(g["parallel"])), pn, ps, po, Pv.ctypes.data_as(_F64P),
        ctypes.c_int64(row), ctypes.c_int64(col), idx.ctypes.data_as(_I64P), w.ctypes.data_as(_F64P))
    return idx[:cnt].copy(), w[:cnt].copy()


# ------------------------------------------------------------------ FBP ----
#
# Filtered back-projection (PYRO-NN update, Sec. 2.2: the reconstruction is
# the back-projection of the sinogram filtered along detector rows by a
# diagonal Fourier-domain filter between an FFT and its inverse).  Readings
# where the paper is silent: the filter K is the DFT of the discrete
# Ram-Lak kernel g (g[0] = 1/4, g[k] = -1/(pi^2 k^2) for odd k, 0 for even
# k != 0; Shepp-Logan: g[k] = -2 / (pi^2 (4 k^2 - 1))) on rows zero-padded
# to at least twice their length, so the product is the linear convolution
# of each row with g; divergent beams weight each pixel by the cosine of
# its ray's angle to the detector normal before filtering (Feldkamp); the
# kernel is in units of the pixel pitch at the rotation axis (du * SID / SDD
# for divergent beams); the back-projection is the voxel-driven (W0/W)^2
# weighted one; the result is scaled by pi / N (full 2 pi orbit, or pi for
# parallel beams).


def ramp_kernel(n, kind="ram-lak"):
    """Discrete filter kernel g[k] for k = 0 .. n-1 (even: g[-k] = g[k])."""
    k = np.arange(n, dtype=np.float64)
    if kind == "ram-lak":
        g = np.where(k % 2 == 1, -1.0 / (math.pi ** 2 * np.maximum(k, 1.0) ** 2), 0.0)
        g[0] = 0.25
    elif kind == "shepp-logan":
        g = -2.0 / (math.pi ** 2 * (4.0 * k * k - 1.0))
    else:
        raise ValueError(kind)
    return g


def cosine_weights(g):
    """Per view, row and column: the cosine of the ray's angle to the
    detector normal, 1 / (|q3| |d|) with q3 the last row of the 3x3 (2-D:
    2x2) part of P and d = (that part)^-1 (u, v, 1) the ray from the source
    to the pixel (q3 . d = 1); ones for parallel beams."""
    nv, nu = g["det"]
    nviews = g["P"].shape[0]
    if g["parallel"]:
        return np.ones((nviews, nv, nu))
    out = np.empty((nviews, nv, nu))
    for k in range(nviews):
        if g["dims"] == 3:
            Q = g["P"][k][:, :3]
            u, v = np.meshgrid(np.arange(nu, dtype=np.float64), np.arange(nv, dtype=np.float64))
            pix = np.stack([u.ravel(), v.ravel(), np.ones(u.size)])
        else:
            Q = g["P"][k][:, :2]
            pix = np.stack([np.arange(nu, dtype=np.float64), np.ones(nu)])
        d = np.linalg.solve(Q, pix)
        out[k] = (1.0 / (np.linalg.norm(Q[-1]) * np.linalg.norm(d, axis=0))).reshape(nv, nu)
    return out


def fbp_filter(sino, g, du_axis, kind="ram-lak"):
    """The filtered sinogram q = (pi / N) (1 / du_axis) F^-1 K F (c p) along
    detector rows, FP64; sino has shape [n_views][rows][cols]."""
    nviews = g["P"].shape[0]
    nv, nu = g["det"]
    p = np.asarray(sino, dtype=np.float64).reshape(nviews, nv, nu) * cosine_weights(g)
    L = 1
    while L < 2 * nu:
        L *= 2
    gk = ramp_kernel(nu, kind)
    circ = np.zeros(L)
    circ[:nu] = gk
    circ[L - nu + 1:] = gk[1:][::-1]
    K = np.fft.fft(circ)
    F = np.fft.fft(p, n=L, axis=-1)
    q = np.real(np.fft.ifft(F * K, axis=-1))[..., :nu]
    return q * (math.pi / nviews) / du_axis


def fbp(sino, g, du_axis, kind="ram-lak", nthreads=0):
    """Filtered back-projection: the voxel-driven back-projection of
    fbp_filter(sino)."""
    return backproject(fbp_filter(sino, g, du_axis, kind), g, nthreads)


# --------------------------------------------------- artifact simulation --
#
# Sinogram-domain artifacts (PYRO-NN update, Sec. 2.4 "Advanced Simulation
# Tool"): additive Gaussian noise with a given mean and standard deviation,
# and ring artifacts (chosen detector columns scaled, e.g. set to zero, over
# a range of views).  Random numbers come from the counter-based generator
# Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11), written out here from
# its published definition; a standard normal pair comes from two uniforms
# by the Box-Muller transform.  Readings where the paper is silent: element
# i of the flat sinogram takes word i mod 4 of the Philox block at counter
# (i div 4, 0, 0, 0) under key (seed, 0); uniforms are ((w >> 11) + 1/2)
# 2^-53, so never 0 or 1; words (0, 1) and (2, 3) of a block form the
# Box-Muller pairs, the first of a pair taking the cosine and the second the
# sine.

_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """(high, low) 64-bit halves of the 128-bit products a * b (uint64)."""
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, a * b


def philox4x64(counter, key, rounds=10):
    """Philox4x64 blocks: counter is 4 uint64 arrays (broadcastable), key 2;
    returns the 4 output words.  Each round multiplies words 0 and 2 by the
    two round constants, swaps and xors the high halves with words 1, 3 and
    the key; the key grows by the two Weyl constants between rounds."""
    c = [np.asarray(x, np.uint64) for x in counter]
    k0, k1 = (np.asarray(x, np.uint64) for x in key)
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r:
                k0 = k0 + np.uint64(_PHILOX_W[0])
                k1 = k1 + np.uint64(_PHILOX_W[1])
            h0, l0 = _mulhilo64(np.uint64(_PHILOX_M[0]), c[0])
            h1, l1 = _mulhilo64(np.uint64(_PHILOX_M[1]), c[2])
            c = [h1 ^ c[1] ^ k0, l1, h0 ^ c[3] ^ k1, l0]
    return c


def standard_normal_at(index, seed):
    """The standard normal draw z_i for flat element indices i (int64)."""
    i = np.asarray(index, dtype=np.int64).astype(np.uint64)
    z = np.zeros(i.shape, dtype=np.uint64)
    w = philox4x64([i >> np.uint64(2), z, z, z], [np.uint64(seed), np.uint64(0)])
    u = [((x >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53 for x in w]
    q = (i & np.uint64(3)).astype(np.int64)
    pair = q >> 1
    ua = np.where(pair == 0, u[0], u[2])
    ub = np.where(pair == 0, u[1], u[3])
    r = np.sqrt(-2.0 * np.log(ua))
    return np.where(q & 1 == 0, r * np.cos(2.0 * math.pi * ub), r * np.sin(2.0 * math.pi * ub))


def gaussian_noise(x, mean, sigma, seed):
    """x + mean + sigma z over the flat elements of x, FP64."""
    x = np.asarray(x, dtype=np.float64)
    return x + mean + sigma * standard_normal_at(np.arange(x.size), seed).reshape(x.shape)


def ring_artifacts(sino, columns, gain, v0, v1):
    """sino[..., v, :, c] times gain for views v0 <= v < v1 and the given
    detector columns; sino is [batch][views][rows][cols].  The product is
    taken in FP32 (the storage precision), so the result is exact."""
    out = np.array(sino, dtype=np.float32, copy=True)
    cols = np.unique(np.asarray(columns, dtype=np.int64))
    out[:, v0:v1, :, cols] = out[:, v0:v1, :, cols] * np.float32(gain)
    return out


def jitter_shifts(n_rows, max_shift, seed):
    """Detector jitter (Sec. 2.4, artifact simulation): the integer shift of
    each detector row (flat index g over batch, view and row), uniform in
    -max_shift .. max_shift, from word 0 of the Philox4x64-10 block at counter
    (g, 0, 0, 0) under key (seed, 1): (w0 mod (2 max_shift + 1)) - max_shift."""
    g = np.arange(n_rows, dtype=np.uint64)
    z = np.zeros_like(g)
    w = philox4x64([g, z, z, z], [np.uint64(seed), np.uint64(1)])
    return (w[0] % np.uint64(2 * max_shift + 1)).astype(np.int64) - max_shift


def detector_jitter(sino, max_shift, seed):
    """Each detector row of sino [..., rows, cols] moved by its shift s along
    the columns: out[c] = in[c - s], zero where c - s leaves the row."""
    a = np.asarray(sino)
    cols = a.shape[-1]
    flat = a.reshape(-1, cols)
    s = jitter_shifts(flat.shape[0], max_shift, seed)
    out = np.zeros_like(flat)
    for g in range(flat.shape[0]):
        for c in range(cols):
            src = c - s[g]
            if 0 <= src < cols:
                out[g, c] = flat[g, src]
    return out.reshape(a.shape)


def gantry_blur(sino, angle_start, angle_step, taps):
    """Gantry motion blur (Sec. 2.4, artifact simulation): each projection
    convolved with a line kernel turned to its acquisition angle.  Reading:
    view k has angle a_k = angle_start + k angle_step; the kernel is the mean
    of `taps` (odd) samples at unit spacing t = -h .. h, h = (taps - 1) / 2,
    along (cos a_k, sin a_k) in detector (column, row) pixel units; samples
    are bilinear with zeros outside the detector.  A single-row projection
    (2-D sinograms) has no row direction: the turned kernel acts through its
    column component, taps at t cos a_k along the row.  sino is
    [batch][views][rows][cols]; FP64."""
    a = np.asarray(sino, dtype=np.float64)
    nb, nv, nr, nc = a.shape
    h = (taps - 1) // 2
    rr, cc = np.meshgrid(np.arange(nr, dtype=np.float64), np.arange(nc, dtype=np.float64), indexing="ij")
    pad = np.zeros((nb, nv, nr + 2, nc + 2))
    pad[:, :, 1:-1, 1:-1] = a                      # pixel (r, c) at pad[r + 1, c + 1]
    out = np.zeros_like(a)
    for k in range(nv):
        ang = angle_start + k * angle_step
        du, dv = math.cos(ang), (math.sin(ang) if nr > 1 else 0.0)
        for t in range(-h, h + 1):
            x, y = cc + t * du, rr + t * dv
            x0, y0 = np.floor(x), np.floor(y)
            fx, fy = x - x0, y - y0
            acc = np.zeros((nb, nr, nc))
            for oy, wy in ((0, 1.0 - fy), (1, fy)):
                for ox, wx in ((0, 1.0 - fx), (1, fx)):
                    yi, xi = (y0 + oy).astype(np.int64), (x0 + ox).astype(np.int64)
                    inside = (yi >= 0) & (yi < nr) & (xi >= 0) & (xi < nc)
                    v = pad[:, k, np.clip(yi, -1, nr) + 1, np.clip(xi, -1, nc) + 1] * inside
                    acc += wy * wx * v
            out[:, k] += acc
    return out / taps
