"""Pins of the FP64 oracle against facts fixed by mathematics, not by itself.

Each test checks the oracle against something independent of its code: an
array sum, a library interpolation routine, an explicit matrix, a closed-form
line integral, a symmetry of the geometry, or an independently composed
camera model.  Together they are meant to catch a dropped term, a wrong sign
or index, or a transposed operand anywhere in the oracle.
"""
import math

import numpy as np
import pytest
from scipy.ndimage import map_coordinates

import workloads as W


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


# ------------------------------------------------------------ helpers ---


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


# ------------------------------------------------ P1/P10: array sums ----


def test_parallel_axis_aligned_views_are_row_and_column_sums(O):
    # 64x64 image at 1 mm, 90 views over 180 deg, 95 bins at 1 mm.
    img, _ = W.ellipse_phantom_2d(1)
    g = O.parallel_2d((64, 64), (1.0, 1.0), 95, 1.0, 90, math.pi)
    p = O.forward(img, g)[:, 0, :]
    rows = img[0].sum(axis=1)  # over x, per y index j
    cols = img[0].sum(axis=0)  # over y, per x index i

    def get(a, i):
        return a[i] if 0 <= i < a.size else 0.0

    # view 0: rays along +x; bin c sits at y = c - 47 mm, i.e. halfway
    # between image rows j = c - 16 and c - 15.
    ref0 = np.array([0.5 * (get(rows, c - 16) + get(rows, c - 15)) for c in range(95)])
    assert np.abs(p[0] - ref0).max() < 1e-12 * np.abs(ref0).max()
    # view 45: rays along +y; u = -x + 47, bin c between columns 78-c, 79-c.
    ref45 = np.array([0.5 * (get(cols, 78 - c) + get(cols, 79 - c)) for c in range(95)])
    assert np.abs(p[45] - ref45).max() < 1e-12 * np.abs(ref45).max()
    # mass conservation of the axis-aligned view: sum_c p[c] * du = sx*sy*sum(img)
    assert abs(p[0].sum() * 1.0 - img.sum()) < 1e-12 * img.sum()


def test_parallel3d_axis_aligned_view_is_a_sum_along_x(O):
    vol, _ = W.ellipsoid_phantom_3d(7, shape=(6, 7, 8), spacing=(1.0, 1.0, 1.0), n_ellipsoids=4)
    # rays along +x, detector columns = y, rows = z, pixel size = voxel size,
    # detector centred on the volume: pixel (c, r) hits voxel row (j, k) = (c, r)
    P = O.parallel3d_matrix([1.0, 0, 0], [0, 0, 0], [0, 1.0, 0], [0, 0, 1.0], (6, 7))
    g = O.cone_geometry((6, 7, 8), (1.0, 1.0, 1.0), (6, 7), (1.0, 1.0), P[None], parallel=True)
    p = O.forward(vol, g)[0]
    assert np.abs(p - vol.sum(axis=2)).max() < 1e-12 * vol.sum(axis=2).max()


def test_cone_central_ray_is_a_half_voxel_average(O):
    # odd detector: the central pixel's ray runs along the x axis through the
    # isocentre; with an even grid it lies midway between four voxel rows.
    vol, _ = W.ellipsoid_phantom_3d(11, shape=(8, 8, 10), spacing=(0.7, 0.7, 0.9), n_ellipsoids=5)
    g = O.circular_cone((8, 8, 10), (0.7, 0.7, 0.9), (7, 9), (1.0, 1.0), 4, 2 * math.pi, 80.0, 130.0)
    p = O.forward(vol, g)
    ref = 0.9 * 0.25 * (vol[3, 3, :] + vol[3, 4, :] + vol[4, 3, :] + vol[4, 4, :]).sum()
    assert abs(p[0, 3, 4] - ref) < 1e-12 * abs(ref)


# ----------------------------------------------- P2: library interpolation --


def test_samples_match_scipy_map_coordinates_cone(O):
    rng = np.random.default_rng(5)
    shape, sp = (9, 10, 12), (0.9, 1.1, 1.0)
    vol = rng.random(shape)
    nv, nu, views = 9, 11, 5
    S, C, eu, ev = O.circular_cone_vectors(views, 2 * math.pi, 60.0, 95.0, (1.3, 1.2))
    P = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], (nv, nu)) for k in range(views)])
    g = O.cone_geometry(shape, sp, (nv, nu), (1.3, 1.2), P)
    p = O.forward(vol, g)
    nz, ny, nx = shape
    s = np.array([sp[2], sp[1], sp[0]])
    o = -0.5 * (np.array([nx, ny, nz]) - 1) * s
    for k in range(views):
        for r in range(nv):
            for c in range(nu):
                X = C[k] + (c - 0.5 * (nu - 1)) * eu[k] + (r - 0.5 * (nv - 1)) * ev[k]
                xi0 = (S[k] - o) / s
                de = (X - S[k]) / s
                a = int(np.argmax(np.abs(de)))
                na = [nx, ny, nz][a]
                m = np.arange(na, dtype=float)
                pts = xi0[None, :] + ((m - xi0[a]) / de[a])[:, None] * de[None, :]
                # map_coordinates wants (z, y, x) index order
                vals = map_coordinates(vol, pts[:, ::-1].T, order=1, mode="grid-constant", cval=0.0)
                D = X - S[k]
                ds = s[a] * np.linalg.norm(D) / abs(D[a])
                ref = ds * vals.sum()
                assert abs(p[k, r, c] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_samples_match_padded_interp_fan(O):
    rng = np.random.default_rng(6)
    ny, nx, sy, sx = 13, 11, 0.8, 1.1
    img = rng.random((1, ny, nx))
    n_cols, du, views, sid, sdd = 17, 0.9, 7, 40.0, 70.0
    g = O.circular_fan((ny, nx), (sy, sx), n_cols, du, views, 2 * math.pi, sid, sdd)
    p = O.forward(img, g)
    o = np.array([-0.5 * (nx - 1) * sx, -0.5 * (ny - 1) * sy])
    s = np.array([sx, sy])
    for k in range(views):
        b = 2 * math.pi * k / views
        S = sid * np.array([math.cos(b), math.sin(b)])
        Cc = -(sdd - sid) * np.array([math.cos(b), math.sin(b)])
        eu = du * np.array([-math.sin(b), math.cos(b)])
        for c in range(n_cols):
            X = Cc + (c - 0.5 * (n_cols - 1)) * eu
            xi0, de = (S - o) / s, (X - S) / s
            a = 0 if abs(de[0]) >= abs(de[1]) else 1
            bax = 1 - a
            acc = 0.0
            for m in range(img.shape[2] if a == 0 else img.shape[1]):
                q = xi0[bax] + (m - xi0[a]) / de[a] * de[bax]
                line = img[0, :, m] if a == 0 else img[0, m, :]
                # np.interp on the zero-padded line (grid -1..n)
                acc += np.interp(q, np.arange(-1, line.size + 1), np.pad(line, 1), left=0.0, right=0.0)
            D = X - S
            ref = s[a] * np.linalg.norm(D) / abs(D[a]) * acc
            assert abs(p[k, 0, c] - ref) <= 1e-12 * max(1.0, abs(ref))


# ------------------------------- sampler variant: quantised weights -------
#
# With weight_bits = B the oracle's sampler variant rounds each in-plane
# weight (the fraction of the crossing position) to the nearest multiple of
# 2^-B, ties upward.  Because floor(p) is an integer, that is linear
# interpolation at the position itself rounded to the 2^-B lattice, so a
# library interpolator evaluated at the rounded positions must agree.


def _snap(p, bits):
    """p rounded to the nearest multiple of 2^-bits, ties upward (every step
    exact in FP64)."""
    t = np.asarray(p, float) * 2.0 ** bits
    q = np.floor(t)
    return np.where(t - q >= 0.5, q + 1.0, q) / 2.0 ** bits


@pytest.mark.parametrize("bits", [3, 8])
def test_quantised_samples_match_map_coordinates_at_snapped_positions(O, bits):
    rng = np.random.default_rng(15)
    shape, sp = (9, 10, 12), (0.9, 1.1, 1.0)
    vol = rng.random(shape)
    nv, nu, views = 9, 11, 5
    S, C, eu, ev = O.circular_cone_vectors(views, 2 * math.pi, 60.0, 95.0, (1.3, 1.2))
    P = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], (nv, nu)) for k in range(views)])
    g = O.cone_geometry(shape, sp, (nv, nu), (1.3, 1.2), P)
    p = O.forward(vol, g, weight_bits=bits)
    exact = O.forward(vol, g)
    nz, ny, nx = shape
    s = np.array([sp[2], sp[1], sp[0]])
    o = -0.5 * (np.array([nx, ny, nz]) - 1) * s
    for k in range(views):
        for r in range(nv):
            for c in range(nu):
                X = C[k] + (c - 0.5 * (nu - 1)) * eu[k] + (r - 0.5 * (nv - 1)) * ev[k]
                xi0 = (S[k] - o) / s
                de = (X - S[k]) / s
                a = int(np.argmax(np.abs(de)))
                m = np.arange([nx, ny, nz][a], dtype=float)
                pts = xi0[None, :] + ((m - xi0[a]) / de[a])[:, None] * de[None, :]
                inplane = [i for i in range(3) if i != a]
                pts[:, inplane] = _snap(pts[:, inplane], bits)
                vals = map_coordinates(vol, pts[:, ::-1].T, order=1, mode="grid-constant", cval=0.0)
                D = X - S[k]
                ref = s[a] * np.linalg.norm(D) / abs(D[a]) * vals.sum()
                assert abs(p[k, r, c] - ref) <= 1e-12 * max(1.0, abs(ref))
    # the rounding is visible, and bounded: each of the two weights moves by
    # at most 2^-(B+1), which moves a sample by at most 2^-B max|v|; a ray
    # has at most 12 samples of at most 1.1 sqrt(3) mm each
    err = np.abs(p - exact)
    assert err.max() > 1e-3 * 2.0 ** -bits * np.abs(exact).max()
    assert err.max() <= 2.0 ** -bits * np.abs(vol).max() * 12 * 1.1 * math.sqrt(3)


def test_quantised_fan_samples_match_padded_interp_at_snapped_positions(O):
    rng = np.random.default_rng(16)
    ny, nx, sy, sx = 13, 11, 0.8, 1.1
    img = rng.random((1, ny, nx))
    n_cols, du, views, sid, sdd, bits = 17, 0.9, 7, 40.0, 70.0, 4
    g = O.circular_fan((ny, nx), (sy, sx), n_cols, du, views, 2 * math.pi, sid, sdd)
    p = O.forward(img, g, weight_bits=bits)
    o = np.array([-0.5 * (nx - 1) * sx, -0.5 * (ny - 1) * sy])
    s = np.array([sx, sy])
    for k in range(views):
        b = 2 * math.pi * k / views
        S = sid * np.array([math.cos(b), math.sin(b)])
        Cc = -(sdd - sid) * np.array([math.cos(b), math.sin(b)])
        eu = du * np.array([-math.sin(b), math.cos(b)])
        for c in range(n_cols):
            X = Cc + (c - 0.5 * (n_cols - 1)) * eu
            xi0, de = (S - o) / s, (X - S) / s
            a = 0 if abs(de[0]) >= abs(de[1]) else 1
            bax = 1 - a
            acc = 0.0
            for m in range(img.shape[2] if a == 0 else img.shape[1]):
                q = _snap(xi0[bax] + (m - xi0[a]) / de[a] * de[bax], bits)
                line = img[0, :, m] if a == 0 else img[0, m, :]
                acc += np.interp(q, np.arange(-1, line.size + 1), np.pad(line, 1), left=0.0, right=0.0)
            D = X - S
            ref = s[a] * np.linalg.norm(D) / abs(D[a]) * acc
            assert abs(p[k, 0, c] - ref) <= 1e-12 * max(1.0, abs(ref))


def _exact_tie_case(O):
    """Rays along +x through index rows (j + 3/16, k + 5/16): every entry is
    dyadic, so each crossing sits exactly on a rounding tie of the 2^-3
    lattice (3/16 * 8 = 1.5, 5/16 * 8 = 2.5)."""
    shape = (6, 7, 8)  # z, y, x
    P = O.parallel3d_matrix([1.0, 0, 0], [0, 3 / 16, 5 / 16], [0, 1.0, 0], [0, 0, 1.0], (6, 7))
    g = O.cone_geometry(shape, (1.0, 1.0, 1.0), (6, 7), (1.0, 1.0), P[None], parallel=True)
    return shape, g


def _exact_tie_expected(vol, wy, wz):
    """Bilinear rows of the zero-padded volume with weights wy, wz, summed
    along x: the ray of pixel (c, r) reads rows (j, k) = (c, r)."""
    pad = np.pad(vol, ((0, 1), (0, 1), (0, 0)))
    s = pad.sum(axis=2)  # [z][y]
    return ((1 - wy) * (1 - wz) * s[:-1, :-1] + wy * (1 - wz) * s[:-1, 1:] + (1 - wy) * wz * s[1:, :-1]
            + wy * wz * s[1:, 1:])


def test_exact_ties_round_upward(O):
    shape, g = _exact_tie_case(O)
    vol = np.random.default_rng(18).random(shape)
    got = O.forward(vol, g, weight_bits=3)[0]
    assert np.abs(got - _exact_tie_expected(vol, 2 / 8, 3 / 8)).max() < 1e-12
    assert np.abs(O.forward(vol, g)[0] - _exact_tie_expected(vol, 3 / 16, 5 / 16)).max() < 1e-12


def test_fine_weight_lattice_converges_to_the_operator(O):
    """Rounding to 2^-40 moves each weight by at most 2^-41: A itself to
    ~1e-11, while a coarse lattice does not."""
    vol, _ = W.ellipsoid_phantom_3d(17, shape=(10, 11, 12), spacing=(1.0, 1.0, 1.0), n_ellipsoids=6)
    g = O.circular_cone((10, 11, 12), (1.0, 1.0, 1.0), (9, 13), (1.4, 1.4), 6, 2 * math.pi, 70.0, 110.0)
    exact = O.forward(vol, g)
    assert _rel(O.forward(vol, g, weight_bits=40), exact) < 1e-10
    assert _rel(O.forward(vol, g, weight_bits=2), exact) > 1e-4


# -------------------------------------------- P3/P4: transpose, dot test --


def _explicit_A(O, g, shape):
    nvox = int(np.prod(shape))
    cols = []
    for j in range(nvox):
        e = np.zeros(nvox)
        e[j] = 1.0
        cols.append(O.forward(e.reshape(shape), g).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("kind", ["parallel2d", "fan2d", "cone3d", "parallel3d"])
def test_adjoint_equals_explicit_transpose(O, kind):
    if kind == "parallel2d":
        shape = (1, 5, 5)
        g = O.parallel_2d((5, 5), (1.0, 1.0), 7, 0.9, 5, math.pi)
    elif kind == "fan2d":
        shape = (1, 5, 6)
        g = O.circular_fan((5, 6), (1.0, 0.8), 9, 0.7, 4, 2 * math.pi, 20.0, 35.0)
    elif kind == "cone3d":
        shape = (4, 4, 5)
        g = O.circular_cone(shape, (1.0, 1.0, 0.8), (5, 5), (1.1, 1.0), 3, 2 * math.pi, 25.0, 40.0)
    else:
        shape = (4, 5, 4)
        P = np.stack([O.parallel3d_matrix([math.cos(t), math.sin(t), 0.3], [0, 0, 0],
                                          [-math.sin(t), math.cos(t), 0], [0, 0, 1.0], (5, 6))
                      for t in (0.3, 1.1, 2.0)])
        g = O.cone_geometry(shape, (1.0, 0.9, 1.0), (5, 6), (1.0, 1.0), P, parallel=True)
    A = _explicit_A(O, g, shape)
    nviews = g["P"].shape[0]
    nv, nu = g["det"]
    At = np.zeros((A.shape[1], A.shape[0]))
    for i in range(A.shape[0]):
        e = np.zeros(A.shape[0])
        e[i] = 1.0
        At[:, i] = O.adjoint(e.reshape(nviews, nv, nu), g).ravel()
    assert np.abs(At - A.T).max() <= 1e-14 * np.abs(A).max()
    # rows of A from the tap list agree with the columns built by projection
    for view in range(nviews):
        for r in range(nv):
            for c in range(nu):
                idx, w = O.ray_taps(g, view, r, c)
                row = np.zeros(A.shape[1])
                np.add.at(row, idx, w)
                assert np.abs(row - A[(view * nv + r) * nu + c]).max() <= 1e-14 * max(1.0, np.abs(row).max())


@pytest.mark.parametrize("dims", [2, 3])
def test_dot_product_adjoint(O, dims):
    rng = np.random.default_rng(12 + dims)
    if dims == 2:
        shape = (1, 40, 33)
        g = O.circular_fan((40, 33), (0.5, 0.6), 61, 0.5, 37, 2 * math.pi, 100.0, 160.0)
    else:
        shape = (17, 20, 23)
        g = O.circular_cone(shape, (0.5, 0.5, 0.5), (21, 30), (0.8, 0.8), 19, 2 * math.pi, 100.0, 160.0)
    x = rng.random(shape)
    y = rng.random((g["P"].shape[0],) + g["det"])
    Ax = O.forward(x, g)
    Aty = O.adjoint(y, g)
    lhs, rhs = float((Ax * y).sum()), float((x * Aty).sum())
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_adjoint_box_restriction_matches_full(O):
    rng = np.random.default_rng(2)
    shape = (9, 8, 10)
    g = O.circular_cone(shape, (1.0, 1.0, 1.0), (8, 9), (1.2, 1.2), 6, 2 * math.pi, 40.0, 64.0)
    y = rng.random((6, 8, 9))
    full = O.adjoint(y, g)
    part = O.adjoint(y, g, box=(2, 7, 1, 5, 3, 9))
    assert np.abs(part - full[3:9, 1:5, 2:7]).max() <= 1e-13 * np.abs(full).max()
    # a different thread count changes only the summation grouping
    one = O.adjoint(y, g, nthreads=1)
    assert np.abs(one - full).max() <= 1e-13 * np.abs(full).max()


# --------------------------------------- P5: analytic line integrals ----


def _smooth_ellipsoid(shape, spacing, centre, Q, rho):
    zc, yc, xc = W.voxel_centres(shape, spacing)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    R = np.stack([X - centre[0], Y - centre[1], Z - centre[2]], axis=-1)
    q = np.einsum("...i,ij,...j->...", R, Q, R)
    return np.where(q < 1.0, rho * (1.0 - q), 0.0)


def _smooth_ellipsoid_integral(p0, d, centre, Q, rho):
    """Integral of rho*(1 - q) over the line p0 + t d (|d| = 1), q <= 1:
    (4/3) rho disc^(3/2) / A^2 with A = d'Qd, B = d'Q(p0-c),
    disc = B^2 - A((p0-c)'Q(p0-c) - 1)."""
    r = p0 - centre
    A = d @ Q @ d
    B = d @ Q @ r
    disc = B * B - A * (r @ Q @ r - 1.0)
    return np.where(disc > 0, (4.0 / 3.0) * rho * np.maximum(disc, 0) ** 1.5 / A**2, 0.0)


def test_cone_converges_to_analytic_smooth_ellipsoid(O):
    # rotated anisotropic smooth ellipsoid in a 64 mm cube; the Joseph
    # projector of its point samples must converge at second order.
    th = 0.4
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(0.7), -math.sin(0.7)], [0, math.sin(0.7), math.cos(0.7)]])
    Rm = Rz @ Rx
    axes = np.array([22.0, 14.0, 10.0])
    Q = Rm @ np.diag(1 / axes**2) @ Rm.T
    centre = np.array([4.0, -3.0, 2.5])
    views, nv, nu, sid, sdd, du = 6, 24, 28, 200.0, 320.0, 2.5
    S, C, eu, ev = O.circular_cone_vectors(views, 2 * math.pi, sid, sdd, (du, du))
    # analytic values per pixel from the trajectory vectors
    ana = np.zeros((views, nv, nu))
    for k in range(views):
        cc, rr = np.meshgrid(np.arange(nu), np.arange(nv))
        X = C[k] + (cc[..., None] - 0.5 * (nu - 1)) * eu[k] + (rr[..., None] - 0.5 * (nv - 1)) * ev[k]
        D = X - S[k]
        D = D / np.linalg.norm(D, axis=-1, keepdims=True)
        for r in range(nv):
            for c in range(nu):
                ana[k, r, c] = _smooth_ellipsoid_integral(S[k], D[r, c], centre, Q, 1.0)
    errs = []
    for n in (16, 32, 64):
        h = 64.0 / n
        vol = _smooth_ellipsoid((n, n, n), (h, h, h), centre, Q, 1.0)
        P = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], (nv, nu)) for k in range(views)])
        g = O.cone_geometry((n, n, n), (h, h, h), (nv, nu), (du, du), P)
        p = O.forward(vol, g)
        errs.append(_rel(p, ana))
    # second order: each halving of h cuts the error by ~4
    assert errs[2] < 1e-2
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_fan_converges_to_analytic_smooth_disc(O):
    centre, R = np.array([3.0, -5.0]), 18.0
    views, n_cols, sid, sdd, du = 8, 40, 150.0, 250.0, 1.8
    ana = np.zeros((views, 1, n_cols))
    for k in range(views):
        b = 2 * math.pi * k / views
        S = sid * np.array([math.cos(b), math.sin(b)])
        Cc = -(sdd - sid) * np.array([math.cos(b), math.sin(b)])
        eu = du * np.array([-math.sin(b), math.cos(b)])
        for c in range(n_cols):
            X = Cc + (c - 0.5 * (n_cols - 1)) * eu
            d = (X - S) / np.linalg.norm(X - S)
            r = centre - S
            bdist = abs(r[0] * d[1] - r[1] * d[0])
            ana[k, 0, c] = (4.0 / 3.0) * max(R * R - bdist * bdist, 0.0) ** 1.5 / (R * R)
    errs = []
    for n in (32, 64, 128):
        h = 48.0 / n
        img = W.smooth_ball_volume((1, n, n), (1.0, h, h), (centre[0], centre[1]), R)
        g = O.circular_fan((n, n), (h, h), n_cols, du, views, 2 * math.pi, sid, sdd)
        errs.append(_rel(O.forward(img, g), ana))
    assert errs[2] < 1e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_parallel_converges_to_analytic_smooth_disc(O):
    centre, R = np.array([-4.0, 6.0]), 20.0
    views, n_cols, du = 12, 61, 1.0
    ana = np.zeros((views, 1, n_cols))
    for k in range(views):
        t = math.pi * k / views
        d = np.array([math.cos(t), math.sin(t)])
        e = np.array([-math.sin(t), math.cos(t)])
        for c in range(n_cols):
            off = (c - 0.5 * (n_cols - 1)) * du
            bdist = abs(off - centre @ e)
            ana[k, 0, c] = (4.0 / 3.0) * max(R * R - bdist * bdist, 0.0) ** 1.5 / (R * R)
    errs = []
    for n in (32, 64, 128):
        h = 56.0 / n
        img = W.smooth_ball_volume((1, n, n), (1.0, h, h), (centre[0], centre[1]), R)
        g = O.parallel_2d((n, n), (h, h), n_cols, du, views, math.pi)
        errs.append(_rel(O.forward(img, g), ana))
    assert errs[2] < 1e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


# ------------------------------------------------ P6: equivariance -------


def test_rotating_volume_by_90deg_shifts_views_by_quarter_orbit(O):
    n, views = 20, 16
    vol, _ = W.ellipsoid_phantom_3d(21, shape=(12, n, n), spacing=(1.0, 1.0, 1.0), n_ellipsoids=6)
    g = O.circular_cone((12, n, n), (1.0, 1.0, 1.0), (16, 30), (1.5, 1.5), views, 2 * math.pi, 80.0, 130.0)
    # rotation by +90 deg about z: g(x, y) = f(y, -x); on the centred grid
    # rot[k, j, i] = f[k, n-1-i, j]
    rot = vol.transpose(0, 2, 1)[:, :, ::-1]
    p = O.forward(vol, g)
    pr = O.forward(rot, g)
    shifted = np.roll(p, views // 4, axis=0)  # pr[k] = p[k - views/4]
    assert _rel(pr, shifted) < 1e-12


# ------------------------------------------ P7: back-projection forms ----


def test_bp_of_constant_sinogram_cone_closed_form(O):
    # every voxel projects well inside the detector; sum_k (D/(D - r cos))^2
    # over a full orbit is N D^3 / (D^2 - r^2)^(3/2) (periodic trapezoid).
    shape, sp = (6, 9, 9), (2.0, 2.0, 2.0)
    views, sid, sdd = 48, 300.0, 480.0
    g = O.circular_cone(shape, sp, (40, 40), (1.0, 1.0), views, 2 * math.pi, sid, sdd)
    b = O.backproject(np.ones((views, 40, 40)), g)
    zc, yc, xc = W.voxel_centres(shape, sp)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    r2 = X**2 + Y**2
    ref = views * sid**3 / (sid**2 - r2) ** 1.5
    assert np.abs(b - ref).max() < 1e-12 * ref.max()


def test_bp_of_constant_sinogram_fan_and_parallel(O):
    views, sid, sdd = 40, 200.0, 330.0
    g = O.circular_fan((7, 8), (2.0, 2.0), 60, 1.0, views, 2 * math.pi, sid, sdd)
    b = O.backproject(np.ones((views, 1, 60)), g)
    _, yc, xc = W.voxel_centres((1, 7, 8), (1.0, 2.0, 2.0))
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    ref = views * sid**3 / (sid**2 - X**2 - Y**2) ** 1.5
    assert np.abs(b[0] - ref).max() < 1e-12 * ref.max()
    gp = O.parallel_2d((7, 8), (2.0, 2.0), 40, 1.0, 30, math.pi)
    bp = O.backproject(np.ones((30, 1, 40)), gp)
    assert np.abs(bp - 30.0).max() < 1e-12


def test_bp_of_linear_sinogram_matches_pinhole_model(O):
    """Bilinear interpolation reproduces a linear detector function exactly,
    so BP of p(c, r) = a c + b r + g equals sum_k w_k (a u_k + b v_k + g)
    with u_k, v_k, w_k from an independent central-projection model."""
    shape, sp = (5, 6, 7), (1.5, 1.5, 1.5)
    nv, nu, views, sid, sdd, du, dv = 30, 34, 9, 150.0, 240.0, 1.1, 0.9
    S, C, eu, ev = O.circular_cone_vectors(views, 2 * math.pi, sid, sdd, (dv, du))
    P = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], (nv, nu)) for k in range(views)])
    g = O.cone_geometry(shape, sp, (nv, nu), (dv, du), P)
    a, bb, gg = 0.37, -0.21, 5.0
    cc, rr = np.meshgrid(np.arange(nu), np.arange(nv))
    sino = np.broadcast_to(a * cc + bb * rr + gg, (views, nv, nu)).copy()
    b = O.backproject(sino, g)
    zc, yc, xc = W.voxel_centres(shape, sp)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    pts = np.stack([X, Y, Z], axis=-1)
    ref = np.zeros(shape)
    for k in range(views):
        n = np.cross(eu[k], ev[k])
        n = n / np.linalg.norm(n)
        depth_det = (C[k] - S[k]) @ n
        depth = (pts - S[k]) @ n
        lam = depth_det / depth
        Xd = S[k] + lam[..., None] * (pts - S[k])
        u = (Xd - C[k]) @ eu[k] / (eu[k] @ eu[k]) + 0.5 * (nu - 1)
        v = (Xd - C[k]) @ ev[k] / (ev[k] @ ev[k]) + 0.5 * (nv - 1)
        w = ((0 - S[k]) @ n / depth) ** 2  # depth of the isocentre over depth of X
        ref += w * (a * u + bb * v + gg)
    assert np.abs(b - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("bits", [3, 8])
def test_quantised_bp_matches_map_coordinates_at_snapped_positions(O, bits):
    """The sampler variant of the back-projection rounds both detector
    weights to the 2^-B lattice: linear interpolation of each view at the
    projected position rounded to that lattice, the projection taken from
    an independent central-projection model."""
    shape, sp = (5, 6, 7), (1.5, 1.5, 1.5)
    nv, nu, views, sid, sdd, du, dv = 14, 16, 7, 150.0, 240.0, 1.1, 0.9
    S, C, eu, ev = O.circular_cone_vectors(views, 2 * math.pi, sid, sdd, (dv, du))
    P = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], (nv, nu)) for k in range(views)])
    g = O.cone_geometry(shape, sp, (nv, nu), (dv, du), P)
    sino = np.random.default_rng(19).random((views, nv, nu))
    b = O.backproject(sino, g, weight_bits=bits)
    zc, yc, xc = W.voxel_centres(shape, sp)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    pts = np.stack([X, Y, Z], axis=-1)
    ref = np.zeros(shape)
    for k in range(views):
        n = np.cross(eu[k], ev[k])
        n = n / np.linalg.norm(n)
        depth = (pts - S[k]) @ n
        Xd = S[k] + ((C[k] - S[k]) @ n / depth)[..., None] * (pts - S[k])
        u = _snap((Xd - C[k]) @ eu[k] / (eu[k] @ eu[k]) + 0.5 * (nu - 1), bits)
        v = _snap((Xd - C[k]) @ ev[k] / (ev[k] @ ev[k]) + 0.5 * (nv - 1), bits)
        w = ((0 - S[k]) @ n / depth) ** 2
        vals = map_coordinates(sino[k], np.stack([v.ravel(), u.ravel()]), order=1, mode="grid-constant", cval=0.0)
        ref += w * vals.reshape(shape)
    assert np.abs(b - ref).max() < 1e-11 * np.abs(ref).max()
    assert np.abs(b - O.backproject(sino, g)).max() > 1e-4 * 2.0 ** -bits * np.abs(ref).max()


def test_quantised_bp_exact_ties_round_upward(O):
    """Rays along +x onto a panel shifted by (3/16, 5/16) pixel: voxel
    (i, j, k) projects to (c, r) = (j - 3/16, k - 5/16) exactly, fractions
    13/16 and 11/16, both ties of the 2^-3 lattice, which round up to 7/8
    and 6/8 (unrounded: 13/16 and 11/16)."""
    shape, det = (6, 7, 8), (6, 7)
    P = O.parallel3d_matrix([1.0, 0, 0], [0, 3 / 16, 5 / 16], [0, 1.0, 0], [0, 0, 1.0], det)
    g = O.cone_geometry(shape, (1.0, 1.0, 1.0), det, (1.0, 1.0), P[None], parallel=True)
    img = np.random.default_rng(20).random(det)
    pad = np.pad(img, ((1, 0), (1, 0)))  # row k - 1 and column j - 1 of index 0 are zero
    for bits, (wu, wv) in ((3, (7 / 8, 6 / 8)), (0, (13 / 16, 11 / 16))):
        # rows k, columns j of the detector for voxel (i, j, k); j < 7 = cols, k < 6 = rows
        col = (1 - wu) * pad[:, :-1] + wu * pad[:, 1:]        # [rows + 1][cols]
        e2 = (1 - wv) * col[:-1, :] + wv * col[1:, :]          # [rows][cols] at (k, j)
        expect = np.broadcast_to(e2[:, :, None], shape)
        got = O.backproject(img[None], g, weight_bits=bits)
        assert np.abs(got - expect).max() < 1e-12, bits


# ------------------------------------------------ P8: geometry identities --


def test_cone_matrix_identities(O):
    views, sid, sdd, det, ds = 10, 750.0, 1200.0, (512, 512), (1.0, 1.0)
    S, C, eu, ev = O.circular_cone_vectors(views, 2 * math.pi, sid, sdd, ds)
    for k in range(views):
        P = O.cone_matrix(S[k], C[k], eu[k], ev[k], det)
        assert np.abs(P @ np.append(S[k], 1.0)).max() < 1e-12 * np.abs(P).max()
        U = P @ np.array([0, 0, 0, 1.0])
        assert abs(U[0] / U[2] - 255.5) < 1e-10 and abs(U[1] / U[2] - 255.5) < 1e-10
        assert abs(U[2] - sid / sdd) < 1e-13
        for c, r in ((0, 0), (511, 0), (17, 300), (511, 511)):
            X = C[k] + (c - 255.5) * eu[k] + (r - 255.5) * ev[k]
            U = P @ np.append(X, 1.0)
            assert abs(U[0] / U[2] - c) < 1e-9 and abs(U[1] / U[2] - r) < 1e-9
        # independent pinhole composition K [R | -R S], f = SDD / pixel
        b = 2 * math.pi * k / views
        Rw = np.array([[-math.sin(b), math.cos(b), 0.0], [0.0, 0.0, 1.0], [-math.cos(b), -math.sin(b), 0.0]])
        K = np.array([[sdd / ds[1], 0, 255.5], [0, sdd / ds[0], 255.5], [0, 0, 1.0]])
        Pk = K @ np.hstack([Rw, -(Rw @ S[k])[:, None]])
        mask = np.abs(P) > 1e-9 * np.abs(P).max()
        ratio = Pk[mask] / P[mask]
        assert np.ptp(ratio) < 1e-9 * np.abs(ratio).mean()
        assert np.all(np.abs(Pk[~mask]) < 1e-6 * np.abs(Pk).max())


def test_fan_and_parallel_matrix_identities(O):
    g = O.circular_fan((8, 8), (1.0, 1.0), 101, 0.5, 12, 2 * math.pi, 1000.0, 1500.0)
    for k, P in enumerate(g["P"]):
        b = 2 * math.pi * k / 12
        S = 1000.0 * np.array([math.cos(b), math.sin(b)])
        assert np.abs(P @ np.append(S, 1.0)).max() < 1e-12 * np.abs(P).max()
        U = P @ np.array([0, 0, 1.0])
        assert abs(U[0] / U[1] - 50.0) < 1e-10 and abs(U[1] - 1000.0 / 1500.0) < 1e-13
    gp = O.parallel_2d((8, 8), (1.0, 1.0), 95, 1.0, 90, math.pi)
    for k, P in enumerate(gp["P"]):
        t = math.pi * k / 90
        X = 3.0 * np.array([-math.sin(t), math.cos(t)]) + 7.0 * np.array([math.cos(t), math.sin(t)])
        assert abs(P[0] @ np.append(X, 1.0) - (47.0 + 3.0)) < 1e-12
        assert np.allclose(P[1], [0, 0, 1])


def test_oracle_reproduces_stored_fixture(O):
    import os

    ref = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "parallel2d_64_forward.txt"))
    img, _ = W.ellipse_phantom_2d(1)
    g = O.parallel_2d((64, 64), (1.0, 1.0), 95, 1.0, 90, math.pi)
    p = O.forward(img, g)[::15, 0, :]
    assert np.abs(p - ref).max() <= 1e-13 * np.abs(ref).max()


# -------------------------------------------- splat (transpose of BP) ----


def _splat_cases(O):
    yield "fan2d", (1, 5, 6), O.circular_fan((5, 6), (1.0, 0.8), 9, 0.7, 4, 2 * math.pi, 20.0, 35.0)
    yield "parallel2d", (1, 5, 5), O.parallel_2d((5, 5), (1.0, 1.0), 7, 0.9, 5, math.pi)
    yield "cone3d", (4, 4, 5), O.circular_cone((4, 4, 5), (1.0, 1.0, 0.8), (5, 5), (1.1, 1.0), 3, 2 * math.pi,
                                               25.0, 40.0)
    import workloads as W

    draws = W.perturbation_draws(5, 3)
    args = (3, 2 * math.pi, 25.0, 40.0, (6, 7), (1.0, 1.2), (4, 5, 4), (0.9, 1.0, 1.1))
    P = np.stack([O.cone_matrix(*v, (6, 7)) for v in zip(*O.trajectory_vectors("perturbed", *args, draws=draws))])
    yield "cone3d_perturbed", (4, 5, 4), O.cone_geometry((4, 5, 4), (0.9, 1.0, 1.1), (6, 7), (1.0, 1.2), P)


def test_splat_is_the_transpose_of_backprojection(O):
    """Column i of the explicit back-projection matrix is the back-projection
    of unit sinogram i; column j of its transpose is the splat of unit
    voxel j.  They agree entry by entry (4 geometries)."""
    for name, shape, g in _splat_cases(O):
        nviews = g["P"].shape[0]
        nv, nu = g["det"]
        npix, nvox = nviews * nv * nu, int(np.prod(shape))
        B = np.zeros((nvox, npix))
        for i in range(npix):
            e = np.zeros(npix)
            e[i] = 1.0
            B[:, i] = O.backproject(e.reshape(nviews, nv, nu), g).ravel()
        Bt = np.zeros((npix, nvox))
        for j in range(nvox):
            e = np.zeros(nvox)
            e[j] = 1.0
            Bt[:, j] = O.splat(e.reshape(shape), g).ravel()
        assert np.abs(B).max() > 0.1, name
        assert np.abs(Bt - B.T).max() <= 1e-14 * np.abs(B).max(), name


def test_splat_dot_product(O):
    rng = np.random.default_rng(21)
    g = O.circular_cone((9, 11, 10), (0.7, 0.8, 0.9), (13, 15), (1.0, 1.1), 7, 2 * math.pi, 60.0, 100.0)
    x = rng.standard_normal((9, 11, 10))
    q = rng.standard_normal((7, 13, 15))
    lhs = float(np.sum(O.backproject(q, g) * x))
    rhs = float(np.sum(q * O.splat(x, g)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


def test_splat_deposits_weight_at_the_pinhole_projection(O):
    """A single voxel projecting inside the detector deposits, per view, the
    total weight (W0/W)^2 with its centroid at the projected (u, v): bilinear
    weights sum to one and reproduce linear functions.  (u, v, W) come from
    an independent pinhole camera K [R | t] with focal length SDD / pitch."""
    shape, sp, det, dd, sid, sdd, nviews = (5, 6, 7), (1.0, 1.0, 1.0), (15, 17), (0.9, 0.8), 50.0, 80.0, 6
    g = O.circular_cone(shape, sp, det, dd, nviews, 2 * math.pi, sid, sdd)
    for (k, j, i) in [(2, 3, 3), (0, 0, 6), (4, 5, 1)]:
        e = np.zeros(shape)
        e[k, j, i] = 1.0
        out = O.splat(e, g)
        X = np.array([(i - 3) * sp[2], (j - 2.5) * sp[1], (k - 2) * sp[0]])
        for view in range(nviews):
            b = 2 * math.pi * view / nviews
            # camera frame: depth along -(cos b, sin b, 0) from the source,
            # image axes e_u = (-sin b, cos b, 0), e_v = +z
            Xc = X - sid * np.array([math.cos(b), math.sin(b), 0.0])
            depth = -Xc @ np.array([math.cos(b), math.sin(b), 0.0])
            u = sdd * (Xc @ np.array([-math.sin(b), math.cos(b), 0.0])) / depth / dd[1] + (det[1] - 1) / 2
            v = sdd * Xc[2] / depth / dd[0] + (det[0] - 1) / 2
            w = (sid / depth) ** 2
            img = out[view]
            rr, cc = np.meshgrid(np.arange(det[0]), np.arange(det[1]), indexing="ij")
            assert abs(img.sum() - w) < 1e-12
            assert abs((img * cc).sum() / w - u) < 1e-10 and abs((img * rr).sum() / w - v) < 1e-10


# ------------------------------------------------------------------ FBP ----


@pytest.mark.parametrize("kind", ["ram-lak", "shepp-logan"])
def test_filter_kernel_frequency_response(O, kind):
    """The discrete kernels' frequency responses: |f| (Ram-Lak) and
    sin(pi |f|) / pi (Shepp-Logan), f in cycles per sample (closed forms of
    the infinite sums; the truncation at 4096 taps leaves < 1e-4)."""
    g = O.ramp_kernel(4096, kind)
    full = np.concatenate([g[::-1][:-1], g])
    k = np.arange(-4095, 4096)
    for f in (0.0, 0.05, 0.13, 0.25, 0.37, 0.5):
        h = float(np.sum(full * np.cos(2 * math.pi * f * k)))
        want = abs(f) if kind == "ram-lak" else math.sin(math.pi * abs(f)) / math.pi
        assert abs(h - want) < 1e-4, (kind, f, h, want)


def _disk_interior_exterior(rec, spacing, R):
    n = rec.shape[0]
    c = (np.arange(n) - (n - 1) / 2) * spacing
    yy, xx = np.meshgrid(c, c, indexing="ij")
    r = np.hypot(xx, yy)
    return rec[r < R - 2].mean(), np.abs(rec[(r > R + 2) & (r < c[-1])]).mean()


def test_fbp_parallel_reconstructs_disk(O):
    """FBP of the exact parallel-beam line integrals of a unit disk
    (2 sqrt(R^2 - s^2)) is 1 inside and 0 outside, up to discretization."""
    R, n, ncol, nv = 20.0, 96, 129, 180
    go = O.parallel_2d((n, n), (0.5, 0.5), ncol, 0.5, nv, math.pi)
    s = (np.arange(ncol) - (ncol - 1) / 2) * 0.5
    p = np.where(np.abs(s) < R, 2 * np.sqrt(np.maximum(R * R - s * s, 0.0)), 0.0)
    inside, outside = _disk_interior_exterior(O.fbp(np.tile(p, (nv, 1, 1)), go, 0.5)[0], 0.5, R)
    assert abs(inside - 1.0) < 0.01 and outside < 0.01, (inside, outside)


def test_fbp_fan_reconstructs_disk(O):
    """Fan-beam FBP (cosine weights, kernel at the axis pitch du SID/SDD,
    (W0/W)^2 back-projection) of a centred unit disk: the ray at detector
    coordinate u passes SID sin(atan(u / SDD)) from the centre."""
    R, n, ncol, nv, sid, sdd, du = 20.0, 96, 181, 240, 400.0, 600.0, 0.5
    go = O.circular_fan((n, n), (0.5, 0.5), ncol, du, nv, 2 * math.pi, sid, sdd)
    u = (np.arange(ncol) - (ncol - 1) / 2) * du
    dist = sid * np.sin(np.abs(np.arctan(u / sdd)))
    p = np.where(dist < R, 2 * np.sqrt(np.maximum(R * R - dist * dist, 0.0)), 0.0)
    inside, outside = _disk_interior_exterior(O.fbp(np.tile(p, (nv, 1, 1)), go, du * sid / sdd)[0], 0.5, R)
    assert abs(inside - 1.0) < 0.01 and outside < 0.01, (inside, outside)


def test_fdk_reconstructs_ball_central_slice(O):
    """Cone-beam FDK of a centred unit ball: exact line integrals from the
    ray-to-centre distance |S x d| / |d|; the central slice is 1 inside and
    0 outside, up to discretization."""
    nz, n, R, nvr, nuc, dd, sid, sdd, nviews = 48, 64, 10.0, 64, 96, 0.75, 400.0, 600.0, 120
    go = O.circular_cone((nz, n, n), (0.5, 0.5, 0.5), (nvr, nuc), (dd, dd), nviews, 2 * math.pi, sid, sdd)
    sino = np.zeros((nviews, nvr, nuc))
    uu, vv = np.meshgrid(np.arange(nuc, dtype=np.float64), np.arange(nvr, dtype=np.float64))
    pix = np.stack([uu.ravel(), vv.ravel(), np.ones(uu.size)])
    for k in range(nviews):
        Q = go["P"][k][:, :3]
        S = -np.linalg.solve(Q, go["P"][k][:, 3])
        d = np.linalg.solve(Q, pix)
        dist = np.linalg.norm(np.cross(S[None, :], d.T), axis=1) / np.linalg.norm(d, axis=0)
        sino[k] = np.where(dist < R, 2 * np.sqrt(np.maximum(R * R - dist ** 2, 0.0)), 0.0).reshape(nvr, nuc)
    rec = O.fbp(sino, go, dd * sid / sdd)
    inside, outside = _disk_interior_exterior(rec[nz // 2 - 1:nz // 2 + 1].mean(axis=0), 0.5, R)
    assert abs(inside - 1.0) < 0.01 and outside < 0.01, (inside, outside)


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def test_cosine_weights_are_cosines_to_the_detector_normal(O):
    """FDK's pre-weight is the cosine of the angle between a pixel's ray
    and the detector normal.  Computed here straight from the trajectory
    vectors -- pixel X = C + (c - (cols-1)/2) e_u + (r - (rows-1)/2) e_v,
    ray X - S, normal e_u x e_v -- and, for the circular orbit, from the
    closed form SDD / sqrt(SDD^2 + u^2 + v^2) in centred detector mm.  A
    wide fan (half-angle 39 deg) and a tilted, rotated, off-centre panel make
    a weight of 1, cos^2 or 1/cos differ by far more than the tolerance."""
    rows, cols, dv, du, sid, sdd, nviews = 24, 401, 0.7, 1.6, 300.0, 400.0, 5
    g = O.circular_cone((8, 8, 8), (1.0, 1.0, 1.0), (rows, cols), (dv, du), nviews, 2 * math.pi, sid, sdd)
    w = O.cosine_weights(g)
    uc = (np.arange(cols) - (cols - 1) / 2) * du
    vc = (np.arange(rows) - (rows - 1) / 2) * dv
    ref = sdd / np.sqrt(sdd ** 2 + uc[None, :] ** 2 + vc[:, None] ** 2)
    assert ref.min() < 0.83  # the weight matters at the panel's edge
    for k in range(nviews):
        assert np.abs(w[k] - ref).max() < 1e-13
    # a panel tilted out of its plane, rotated in it and shifted off-centre
    rng = np.random.default_rng(11)
    for k in range(4):
        S = np.array([sid, 0.0, 0.0]) + rng.normal(0, 5, 3)
        C = np.array([sid - sdd, 0.0, 0.0]) + rng.normal(0, 20, 3)
        a, b = rng.uniform(-0.4, 0.4, 2)
        eu = du * _unit([math.sin(a), math.cos(a), 0.3 * b])
        ev = dv * _unit(np.cross(_unit([math.cos(a) * math.cos(b), -math.sin(a), math.sin(b)]), eu / du))
        P = O.cone_matrix(S, C, eu, ev, (rows, cols))
        gk = O.cone_geometry((8, 8, 8), (1.0, 1.0, 1.0), (rows, cols), (dv, du), P[None])
        cc, rr = np.meshgrid(np.arange(cols, dtype=float), np.arange(rows, dtype=float))
        X = C + (cc[..., None] - (cols - 1) / 2) * eu + (rr[..., None] - (rows - 1) / 2) * ev
        d = X - S
        n = np.cross(eu, ev)
        cosv = np.abs(d @ n) / (np.linalg.norm(d, axis=-1) * np.linalg.norm(n))
        assert np.abs(O.cosine_weights(gk)[0] - cosv).max() < 1e-12
    # fan: SDD / sqrt(SDD^2 + u^2); parallel: ones
    gf = O.circular_fan((8, 8), (1.0, 1.0), cols, du, nviews, 2 * math.pi, sid, sdd)
    wf = O.cosine_weights(gf)
    assert np.abs(wf[:, 0, :] - sdd / np.sqrt(sdd ** 2 + uc ** 2)[None, :]).max() < 1e-13
    gp = O.parallel_2d((8, 8), (1.0, 1.0), cols, du, nviews, math.pi)
    assert np.array_equal(O.cosine_weights(gp), np.ones((nviews, 1, cols)))


def _radial_max_dev(rec, spacing, R):
    n = rec.shape[-1]
    c = (np.arange(n) - (n - 1) / 2) * spacing
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return float(np.abs(rec[np.hypot(xx, yy) < R - 3] - 1.0).max())


def test_fan_fdk_short_source_distance_reconstructs_disk(O):
    """A short-SDD fan (SID 100, SDD 150) around a centred unit disk of
    radius 45 mm: the disk's edge rays leave the central ray at 26.7 deg,
    where the cosine pre-weight is 0.89.  The FBP is 1 to within 1% on the
    whole interior; without the weight (or squared, or inverted) it misses by
    more than 8% somewhere inside.  Exact line integrals: the ray at detector
    coordinate u passes SID sin(atan(u / SDD)) from the centre."""
    R, n, ncol, nv, sid, sdd, du = 45.0, 200, 401, 360, 100.0, 150.0, 0.5
    go = O.circular_fan((n, n), (0.5, 0.5), ncol, du, nv, 2 * math.pi, sid, sdd)
    u = (np.arange(ncol) - (ncol - 1) / 2) * du
    dist = sid * np.sin(np.abs(np.arctan(u / sdd)))
    p = np.where(dist < R, 2 * np.sqrt(np.maximum(R * R - dist * dist, 0.0)), 0.0)
    rec = O.fbp(np.tile(p, (nv, 1, 1)), go, du * sid / sdd)[0]
    assert _radial_max_dev(rec, 0.5, R) < 0.01


def test_cone_fdk_short_source_distance_reconstructs_ball(O):
    """Cone-beam FDK with SID 100, SDD 150 of a centred unit ball of radius
    42 mm (edge rays 24.8 deg off the central ray): its central slices are 1
    to within 1%.  The line integrals are exact chords, from each ray's
    distance to the centre |S x d| / |d| with S and d from the matrices."""
    nz, n, R, nvr, nuc, dd, sid, sdd, nviews = 4, 184, 42.0, 9, 361, 0.5, 100.0, 150.0, 360
    go = O.circular_cone((nz, n, n), (0.5, 0.5, 0.5), (nvr, nuc), (dd, dd), nviews, 2 * math.pi, sid, sdd)
    sino = np.zeros((nviews, nvr, nuc))
    uu, vv = np.meshgrid(np.arange(nuc, dtype=np.float64), np.arange(nvr, dtype=np.float64))
    pix = np.stack([uu.ravel(), vv.ravel(), np.ones(uu.size)])
    for k in range(nviews):
        Q = go["P"][k][:, :3]
        S = -np.linalg.solve(Q, go["P"][k][:, 3])
        d = np.linalg.solve(Q, pix)
        dist = np.linalg.norm(np.cross(S[None, :], d.T), axis=1) / np.linalg.norm(d, axis=0)
        sino[k] = np.where(dist < R, 2 * np.sqrt(np.maximum(R * R - dist ** 2, 0.0)), 0.0).reshape(nvr, nuc)
    rec = O.fbp(sino, go, dd * sid / sdd)
    assert _radial_max_dev(rec[1:3].mean(axis=0), 0.5, R) < 0.01


# ---------------------------------------------- trajectory generators ----


def _sources(P):
    return np.stack([-np.linalg.solve(p[:, :3], p[:, 3]) for p in P])


def test_helical_trajectory_has_the_requested_pitch(O):
    """Helical pitch = table feed per turn / collimation at the isocentre.
    The feed comes from the sources of the composed matrices; the
    collimation is the length of the rotation axis whose points project
    between the outer edges of the first and last detector rows
    (v = -1/2 and v = rows - 1/2), solved from the matrix of one view."""
    rows, cols, dv, du, sid, sdd, N = 64, 48, 1.5, 1.0, 750.0, 1200.0, 90
    for pitch in (0.5, 1.25):
        S, C, eu, ev = O.trajectory_vectors("helical", N, 2 * math.pi, sid, sdd, (rows, cols), (dv, du),
                                            (32, 32, 32), (1.0, 1.0, 1.0), pitch=pitch)
        P = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], (rows, cols)) for k in range(N)])
        Sz = _sources(P)[:, 2]
        feed = (Sz[-1] - Sz[0]) * N / (N - 1)
        assert np.allclose(np.diff(Sz), feed / N, rtol=0, atol=1e-9)

        def z_at(p, v):  # axis point (0, 0, z) with V / W = v
            return -(p[1, 3] - v * p[2, 3]) / (p[1, 2] - v * p[2, 2])

        col = abs(z_at(P[7], rows - 0.5) - z_at(P[7], -0.5))
        assert abs(feed / col - pitch) < 1e-9
        assert abs(0.5 * (Sz[0] + Sz[-1] + feed / N)) < 1e-9  # one turn centred on z = 0


def test_sinusoidal_trajectory_amplitude_and_frequency(O):
    """The sinusoidal orbit's source height is a pure sinusoid of two
    periods per turn and amplitude nz sz / 4 (read from the matrices'
    sources, N divisible by 8 so the samples reach the peaks); the detector
    follows the source: its centre pixel stays at the source's height."""
    N, rows, cols, nz, sz = 96, 32, 40, 40, 0.8
    S, C, eu, ev = O.trajectory_vectors("sinusoidal", N, 2 * math.pi, 750.0, 1200.0, (rows, cols), (1.0, 1.0),
                                        (nz, 16, 16), (sz, 1.0, 1.0))
    P = np.stack([O.cone_matrix(S[k], C[k], eu[k], ev[k], (rows, cols)) for k in range(N)])
    Sz = _sources(P)[:, 2]
    assert abs(0.5 * (Sz.max() - Sz.min()) - nz * sz / 4) < 1e-9
    spec = np.abs(np.fft.rfft(Sz))
    assert np.argmax(spec) == 2 and np.delete(spec, 2).max() < 1e-9 * spec[2]
    for k in range(N):
        # the ray of the centre pixel runs level: the panel's centre sits at
        # the source's height
        d = np.linalg.solve(P[k][:, :3], [(cols - 1) / 2, (rows - 1) / 2, 1.0])
        assert abs(d[2]) < 1e-9 * np.linalg.norm(d)


def test_perturbed_trajectory_statistics(O):
    """The perturbed orbit differs from the circular one by i.i.d. N(0, 0.5 mm)
    source shifts and an N(0, 0.5 deg) in-panel detector rotation; both are
    read back from the composed matrices (sources, and the angle of the
    column direction e_u = first column of the inverse 3x3 block)."""
    import workloads as W

    N, rows, cols = 2000, 16, 16
    args = (N, 2 * math.pi, 750.0, 1200.0, (rows, cols), (1.0, 1.0), (16, 16, 16), (1.0, 1.0, 1.0))
    P0 = [O.cone_matrix(*v, (rows, cols)) for v in zip(*O.trajectory_vectors("circular", *args))]
    Pp = [O.cone_matrix(*v, (rows, cols)) for v in zip(*O.trajectory_vectors("perturbed", *args,
                                                                            draws=W.perturbation_draws(7, N)))]
    dS = _sources(Pp) - _sources(P0)
    assert abs(dS.std() - 0.5) < 0.02 and abs(dS.mean()) < 0.02
    ang = []
    for p0, p1 in zip(P0, Pp):
        e0 = np.linalg.inv(p0[:, :3])[:, 0]
        e1 = np.linalg.inv(p1[:, :3])[:, 0]
        ang.append(math.atan2(np.linalg.norm(np.cross(e0, e1)), e0 @ e1))
    assert abs(math.degrees(np.sqrt(np.mean(np.square(ang)))) - 0.5) < 0.03
    # the rotation keeps the panel's pixel grid square: e_u stays normal to e_v
    for p1 in Pp:
        M = np.linalg.inv(p1[:, :3])
        assert abs(M[:, 0] @ M[:, 1]) < 1e-12 * np.linalg.norm(M[:, 0]) * np.linalg.norm(M[:, 1])


# ------------------------------------------------- artifact simulation ----


def test_philox_matches_numpy_bit_generator(O):
    """numpy's Philox bit generator is Philox4x64-10; it steps its counter
    before each block, so its first four raw words are the block at
    counter + 1.  Cases include a carry out of the low counter word."""
    for key, ctr in [((0, 0), (0, 0, 0, 0)), ((123, 456), (7, 0, 0, 0)),
                     ((2 ** 64 - 1, 5), (2 ** 64 - 1, 3, 0, 9)), ((0xDEADBEEF, 0), (41, 0, 0, 0))]:
        raw = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64)).random_raw(4)
        c0 = (ctr[0] + 1) % 2 ** 64
        c1 = (ctr[1] + (ctr[0] + 1) // 2 ** 64) % 2 ** 64
        out = O.philox4x64([np.uint64(c0), np.uint64(c1), np.uint64(ctr[2]), np.uint64(ctr[3])],
                           [np.uint64(key[0]), np.uint64(key[1])])
        assert [int(v) for v in out] == [int(v) for v in raw]


def test_mulhilo64_matches_python_integers(O):
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2 ** 63, 200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, 200, dtype=np.uint64) * np.uint64(2)
    hi, lo = O._mulhilo64(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


def test_gaussian_noise_is_standard_normal(O):
    """10^6 draws: Kolmogorov-Smirnov against N(0, 1), and each of the four
    words of a block (cosine and sine halves of both pairs) separately."""
    from scipy import stats

    z = O.standard_normal_at(np.arange(1_000_000), seed=2024)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    for q in range(4):
        assert stats.kstest(z[q::4], "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5e-3 and abs(z.std() - 1.0) < 5e-3
    # pairs from one block are uncorrelated, and other seeds differ
    assert abs(np.corrcoef(z[0::4], z[1::4])[0, 1]) < 5e-3
    assert not np.array_equal(z[:100], O.standard_normal_at(np.arange(100), seed=2025))
    x = np.full((3, 5, 7), 2.0)
    y = O.gaussian_noise(x, 0.5, 3.0, seed=9)
    assert np.allclose((y - 2.5) / 3.0, O.standard_normal_at(np.arange(105), 9).reshape(3, 5, 7))


def test_ring_artifacts_touch_only_the_chosen_columns(O):
    rng = np.random.default_rng(1)
    s = rng.random((2, 6, 3, 10)).astype(np.float32)
    r = O.ring_artifacts(s, [7, 2, 7], 0.0, 1, 4)
    changed = np.argwhere(r != s)
    assert set(map(tuple, changed[:, [1, 3]])) == {(v, c) for v in (1, 2, 3) for c in (2, 7)}
    assert np.all(r[:, 1:4, :, [2, 7]] == 0.0)


def test_detector_jitter_shifts_rows(O):
    """Shifts are uniform over -m .. m (chi-square on 60000 rows) and each
    row equals np.roll of the input with the wrapped part zeroed."""
    from scipy import stats

    s = O.jitter_shifts(60000, 3, seed=8)
    counts = np.bincount(s + 3, minlength=7)
    assert s.min() == -3 and s.max() == 3
    assert stats.chisquare(counts).pvalue > 1e-3
    x = np.random.default_rng(2).random((2, 3, 4, 9))
    y = O.detector_jitter(x, 2, seed=4)
    sh = O.jitter_shifts(24, 2, seed=4)
    for g, row in enumerate(x.reshape(-1, 9)):
        ref = np.roll(row, sh[g])
        if sh[g] > 0:
            ref[:sh[g]] = 0.0
        elif sh[g] < 0:
            ref[sh[g]:] = 0.0
        assert np.array_equal(y.reshape(-1, 9)[g], ref)
    assert np.array_equal(O.detector_jitter(x, 0, seed=4), x)


def test_gantry_blur_matches_map_coordinates(O):
    """Each tap equals scipy's order-1 map_coordinates with zero padding
    (grid-constant); one tap is the identity; a view at angle 0 blurs along
    the columns only, so a constant row stays constant away from its ends."""
    rng = np.random.default_rng(4)
    s = rng.random((2, 3, 7, 9))
    got = O.gantry_blur(s, 0.3, 0.9, 5)
    rr, cc = np.meshgrid(np.arange(7.0), np.arange(9.0), indexing="ij")
    for b in range(2):
        for k in range(3):
            a = 0.3 + 0.9 * k
            ref = sum(map_coordinates(s[b, k], [rr + t * math.sin(a), cc + t * math.cos(a)], order=1,
                                      mode="grid-constant", cval=0.0) for t in range(-2, 3)) / 5
            assert np.abs(got[b, k] - ref).max() < 1e-12
    assert np.abs(O.gantry_blur(s, 0.3, 0.9, 1) - s).max() < 1e-15
    flat = np.ones((1, 1, 4, 12))
    g0 = O.gantry_blur(flat, 0.0, 0.0, 3)
    assert np.abs(g0[..., 1:-1] - 1.0).max() < 1e-15 and np.abs(g0[..., 0] - 2.0 / 3.0).max() < 1e-15


def test_gantry_blur_single_row_uses_the_column_component(O):
    """A single-row projection has no row direction: the turned kernel acts
    along the row through its column component, so a view at pi/2 is
    unchanged, a constant row stays constant away from its ends at every
    angle (no darkening by taps leaving the row), and a view at angle a
    equals zero-padded np.interp samples at c + t cos a."""
    rng = np.random.default_rng(6)
    s = rng.random((2, 4, 1, 30))
    got = O.gantry_blur(s, 0.0, math.pi / 2, 5)
    assert np.abs(got[:, 1] - s[:, 1]).max() < 1e-15 and np.abs(got[:, 3] - s[:, 3]).max() < 1e-12
    flat = O.gantry_blur(np.ones((1, 5, 1, 40)), 0.1, 0.6, 7)
    assert np.abs(flat[..., 4:-4] - 1.0).max() < 1e-12
    a = 0.7
    one = O.gantry_blur(s[:, :1], a, 0.0, 5)
    c, cp = np.arange(30.0), np.arange(-1.0, 31.0)
    for b in range(2):
        row = np.pad(s[b, 0, 0], 1)
        ref = sum(np.interp(c + t * math.cos(a), cp, row, left=0.0, right=0.0) for t in range(-2, 3)) / 5
        assert np.abs(one[b, 0, 0] - ref).max() < 1e-12
