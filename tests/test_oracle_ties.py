"""Exact dominant-axis ties in the oracle (CPU).

The ray-driven projector integrates along the planes of the ray's dominant
index axis; when |delta_x| = |delta_y| exactly the geometry does not decide,
and the reading is that the lowest axis (x) wins.  On a diagonal the two
choices give the same sum in exact arithmetic: the x-planes' crossings
interpolate along y with weights (1 - f, f), the y-planes' crossings along x
with weights (f, 1 - f), and after re-indexing both are the same weighted
sum over the same lattice points (zero padding, all planes); the length per
plane s_a |D| / |D_a| is the same for a = x and a = y because
|D_x| / s_x = |D_y| / s_y.  So A has no jump at a tie, and what a projector
must get right there is that its adjoint counts every tie ray exactly once
(one pass axis, not both).

These pins check, on the exact-tie geometries of ``golden/diagonal_ties.json``,
that stretching the x spacing by 1 -/+ 2^-30 (x, then y, strictly dominant
on the former tie rays) moves every ray by < 1e-7 relative, and that the
oracle's adjoint is still the transpose there (dot test).
"""
import numpy as np
import pytest

import oracle as O
import tie_cases as T


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("name", T.NAMES)
def test_tie_rays_are_continuous_in_the_axis_choice(name):
    c = T.load(name)
    vol = T.phantom(c)
    base = O.forward(vol, T.oracle_geometry(O, c))
    m = T.tie_mask(c)
    assert np.linalg.norm(base[m]) > 0.1 * np.linalg.norm(base) / np.sqrt(m.size / m.sum())
    for f in (1.0 - 2.0 ** -30, 1.0 + 2.0 ** -30):
        moved = O.forward(vol, T.oracle_geometry(O, c, f))
        assert _rel(moved[m], base[m]) < 1e-7
        assert _rel(moved, base) < 1e-7


@pytest.mark.parametrize("name", T.NAMES)
def test_tie_adjoint_dot(name):
    c = T.load(name)
    g = T.oracle_geometry(O, c)
    rng = np.random.default_rng(5)
    x = rng.random(tuple(c["vol_shape"]))
    y = rng.random((len(c["P"]),) + tuple(c["det_shape"]))
    ax = O.forward(x, g)
    aty = O.adjoint(y, g)
    lhs, rhs = float((ax * y).sum()), float((x * aty).sum())
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(ax) * np.linalg.norm(y)
