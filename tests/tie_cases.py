"""Loads the exact-tie geometries of ``golden/diagonal_ties.json`` (explicit
projection matrices whose pixel rays have |delta_x| = |delta_y| exactly) for
the oracle and for the product binding, plus their phantoms."""
import json
import os

import numpy as np

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
NAMES = ["cone_diagonal", "fan_diagonal", "parallel3d_diagonal", "parallel2d_diagonal"]


def load(name):
    with open(os.path.join(HERE, "golden", "diagonal_ties.json")) as f:
        return json.load(f)[name]


def oracle_geometry(O, c, sx_factor=1.0):
    """Oracle geometry; ``sx_factor`` stretches the x spacing (tie breaking)."""
    sp = list(c["vol_spacing"])
    sp[2] *= sx_factor
    par = c["beam"] == "parallel"
    P = np.asarray(c["P"], dtype=np.float64)
    if c["ndim"] == 3:
        return O.cone_geometry(c["vol_shape"], sp, c["det_shape"], (1.0, 1.0), P, parallel=par)
    return O.image_geometry(c["vol_shape"][1:], sp[1:], c["det_shape"][1], P, parallel=par)


def product_geometry(pn, c):
    return pn.Geometry(c["ndim"], c["beam"], tuple(c["vol_shape"]), tuple(c["vol_spacing"]), tuple(c["det_shape"]),
                       np.asarray(c["P"], dtype=np.float64))


def phantom(c, seed=606):
    shp, sp = tuple(c["vol_shape"]), tuple(c["vol_spacing"])
    if c["ndim"] == 3:
        return W.ellipsoid_phantom_3d(seed, shp, sp, 8)[0]
    return W.ellipse_phantom_2d(seed, shp[1:], sp[1:])[0]


def tie_mask(c):
    """Boolean [views, rows, cols]: the pixels whose rays tie."""
    n_views = len(c["P"])
    m = np.zeros((n_views,) + tuple(c["det_shape"]), dtype=bool)
    if c["tie_column"] is None:
        m[:] = True
    else:
        m[:, :, c["tie_column"]] = True
    return m
