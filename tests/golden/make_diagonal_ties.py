"""Writes ``diagonal_ties.json``: explicit projection matrices whose rays tie
exactly between the x and y axes (|delta_x| = |delta_y|), the one place where
the ray-driven projector's choice of dominant axis is not decided by the
geometry alone (the reading is: ties go to the lowest axis, x).

These are inputs, not expected values.  Every matrix is built with exact
rational arithmetic from a direction matrix N (the ray of pixel (u, v) is
N (u, v, 1)) whose determinant is a power of two, so P = N^-1 [I | -S] has
dyadic entries with few bits.  Any cofactor inverse in FP64 then recovers N
exactly, and both sides of a parity test see bit-identical ray directions:
a tie on one side is a tie on the other.  Run from the repository root:

    python tests/golden/make_diagonal_ties.py
"""
import json
import os
from fractions import Fraction as Fr

HERE = os.path.dirname(os.path.abspath(__file__))


def inv3(m):
    a, b, c, d, e, f, g, h, i = [Fr(x) for r in m for x in r]
    det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g)
    adj = [[e * i - f * h, c * h - b * i, b * f - c * e],
           [f * g - d * i, a * i - c * g, c * d - a * f],
           [d * h - e * g, b * g - a * h, a * e - b * d]]
    return [[x / det for x in r] for r in adj], det


def inv2(m):
    (a, b), (c, d) = [[Fr(x) for x in r] for r in m]
    det = a * d - b * c
    return [[d / det, -b / det], [-c / det, a / det]], det


def dyadic(x):
    x = Fr(x)
    den = x.denominator
    assert den & (den - 1) == 0, f"{x} is not dyadic"
    return float(x)


def cone_view(N, S):
    M, det = inv3(N)
    assert abs(det.numerator) & (abs(det.numerator) - 1) == 0 and det.denominator == 1
    p4 = [-sum(M[r][c] * Fr(S[c]) for c in range(3)) for r in range(3)]
    return [[dyadic(M[r][c]) for c in range(3)] + [dyadic(p4[r])] for r in range(3)]


def fan_view(N, S):
    M, det = inv2(N)
    assert abs(det.numerator) & (abs(det.numerator) - 1) == 0 and det.denominator == 1
    p3 = [-sum(M[r][c] * Fr(S[c]) for c in range(2)) for r in range(2)]
    return [[dyadic(M[r][c]) for c in range(2)] + [dyadic(p3[r])] for r in range(2)]


def main():
    d, cm, rm = 256, 32, 32
    out = {}
    # cone: ray of pixel (u, v) is (d + cm - u, d - cm + u, v - rm) from the
    # source (-200, -200, 0); column cm runs along the diagonal x = y.  The
    # second view mirrors x (source (200, -200, 0), ray (u - d - cm, ...)).
    N1 = [[-1, 0, d + cm], [1, 0, d - cm], [0, 1, -rm]]
    N2 = [[1, 0, -(d + cm)], [1, 0, d - cm], [0, 1, -rm]]
    out["cone_diagonal"] = dict(
        ndim=3, beam="cone", vol_shape=[32, 32, 32], vol_spacing=[1.0, 1.0, 1.0], det_shape=[64, 64],
        P=[cone_view(N1, (-200, -200, 0)), cone_view(N2, (200, -200, 0))], tie_column=cm,
    )
    # fan: the same in the plane, image 40 x 48 (ny, nx)
    F1 = [[-1, d + cm], [1, d - cm]]
    F2 = [[1, -(d + cm)], [1, d - cm]]
    out["fan_diagonal"] = dict(
        ndim=2, beam="fan", vol_shape=[1, 40, 48], vol_spacing=[1.0, 1.0, 1.0], det_shape=[1, 64],
        P=[fan_view(F1, (-200, -200)), fan_view(F2, (200, -200))], tie_column=cm,
    )
    # 3-D parallel beam along (1, 1, 1/4): every ray ties
    out["parallel3d_diagonal"] = dict(
        ndim=3, beam="parallel", vol_shape=[32, 32, 32], vol_spacing=[1.0, 1.0, 1.0], det_shape=[48, 64],
        P=[[[1.0, -1.0, 0.0, 32.0], [-0.125, -0.125, 1.0, 24.0], [0.0, 0.0, 0.0, 1.0]],
           [[1.0, 1.0, 0.0, 32.0], [0.125, -0.125, 1.0, 24.0], [0.0, 0.0, 0.0, 1.0]]],
        tie_column=None,
    )
    # 2-D parallel beam along (1, 1) and (1, -1): every ray ties
    out["parallel2d_diagonal"] = dict(
        ndim=2, beam="parallel", vol_shape=[1, 40, 48], vol_spacing=[1.0, 1.0, 1.0], det_shape=[1, 96],
        P=[[[1.0, -1.0, 47.5], [0.0, 0.0, 1.0]], [[1.0, 1.0, 47.5], [0.0, 0.0, 1.0]]],
        tie_column=None,
    )
    with open(os.path.join(HERE, "diagonal_ties.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
