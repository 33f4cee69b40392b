"""Exact pin of the oracle's edge points (eq. intersection): on a cube edge
the trilinear interpolant of eq. linear1 is linear, so for corner values taken
from a trilinear field the crossing of g = c is the field's own root on that
edge.  With dyadic coefficients and lattice coordinates every corner value is
exact in double precision, and the root is compared with exact rational
arithmetic; the set of crossing edges is enumerated independently."""
from fractions import Fraction

import numpy as np

import oracle

CORNER = [(v & 1, (v >> 1) & 1, (v >> 2) & 1) for v in range(8)]


def field(coef, X, Y, Z):
    """sum over subsets e of {x, y, z} of coef[e] * prod x_i (trilinear)."""
    t = [1, X, Y, X * Y, Z, X * Z, Y * Z, X * Y * Z]
    return sum(cf * ti for cf, ti in zip(coef, t))


def leaves_and_values(coef, origin, h0, K):
    # level-2 cubes of one block and level-3 cubes of a disjoint one
    cubes = [(2, i, j, k) for i in range(8, 14) for j in range(8, 14) for k in range(8, 14)]
    cubes += [(3, i, j, k) for i in range(30, 40) for j in range(31, 39) for k in range(30, 37)]
    ijk = np.array([c[1:] for c in cubes], dtype=np.int32)
    level = np.array([c[0] for c in cubes], dtype=np.uint8)
    cp = np.zeros((len(cubes), 8))
    for q, (lev, i, j, k) in enumerate(cubes):
        h = h0 / 2 ** lev
        for v, (dx, dy, dz) in enumerate(CORNER):
            X, Y, Z = (origin[0] + (i + dx) * h, origin[1] + (j + dy) * h, origin[2] + (k + dz) * h)
            cp[q, v] = field(coef, X, Y, Z)
    return cubes, ijk, level, cp


def test_edge_points_are_the_exact_roots_of_a_trilinear_field():
    origin, h0, K = np.array([-8.0, -6.0, -4.0]), 2.0, 3
    # dyadic coefficients: all corner values exact in double precision
    coef = [Fraction(3, 4), Fraction(1, 8), Fraction(-1, 16), Fraction(1, 32),
            Fraction(3, 64), Fraction(-1, 64), Fraction(1, 128), Fraction(1, 256)]
    c = 0.883
    cubes, ijk, level, cp = leaves_and_values([float(x) for x in coef], origin, h0, K)
    for q, (lev, i, j, k) in enumerate(cubes):   # exactness of the inputs
        h = Fraction(h0) / 2 ** lev
        for v, (dx, dy, dz) in enumerate(CORNER):
            X = Fraction(origin[0]) + (i + dx) * h
            Y = Fraction(origin[1]) + (j + dy) * h
            Z = Fraction(origin[2]) + (k + dz) * h
            assert Fraction(cp[q, v]) == field(coef, X, Y, Z)
    res = oracle.extract(ijk, level, cp, c, origin, h0, K, conf=5)
    assert res.n_vert > 100
    # expected crossing edges, one per key
    want = {}
    hmin = h0 / 2 ** K
    for q, (lev, i, j, k) in enumerate(cubes):
        sh = K - lev
        for axis in range(3):
            for v0 in range(8):
                if (v0 >> axis) & 1:
                    continue
                v1 = v0 | (1 << axis)
                f0, f1 = cp[q, v0], cp[q, v1]
                if (f0 >= c) == (f1 >= c):
                    continue
                d = CORNER[v0]
                X, Y, Z = (i + d[0]) << sh, (j + d[1]) << sh, (k + d[2]) << sh
                key = (5 << 53) | (lev << 50) | (axis << 48) | (X << 32) | (Y << 16) | Z
                want[key] = (Fraction(c) - Fraction(f0)) / (Fraction(f1) - Fraction(f0))
    assert sorted(want) == [int(k) for k in res.vkey]
    for key, t, xyz in zip(res.vkey, res.vt, res.vxyz):
        t_exact = want[int(key)]
        # the root of the field along the edge, to the last bits of t
        assert abs(Fraction(t) - t_exact) <= Fraction(2, 2 ** 52) * abs(t_exact) + Fraction(1, 2 ** 1074)
        # and the point lies on the field's level set
        g = field(coef, *[Fraction(x) for x in xyz])
        assert abs(float(g - Fraction(c))) <= 1e-15
        assert 0.0 <= t <= 1.0
    _ = hmin
