"""Pins for the oracle's Stage-2 mesh functions (oracle/mesh.py) against
closed forms and hand-built meshes.  CPU only.

* Face pairing: the brute-force connectivity of {g >= c} on a bilinear face
  agrees with the classical saddle-value criterion (the two corners at or
  above c are connected through the face iff the bilinear's value at its
  saddle point is >= c), away from ties.
* Loops: a planar field crossing four parallel edges gives one loop of four;
  every crossing edge lies in exactly two face segments.
* The mesh checker on meshes whose answers are known: a tetrahedron, an
  octahedron and a torus (closed, Euler characteristic 2, 2 and 0, exact
  volumes), a tetrahedron with a face missing (three boundary edges), a
  flipped face (misoriented edges), two tetrahedra sharing one vertex (one
  vertex whose neighbourhood is two loops), two crossing triangles.
* Condition (c) is decided exactly: a vertex on a face or an edge meets it,
  one smallest double off the plane it does not (or crosses), coplanar
  pairs overlap, touch or stay apart as built, and two slivers separated by
  a lattice plane, which tolerance-based tests report as crossing, do not
  meet.
* Closing open faces: on a sampled field whose crossing cubes form one
  face-connected set, dropping most of them and closing gives back exactly
  the dropped cubes with their values.
"""
import numpy as np
import pytest

from oracle import mesh as om


def test_face_pairing_matches_saddle_criterion():
    rng = np.random.default_rng(5)
    c, n = 1.0, 0
    while n < 60:
        hi = c + rng.uniform(0.05, 1.0, 2)
        lo = c - rng.uniform(0.05, 1.0, 2)
        if rng.random() < 0.5:
            F = [[hi[0], lo[0]], [lo[1], hi[1]]]   # (0,0), (1,1) high
        else:
            F = [[lo[0], hi[0]], [hi[1], lo[1]]]   # (0,1), (1,0) high
        h00, h01, h10, h11 = F[0][0], F[0][1], F[1][0], F[1][1]
        sad = (h00 * h11 - h10 * h01) / (h00 + h11 - h10 - h01)
        if abs(sad - c) < 0.05:
            continue
        assert om.high_corners_joined(F, c) == (sad >= c), (F, sad)
        n += 1


def test_planar_field_one_loop_of_four():
    # g = c + (x - 0.4): the four edges along x cross, one loop around them
    f = [1.0 + ((v & 1) - 0.4) for v in range(8)]
    segs = om.leaf_face_segments(f, 1.0)
    loops = om.loops_from_segments(segs)
    assert len(loops) == 1 and sorted(loops[0]) == [0, 1, 2, 3]


def test_every_crossing_edge_in_two_segments():
    rng = np.random.default_rng(9)
    for _ in range(300):
        f = 1.0 + rng.normal(size=8)
        segs = om.leaf_face_segments(f, 1.0)
        cross = [e for e in range(12)
                 if (f[om.edge_corners(e)[0]] >= 1.0) != (f[om.edge_corners(e)[1]] >= 1.0)]
        cnt = {}
        for s in segs:
            for e in s:
                cnt[e] = cnt.get(e, 0) + 1
        assert sorted(cnt) == sorted(cross) and all(v == 2 for v in cnt.values())
        assert sum(len(L) for L in om.loops_from_segments(segs)) == len(cross)


TET = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float),
       np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]]))


def test_tetrahedron():
    r = om.check_mesh(*TET)
    assert r["boundary_edges"] == r["nonmanifold_edges"] == r["misoriented_edges"] == 0
    assert r["nonmanifold_vertices"] == 0 and r["intersecting_pairs"] == 0
    assert r["euler"] == 2 and r["components"] == 1
    assert abs(r["volume"] - 1 / 6) < 1e-15  # outward orientation


def test_octahedron_volume_and_area():
    X = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    T = []
    for a in (0, 1):
        for b in (2, 3):
            for c in (4, 5):
                t = [a, b, c]
                n = np.cross(X[b] - X[a], X[c] - X[a])
                if np.dot(n, X[a] + X[b] + X[c]) < 0:
                    t = [a, c, b]
                T.append(t)
    r = om.check_mesh(X, np.array(T))
    assert r["euler"] == 2 and r["nonmanifold_vertices"] == 0 and r["misoriented_edges"] == 0
    assert abs(r["volume"] - 4 / 3) < 1e-14
    assert abs(r["area"] - 8 * np.sqrt(3) / 2) < 1e-13


def test_torus_euler_zero():
    n, m, R, a = 12, 8, 3.0, 1.0
    X = np.array([[(R + a * np.cos(v * 2 * np.pi / m)) * np.cos(u * 2 * np.pi / n),
                   (R + a * np.cos(v * 2 * np.pi / m)) * np.sin(u * 2 * np.pi / n),
                   a * np.sin(v * 2 * np.pi / m)] for u in range(n) for v in range(m)])
    T = []
    for u in range(n):
        for v in range(m):
            p, q = u * m + v, ((u + 1) % n) * m + v
            p1, q1 = u * m + (v + 1) % m, ((u + 1) % n) * m + (v + 1) % m
            T += [[p, q, q1], [p, q1, p1]]
    r = om.check_mesh(X, np.array(T), cell=1.5)
    assert r["euler"] == 0 and r["components"] == 1
    assert r["nonmanifold_vertices"] == 0 and r["intersecting_pairs"] == 0
    assert r["misoriented_edges"] == 0


def test_defects_counted():
    X, T = TET
    r = om.check_mesh(X, T[:3])          # a face missing
    assert r["boundary_edges"] == 3 and r["nonmanifold_vertices"] == 3
    T2 = T.copy()
    T2[3] = T2[3][::-1]                    # one face flipped
    r = om.check_mesh(X, T2)
    assert r["misoriented_edges"] == 3 and r["boundary_edges"] == 0
    # two tetrahedra sharing vertex 0: its neighbourhood is two loops
    Y = np.vstack([X, -X[1:]])
    T3 = np.vstack([T, np.array([[0, 6, 5], [0, 5, 4], [0, 4, 6], [4, 5, 6]])])
    r = om.check_mesh(Y, T3)
    assert r["nonmanifold_vertices"] == 1 and r["boundary_edges"] == 0
    assert r["euler"] == 3


def test_crossing_triangles():
    X = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0], [0.5, 0.5, -1], [0.5, 0.5, 1], [3, 3, 0]], float)
    r = om.check_mesh(X, np.array([[0, 1, 2], [3, 4, 5]]))
    assert r["intersecting_pairs"] == 1
    Z = X.copy()
    Z[3:, 2] += 5.0
    assert om.check_mesh(Z, np.array([[0, 1, 2], [3, 4, 5]]))["intersecting_pairs"] == 0


def test_intersection_is_exact_at_contact():
    # closed triangles: a vertex exactly on the other's face meets it; moved
    # off the plane by the smallest double, the pair is apart on that side
    # and crossing on the other
    T = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    for z, meets in ((0.0, True), (5e-324, False), (-5e-324, True)):
        U = np.array([[0.25, 0.25, z], [0.25, 0.5, 1.0], [0.5, 0.25, 1.0]])
        assert om.tris_intersect(T, U) == meets, z
        assert om.tris_intersect(U, T) == meets, z
    # a vertex exactly on an edge (x + y = 1 on the hypotenuse) meets it
    U = np.array([[0.5, 0.5, 0.0], [0.5, 0.5, 1.0], [1.0, 1.0, 1.0]])
    assert om.tris_intersect(T, U)
    # coplanar: overlapping, touching at a vertex, and apart
    assert om.tris_intersect(T, np.array([[0.2, 0.2, 0], [2, 0.2, 0], [0.2, 2, 0]]))
    assert om.tris_intersect(T, np.array([[1, 0, 0], [2, 0, 0], [2, 1, 0]]))
    assert not om.tris_intersect(T, np.array([[1 + 1e-15, 0, 0], [2, 0, 0], [2, 1, 0]]))


def test_sliver_near_miss_is_not_an_intersection():
    # two slivers around a lattice corner (4, -1, 4) where the surface passes
    # through it: every vertex of the first has x > 4 and every vertex of the
    # second x <= 4, so the plane x = 4 separates them; tolerance-based tests
    # report this pair as crossing
    T1 = np.array([[4.0000005, -1.0, 4.0], [4.149170512684766, -1.5, 4.0],
                   [4.363400953262453, -1.0, 3.5]])
    T2 = np.array([[3.5, -0.5, 4.000011358053928], [4.0, -1.0, 4.000000500000001],
                   [4.0, -0.9999995, 4.0]])
    assert T1[:, 0].min() > 4.0 >= T2[:, 0].max()
    assert not om.tris_intersect(T1, T2)
    X = np.concatenate([T1, T2])
    assert om.check_mesh(X, np.array([[0, 1, 2], [3, 4, 5]]))["intersecting_pairs"] == 0


def test_closure_restores_dropped_surface_cubes():
    # phi of two overlapping spheres sampled on a lattice: the cubes whose
    # corners straddle c are face-connected through crossing faces (one
    # connected surface, no corner value equal to c), so dropping any of them
    # but one and closing the open faces must give back exactly the full set
    # -- and nothing outside it, since only crossing faces are followed
    n, h, c = 24, 0.35, 1.0
    X = np.stack(np.meshgrid(*[np.arange(n + 1) * h - 4.0] * 3, indexing="ij"), -1)
    f = np.exp(-((X - [0.3, 0.1, -0.2]) ** 2).sum(-1) + 4.0) + \
        np.exp(-((X - [1.6, 0.4, 0.3]) ** 2).sum(-1) + 3.0)
    cubes, vals = [], []
    for q in np.ndindex(n, n, n):
        v = np.array([f[q[0] + (k & 1), q[1] + ((k >> 1) & 1), q[2] + ((k >> 2) & 1)]
                      for k in range(8)])
        if (v >= c).any() and (v < c).any():
            cubes.append(q)
            vals.append(v)
    assert len(cubes) > 300
    rng = np.random.default_rng(3)
    keep = rng.random(len(cubes)) < 0.3
    keep[0] = True
    ijk = np.array(cubes)[keep]
    cp = np.array(vals)[keep]
    added, aphi = om.close_open_faces(ijk, cp, np.ones(len(ijk), bool), c, (n, n, n),
                                      lambda P: f[P[:, 0], P[:, 1], P[:, 2]])
    want = sorted(tuple(q) for q, k in zip(cubes, keep) if not k)
    assert added == want
    for q, v in zip(added, aphi):
        assert np.array_equal(v, vals[cubes.index(q)])
    # nothing to add on the full set
    added, _ = om.close_open_faces(np.array(cubes), np.array(vals), np.ones(len(cubes), bool),
                                   c, (n, n, n), lambda P: f[P[:, 0], P[:, 1], P[:, 2]])
    assert added == []


def test_split_coarse_equals_direct_enumeration():
    # a sampled field on the finest lattice; leaves of level K - 1 (2x2x2
    # blocks) and K - 2 (4x4x4) taken over parts of it: the cubes that
    # replace the coarse SURFACE leaves are exactly the straddling finest
    # cubes inside them, with the sampled values
    n, h, c, K = 16, 0.5, 1.0, 3
    X = np.stack(np.meshgrid(*[np.arange(n + 1) * h - 4.0] * 3, indexing="ij"), -1)
    f = np.exp(-((X - [0.3, 0.1, -0.2]) ** 2).sum(-1) + 4.0)
    ijk, level, cp = [], [], []
    for q in np.ndindex(n // 4, n // 4, n // 4):  # level K - 2 blocks over x < n/2
        if q[0] >= n // 8:
            continue
        b = np.array(q) * 4
        ijk.append(q); level.append(K - 2)
        cp.append([f[b[0] + 4 * (v & 1), b[1] + 4 * ((v >> 1) & 1), b[2] + 4 * ((v >> 2) & 1)]
                   for v in range(8)])
    for q in np.ndindex(n // 2, n // 2, n // 2):  # level K - 1 blocks over x >= n/2
        if q[0] < n // 4:
            continue
        b = np.array(q) * 2
        ijk.append(q); level.append(K - 1)
        cp.append([f[b[0] + 2 * (v & 1), b[1] + 2 * ((v >> 1) & 1), b[2] + 2 * ((v >> 2) & 1)]
                   for v in range(8)])
    ijk, level, cp = np.array(ijk), np.array(level), np.array(cp)
    surf = (cp >= c).any(1) & (cp < c).any(1)
    cubes = om.split_coarse(ijk, level, cp, surf, K, lambda P: f[P[:, 0], P[:, 1], P[:, 2]])
    got, vals = om.straddling(cubes, c)
    want = []
    for q, l, s in zip(ijk, level, surf):
        if not s:
            continue
        sh = K - int(l)
        for d in np.ndindex(1 << sh, 1 << sh, 1 << sh):
            p = (int(q[0] << sh) + d[0], int(q[1] << sh) + d[1], int(q[2] << sh) + d[2])
            v = np.array([f[p[0] + (k & 1), p[1] + ((k >> 1) & 1), p[2] + ((k >> 2) & 1)]
                          for k in range(8)])
            if (v >= c).any() and (v < c).any():
                want.append(p)
    assert surf.sum() > 10 and len(want) > 50
    assert got == sorted(want)
    for p, v in zip(got, vals):
        assert np.array_equal(v, [f[p[0] + (k & 1), p[1] + ((k >> 1) & 1), p[2] + ((k >> 2) & 1)]
                                  for k in range(8)])
