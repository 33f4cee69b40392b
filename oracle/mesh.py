"""Oracle for the host Stage 2 (Section 2.3) and the manifold conditions
(Section 3.2).  TEST INFRASTRUCTURE ONLY: nothing in the product path may
import it; only the test-suite uses it.  Plain numpy/scipy, slow, written
from the definitions:

* face segments of a leaf -- on a face the trilinear g is bilinear, and the
  curve g = c joins the face's edge points (eq. intersection) in pairs; with
  four of them (corners alternating about c) the pairing follows which
  corners the region g >= c connects, found here by brute force: the face is
  sampled on a fine grid and the connected components of {g >= c} labelled;
* the loops those segments form on the cube's boundary;
* closing open faces (the cubes across crossing faces with no SURFACE leaf
  across, added until none is left), and the cubes of the finest level that
  replace coarser SURFACE leaves;
* a mesh checker: (a) every edge in exactly two triangles, traversed in
  opposite directions; (b) the triangles around every vertex form a single
  loop; (c) no two closed triangles without a shared vertex meet (brute
  force over all pairs, segment-triangle tests decided by exact orientation
  signs); plus components, Euler characteristic, area and enclosed volume.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


# ---- cube numbering (corner v = dx + 2 dy + 4 dz; edge e along axis e // 4,
# the other two axes in ascending order at offsets (e & 1, (e >> 1) & 1)) ----

def edge_offsets(e):
    axis = e >> 2
    others = sorted({0, 1, 2} - {axis})
    off = [0, 0, 0]
    off[others[0]] = e & 1
    off[others[1]] = (e >> 1) & 1
    return axis, off


def edge_corners(e):
    axis, off = edge_offsets(e)
    v0 = off[0] + 2 * off[1] + 4 * off[2]
    return v0, v0 + (1 << axis)


def edge_key(conf, level, K, ijk, e):
    """Key of a leaf's edge e: conf | level | axis | finest-lattice lower end
    (the vertex order of the edge-point list)."""
    axis, off = edge_offsets(e)
    sh = K - level
    X, Y, Z = [(int(ijk[a]) + off[a]) << sh for a in range(3)]
    return (conf << 53) | (level << 50) | (axis << 48) | (X << 32) | (Y << 16) | Z


def face_edges(a, s):
    """Edges of the face u_a = s with their two corners."""
    out = []
    for e in range(12):
        axis, off = edge_offsets(e)
        if axis != a and off[a] == s:
            out.append(e)
    return out


# ---- face pairing by brute force ----------------------------------------------

def high_corners_joined(F, c, n=401):
    """F[p][q]: a face's corner values (p, q in {0,1}), corners alternating
    about c.  True if the two corners with value >= c lie in one connected
    component of {bilinear >= c} (sampled on an n x n grid)."""
    t = np.linspace(0.0, 1.0, n)
    P, Q = np.meshgrid(t, t, indexing="ij")
    h = (F[0][0] * (1 - P) * (1 - Q) + F[1][0] * P * (1 - Q) + F[0][1] * (1 - P) * Q
         + F[1][1] * P * Q)
    lab, _ = ndimage.label(h >= c)
    hi = [(p, q) for p in (0, 1) for q in (0, 1) if F[p][q] >= c]
    assert len(hi) == 2
    (p0, q0), (p1, q1) = hi
    return lab[p0 * (n - 1), q0 * (n - 1)] == lab[p1 * (n - 1), q1 * (n - 1)]


def leaf_face_segments(f, c):
    """The face segments of a leaf with corner values f[8]: a set of
    frozensets {e1, e2} of cube edge indices."""
    segs = set()
    for a in range(3):
        p_ax, q_ax = sorted({0, 1, 2} - {a})
        for s in (0, 1):
            def corner(p, q):
                off = [0, 0, 0]
                off[a], off[p_ax], off[q_ax] = s, p, q
                return off[0] + 2 * off[1] + 4 * off[2]
            cuts = []
            for e in face_edges(a, s):
                v0, v1 = edge_corners(e)
                if (f[v0] >= c) != (f[v1] >= c):
                    cuts.append(e)
            if len(cuts) == 2:
                segs.add(frozenset(cuts))
            elif len(cuts) == 4:
                F = [[f[corner(p, q)] for q in (0, 1)] for p in (0, 1)]
                joined = high_corners_joined(F, c)
                # cut off each corner of the separated kind: pair its edges
                for p in (0, 1):
                    for q in (0, 1):
                        v = corner(p, q)
                        if (f[v] >= c) == joined:
                            continue
                        mine = [e for e in cuts if v in edge_corners(e)]
                        assert len(mine) == 2
                        segs.add(frozenset(mine))
    return segs


def loops_from_segments(segs):
    """Cycles (lists of edge indices) formed by the segments."""
    nb = {}
    for sg in segs:
        a, b = tuple(sg)
        nb.setdefault(a, []).append(b)
        nb.setdefault(b, []).append(a)
    assert all(len(v) == 2 for v in nb.values())
    seen, loops = set(), []
    for start in sorted(nb):
        if start in seen:
            continue
        loop, prev, cur = [start], None, start
        seen.add(start)
        while True:
            nxt = nb[cur][0] if nb[cur][0] != prev else nb[cur][1]
            prev, cur = cur, nxt
            if cur == start:
                break
            loop.append(cur)
            seen.add(cur)
        loops.append(loop)
    return loops


# ---- mesh checker ---------------------------------------------------------------

# ---- condition (c): exact intersection of closed triangles ---------------
# Every decision is the sign of an orientation determinant.  The coordinates
# are doubles, hence dyadic rationals, so integers give the exact sign; the
# vectorised pass uses a sign computed in doubles only where it clears an
# error bound (1e-14 of the sum of the magnitudes of the determinant's terms;
# the rounding error of this evaluation is below 8e-16 of it, Shewchuk,
# "Adaptive precision floating-point arithmetic and fast robust geometric
# predicates", 1997) and leaves the other pairs to the exact test.

def _exact_ints(*pts):
    """The coordinates of the points as integers over one common denominator:
    a double is n / 2^k exactly, so scaling every coordinate by the largest
    2^k keeps every sign and ratio."""
    rat = [float(x).as_integer_ratio() for pt in pts for x in pt]
    den = max(d for _, d in rat)
    v = [n * (den // d) for n, d in rat]
    k = len(pts[0])
    return [v[i * k:(i + 1) * k] for i in range(len(pts))]


def _orient3d_exact(a, b, c, d):
    """Sign of det[a - d; b - d; c - d], exactly (integer arithmetic)."""
    a, b, c, d = _exact_ints(a[:3], b[:3], c[:3], d[:3])
    A = [a[i] - d[i] for i in range(3)]
    B = [b[i] - d[i] for i in range(3)]
    C = [c[i] - d[i] for i in range(3)]
    det = (A[0] * (B[1] * C[2] - B[2] * C[1]) - A[1] * (B[0] * C[2] - B[2] * C[0])
           + A[2] * (B[0] * C[1] - B[1] * C[0]))
    return (det > 0) - (det < 0)


def _orient2d_exact(a, b, c):
    """Sign of det[a - c; b - c] in the plane, exactly."""
    a, b, c = _exact_ints(a[:2], b[:2], c[:2])
    det = (a[0] - c[0]) * (b[1] - c[1]) - (a[1] - c[1]) * (b[0] - c[0])
    return (det > 0) - (det < 0)


def _on_segment2(p, q, r):
    """r on the closed segment pq, given that the three are collinear."""
    return (min(p[0], q[0]) <= r[0] <= max(p[0], q[0])
            and min(p[1], q[1]) <= r[1] <= max(p[1], q[1]))


def _segments_meet2(p, q, r, s):
    o1, o2 = _orient2d_exact(p, q, r), _orient2d_exact(p, q, s)
    o3, o4 = _orient2d_exact(r, s, p), _orient2d_exact(r, s, q)
    if o1 * o2 < 0 and o3 * o4 < 0:
        return True
    return ((o1 == 0 and _on_segment2(p, q, r)) or (o2 == 0 and _on_segment2(p, q, s))
            or (o3 == 0 and _on_segment2(r, s, p)) or (o4 == 0 and _on_segment2(r, s, q)))


def _in_triangle2(p, a, b, c):
    s = (_orient2d_exact(a, b, p), _orient2d_exact(b, c, p), _orient2d_exact(c, a, p))
    return all(x >= 0 for x in s) or all(x <= 0 for x in s)


def segment_meets_triangle(p, q, a, b, c):
    """Does the closed segment pq meet the closed triangle abc?  Exact."""
    op, oq = _orient3d_exact(a, b, c, p), _orient3d_exact(a, b, c, q)
    if op * oq > 0:
        return False
    if op == 0 and oq == 0:
        # in the triangle's plane: project out the axis along which its
        # normal is largest (orientations are kept)
        n = np.cross(np.asarray(b, float) - a, np.asarray(c, float) - a)
        keep = [i for i in range(3) if i != int(np.argmax(np.abs(n)))]
        P, Q, A, B, C = ([float(x[i]) for i in keep] for x in (p, q, a, b, c))
        return (_in_triangle2(P, A, B, C) or _in_triangle2(Q, A, B, C)
                or _segments_meet2(P, Q, A, B) or _segments_meet2(P, Q, B, C)
                or _segments_meet2(P, Q, C, A))
    # pq crosses the plane (or ends on it): the crossing is in the triangle
    # iff pq passes every directed edge on the same side
    s = (_orient3d_exact(p, q, a, b), _orient3d_exact(p, q, b, c), _orient3d_exact(p, q, c, a))
    return all(x >= 0 for x in s) or all(x <= 0 for x in s)


def tris_intersect(T1, T2):
    """Do two closed triangles (3 x 3 arrays) meet?  They do iff an edge of
    one meets the other.  Exact."""
    for a in range(3):
        if (segment_meets_triangle(T1[a], T1[(a + 1) % 3], *T2)
                or segment_meets_triangle(T2[a], T2[(a + 1) % 3], *T1)):
            return True
    return False


def _orient3d_vec(a, b, c, d):
    """Signs of det[a - d; b - d; c - d] over rows, in doubles, and whether
    each is certain (clears the error bound)."""
    A, B, C = a - d, b - d, c - d
    t0 = B[:, 1] * C[:, 2] - B[:, 2] * C[:, 1]
    t1 = B[:, 2] * C[:, 0] - B[:, 0] * C[:, 2]
    t2 = B[:, 0] * C[:, 1] - B[:, 1] * C[:, 0]
    det = A[:, 0] * t0 + A[:, 1] * t1 + A[:, 2] * t2
    mag = (np.abs(A[:, 0]) * (np.abs(B[:, 1] * C[:, 2]) + np.abs(B[:, 2] * C[:, 1]))
           + np.abs(A[:, 1]) * (np.abs(B[:, 2] * C[:, 0]) + np.abs(B[:, 0] * C[:, 2]))
           + np.abs(A[:, 2]) * (np.abs(B[:, 0] * C[:, 1]) + np.abs(B[:, 1] * C[:, 0])))
    sure = np.abs(det) > 1e-14 * mag
    # four points with one coordinate exactly equal lie in a lattice plane:
    # the determinant is exactly zero (common for sides on a cube face)
    flat = np.zeros(len(det), dtype=bool)
    for k in range(3):
        flat |= (a[:, k] == b[:, k]) & (b[:, k] == c[:, k]) & (c[:, k] == d[:, k])
    return np.where(sure & ~flat, np.sign(det), 0).astype(np.int8), sure | flat


def _seg_tri_vec(p, q, A, B, C):
    """segment_meets_triangle over rows in doubles: (meets, certain).  Rows
    where a sign needed is uncertain, or the segment lies in the plane, are
    not certain."""
    op, sp = _orient3d_vec(A, B, C, p)
    oq, sq = _orient3d_vec(A, B, C, q)
    apart = sp & sq & (op * oq > 0)
    s1, u1 = _orient3d_vec(p, q, A, B)
    s2, u2 = _orient3d_vec(p, q, B, C)
    s3, u3 = _orient3d_vec(p, q, C, A)
    inside = ((s1 >= 0) & (s2 >= 0) & (s3 >= 0)) | ((s1 <= 0) & (s2 <= 0) & (s3 <= 0))
    # the segment in the triangle's plane is left to the exact test
    crossing = sp & sq & ~apart & ~((op == 0) & (oq == 0))
    certain = apart | (crossing & u1 & u2 & u3)
    return crossing & u1 & u2 & u3 & inside, certain


def check_mesh(xyz, tri, intersections=True, cell=None):
    """Manifold conditions and invariants of a triangle mesh (Section 3.2).
    cell: optional edge length of a bucket grid that limits the pairs tested
    for (c) to triangles in touching buckets (all pairs when None)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    nv, nt = len(xyz), len(tri)
    rep = {}
    # (a)
    edges = {}
    for t, (a, b, c) in enumerate(tri):
        for u, v in ((a, b), (b, c), (c, a)):
            edges.setdefault((min(u, v), max(u, v)), []).append(1 if u < v else -1)
    bnd = [e for e, d in edges.items() if len(d) == 1]
    nonman = [e for e, d in edges.items() if len(d) > 2]
    misor = [e for e, d in edges.items() if len(d) == 2 and sum(d) != 0]
    rep["boundary_edges"], rep["nonmanifold_edges"] = len(bnd), len(nonman)
    rep["misoriented_edges"] = len(misor)
    bad = set()
    for e in bnd + nonman + misor:
        bad.update(e)
    # (b): the sides opposite v in its triangles form one cycle
    opp = {}
    for a, b, c in tri:
        opp.setdefault(a, []).append((b, c))
        opp.setdefault(b, []).append((c, a))
        opp.setdefault(c, []).append((a, b))
    for v, link in opp.items():
        deg = {}
        for s in link:
            for w in s:
                deg[w] = deg.get(w, 0) + 1
        ok = all(d == 2 for d in deg.values())
        if ok:
            # walk one cycle and require it to use every side
            nb = {}
            for x, y in link:
                nb.setdefault(x, []).append(y)
                nb.setdefault(y, []).append(x)
            start = link[0][0]
            prev, cur, n = None, start, 0
            while True:
                nxt = nb[cur][0] if nb[cur][0] != prev else nb[cur][1]
                prev, cur = cur, nxt
                n += 1
                if cur == start or n > len(link):
                    break
            ok = cur == start and n == len(link)
        if not ok:
            bad.add(v)
    rep["nonmanifold_vertices"] = len(bad)
    # components, Euler characteristic
    parent = list(range(nv))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    used = np.zeros(nv, dtype=bool)
    for a, b, c in tri:
        used[[a, b, c]] = True
        for u, v in ((a, b), (b, c)):
            ru, rv = find(u), find(v)
            if ru != rv:
                parent[ru] = rv
    rep["components"] = len({find(v) for v in range(nv) if used[v]})
    rep["euler"] = int(used.sum()) - len(edges) + nt
    P = xyz[tri]
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    rep["area"] = float(0.5 * np.linalg.norm(cr, axis=1).sum())
    rep["volume"] = float(np.einsum("ij,ij->i", P[:, 0], np.cross(P[:, 1], P[:, 2])).sum() / 6.0)
    # (c)
    if intersections:
        if cell is None:
            I, J = np.triu_indices(nt, 1)
        else:
            cen = P.mean(axis=1)
            key = np.floor(cen / cell).astype(np.int64)
            buckets = {}
            for i, k in enumerate(map(tuple, key)):
                buckets.setdefault(k, []).append(i)
            Is, Js = [], []
            for k, lst in buckets.items():
                a = np.array(lst)
                for d in np.ndindex(3, 3, 3):
                    k2 = (k[0] + d[0] - 1, k[1] + d[1] - 1, k[2] + d[2] - 1)
                    b = buckets.get(k2)
                    if b is None:
                        continue
                    ii, jj = np.meshgrid(a, np.array(b), indexing="ij")
                    m = ii < jj
                    Is.append(ii[m])
                    Js.append(jj[m])
            I = np.concatenate(Is) if Is else np.zeros(0, np.int64)
            J = np.concatenate(Js) if Js else np.zeros(0, np.int64)
        share = np.zeros(len(I), dtype=bool)
        for a in range(3):
            for b in range(3):
                share |= tri[I, a] == tri[J, b]
        I, J = I[~share], J[~share]
        # closed triangles can meet only if their bounding boxes overlap (an
        # exact comparison of doubles)
        lo, hi = P.min(axis=1), P.max(axis=1)
        box = np.all(lo[I] <= hi[J], axis=1) & np.all(lo[J] <= hi[I], axis=1)
        I, J = I[box], J[box]
        hit = np.zeros(len(I), dtype=bool)
        sure = np.ones(len(I), dtype=bool)
        for a in range(3):
            for U, V in ((I, J), (J, I)):
                h, c = _seg_tri_vec(P[U, a], P[U, (a + 1) % 3], P[V, 0], P[V, 1], P[V, 2])
                hit |= h
                sure &= c
        # pairs no certain sign decided: exactly
        for k in np.flatnonzero(~hit & ~sure):
            hit[k] = tris_intersect(P[I[k]], P[J[k]])
        rep["intersecting_pairs"] = int(hit.sum())
    return rep


# ---- closing open faces -----------------------------------------------------
# Reading (the paper is silent here): a crossing face of a SURFACE leaf with
# no SURFACE leaf across is open, because the bound discarded a coarse cube
# although phi at finest lattice points inside it crosses c.  The cube of the
# leaves' level across each such face is added as a SURFACE leaf, again for
# the added cubes, until no open face is left (or the cube lies outside the
# root grid).  Corner values of a lattice point that is a corner of a SURFACE
# leaf are that leaf's; other points are evaluated by `phi_at`.

FACE_CORNERS = [[v for v in range(8) if ((v >> (f >> 1)) & 1) == (f & 1)] for f in range(6)]


def open_faces(front, cubes, c):
    """Open faces of the cubes `front` {ijk: corner values [8]} with respect
    to the SURFACE cubes `cubes` (same form): a list of (ijk, face, ijk
    across)."""
    out = []
    for q, f in front.items():
        for fc in range(6):
            hi = [f[v] >= c for v in FACE_CORNERS[fc]]
            if all(hi) or not any(hi):
                continue
            r = list(q)
            r[fc >> 1] += 1 if (fc & 1) else -1
            if tuple(r) not in cubes:
                out.append((q, fc, tuple(r)))
    return out


def close_open_faces(ijk, corner_phi, surface, c, dims, phi_at, rounds=64):
    """The cubes added across open faces (sorted list of ijk) and their
    corner values.  ijk, corner_phi: the leaves of one level; surface: their
    SURFACE flags; dims: cubes per axis at that level; phi_at(P): phi at
    lattice points P [m, 3] (integer coordinates at that level)."""
    cubes = {tuple(int(x) for x in q): np.asarray(f, float)
             for q, f, s in zip(ijk, corner_phi, surface) if s}
    known = {}
    for q, f in cubes.items():
        for v in range(8):
            known[(q[0] + (v & 1), q[1] + ((v >> 1) & 1), q[2] + ((v >> 2) & 1))] = f[v]
    added = {}
    front = dict(cubes)
    for _ in range(rounds):
        new = sorted({r for _, _, r in open_faces(front, cubes, c)
                      if all(0 <= r[a] < dims[a] for a in range(3))})
        if not new:
            break
        pts = sorted({(r[0] + (v & 1), r[1] + ((v >> 1) & 1), r[2] + ((v >> 2) & 1))
                      for r in new for v in range(8)} - set(known))
        if pts:
            vals = phi_at(np.array(pts, dtype=np.int64))
            known.update(zip(pts, (float(x) for x in vals)))
        front = {}
        for r in new:
            f = np.array([known[(r[0] + (v & 1), r[1] + ((v >> 1) & 1), r[2] + ((v >> 2) & 1))]
                          for v in range(8)])
            cubes[r] = front[r] = added[r] = f
    keys = sorted(added)
    return keys, np.array([added[k] for k in keys]).reshape(-1, 8)


# ---- coarser SURFACE leaves -------------------------------------------------
# Reading (the paper meshes cubes of different sizes against each other): a
# SURFACE leaf above the finest level K is meshed through the cubes of level
# K inside it whose corner values straddle c.  Values at lattice points that
# are corners of the coarse leaf, or of a SURFACE leaf of level K, are those
# leaves' values; other points are evaluated by `phi_at`.

def split_coarse(ijk, level, corner_phi, surface, K, phi_at):
    """Every level-K cube inside the SURFACE leaves above level K, as
    {ijk: corner values [8]} (`straddling` keeps those whose values lie on
    both sides of c).  ijk, level, corner_phi, surface: the leaves;
    phi_at(P): phi at level-K lattice points P [m, 3]."""
    known = {}
    coarse = []
    for q, l, f, s in zip(ijk, level, corner_phi, surface):
        if not s:
            continue
        sh = K - int(l)
        b = tuple(int(x) << sh for x in q)
        n = 1 << sh
        for v in range(8):
            known[(b[0] + (v & 1) * n, b[1] + ((v >> 1) & 1) * n, b[2] + ((v >> 2) & 1) * n)] = \
                float(f[v])
        if sh > 0:
            coarse.append((b, n))
    pts = sorted({(b[0] + x, b[1] + y, b[2] + z) for b, n in coarse
                  for x in range(n + 1) for y in range(n + 1) for z in range(n + 1)} - set(known))
    if pts:
        known.update(zip(pts, (float(v) for v in phi_at(np.array(pts, dtype=np.int64)))))
    out = {}
    for b, n in coarse:
        for x in range(n):
            for y in range(n):
                for z in range(n):
                    f = np.array([known[(b[0] + x + (v & 1), b[1] + y + ((v >> 1) & 1),
                                         b[2] + z + ((v >> 2) & 1))] for v in range(8)])
                    out[(b[0] + x, b[1] + y, b[2] + z)] = f
    return out


def straddling(cubes, c):
    """The cubes of {ijk: corner values} whose values lie on both sides of c
    (sorted list of ijk, values [k, 8])."""
    keys = sorted(k for k, f in cubes.items() if (f >= c).any() and (f < c).any())
    return keys, np.array([cubes[k] for k in keys]).reshape(-1, 8)
