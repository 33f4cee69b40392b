"""Pins of the oracle's stage-two points (Section 2.3: extreme points on the
faces, eq. curve; fold curves, eq. fold1; critical points, eq. critical) on
the trilinear interpolant of eq. linear1, against what the mathematics fixes:

* closed forms: a hyperbolic paraboloid s (x - x0)(y - y0) + k (z - z0) + c
  (one fold line along x, one along y, a saddle), and the symmetric
  c + 1/4 + xy + yz + zx, which has the largest possible set of points (two
  fold lines along every axis, two critical points for every pair) at
  coordinates +-1/2;
* every point of random cubes satisfies its equations when the interpolant
  is evaluated independently (the eight-term sum of eq. linear1), and both
  ends of a fold segment lie on the surface (the paper's remark that the
  trilinear fold curves are straight segments ending at extreme points);
* the number of solutions agrees with a brute-force scan along the zero set
  of the derivative(s);
* invariance under scaling of the values, axis permutations and mirrors;
* a single atom gives no fold segments and no critical points (its phi
  changes monotonically along every edge of a cube not centred on it), and
  degenerate cubes when its centre lies on a cube mid-plane.
"""
import itertools

import numpy as np
import pytest

import oracle

CORNERS = np.array([[2 * (v & 1) - 1, 2 * ((v >> 1) & 1) - 1, 2 * ((v >> 2) & 1) - 1]
                    for v in range(8)], dtype=np.float64)


def corner_values(fn):
    return np.array([fn(*CORNERS[v]) for v in range(8)], dtype=np.float64)


def g_eval(f, p):
    """eq. linear1 written out: the eight-term sum of corner values times
    (1 +- x)(1 +- y)(1 +- z) / 8."""
    p = np.atleast_2d(p)
    w = np.ones((len(p), 8))
    for a in range(3):
        w *= 1.0 + CORNERS[None, :, a] * p[:, a:a + 1]
    return (w @ f) / 8.0


def dg(f, p, a):
    """dg/dx_a: g is linear in x_a, so g(x_a = 1) - g(x_a = -1) over 2 is exact."""
    p = np.atleast_2d(p).copy()
    p1, p0 = p.copy(), p.copy()
    p1[:, a], p0[:, a] = 1.0, -1.0
    return (g_eval(f, p1) - g_eval(f, p0)) / 2.0


def records(f, c):
    r, margin, ndeg, mis = oracle.stage2_cube(f, c)
    return r, margin, ndeg, mis


def test_hyperbolic_paraboloid():
    f = corner_values(lambda x, y, z: z - x * y)
    r, margin, ndeg, mis = records(f, 0.0)
    assert ndeg == 0 and mis == 0
    got = sorted(zip(r["kind"], r["axis"], r["root"], map(tuple, r["loc"])))
    want = [(0, 0, 0, (-1.0, 0.0, 0.0)), (0, 1, 0, (0.0, -1.0, 0.0)), (1, 2, 0, (0.0, 0.0, 0.0))]
    assert len(got) == len(want)
    for g_, w_ in zip(got, want):
        assert g_[:3] == w_[:3]
        assert np.allclose(g_[3], w_[3], atol=1e-15)


@pytest.mark.parametrize("seed", range(40))
def test_shifted_saddle(seed):
    rng = np.random.default_rng(seed)
    x0, y0, z0 = rng.uniform(-0.9, 0.9, 3)
    s = rng.choice([-1.0, 1.0]) * rng.uniform(0.3, 3.0)
    k = rng.choice([-1.0, 1.0]) * rng.uniform(0.3, 3.0)
    c = rng.uniform(0.2, 2.0)
    perm = list(itertools.permutations(range(3)))[seed % 6]
    # g in permuted coordinates: q = (x, y, z)[perm]
    fn = lambda *p: s * (p[perm[0]] - x0) * (p[perm[1]] - y0) + k * (p[perm[2]] - z0) + c  # noqa
    r, margin, ndeg, mis = records(corner_values(fn), c)
    assert ndeg == 0 and mis == 0
    q0 = np.zeros(3)
    q0[perm[0]], q0[perm[1]], q0[perm[2]] = x0, y0, z0
    folds = {(int(a), int(k_)): tuple(l) for kd, a, k_, l in
             zip(r["kind"], r["axis"], r["root"], r["loc"]) if kd == 0}
    crit = [(int(a), tuple(l)) for kd, a, l in zip(r["kind"], r["axis"], r["loc"]) if kd == 1]
    # fold along the axis perm[0] through (y0, z0) coordinates, along perm[1]
    # through (x0, z0); none along perm[2]; one critical point for the pair
    # (perm[0], perm[1]) at q0
    assert set(folds) == {(perm[0], 0), (perm[1], 0)}
    for a in (perm[0], perm[1]):
        want = q0.copy()
        want[a] = -1.0
        assert np.allclose(folds[(a, 0)], want, atol=1e-12)
    assert len(crit) == 1 and crit[0][0] == perm[2]
    assert np.allclose(crit[0][1], q0, atol=1e-12)


def test_all_twelve_points():
    c = 1.0
    f = corner_values(lambda x, y, z: c + 0.25 + x * y + y * z + z * x)
    r, margin, ndeg, mis = records(f, c)
    assert ndeg == 0 and mis == 0 and len(r["kind"]) == 12
    h = 0.5
    want = []
    # folds along a through (u, v) = (-1/2, 1/2) then (1/2, -1/2), u the lower axis
    for a in range(3):
        for k, (u, v) in enumerate([(-h, h), (h, -h)]):
            p = np.zeros(3)
            o = [i for i in range(3) if i != a]
            p[a], p[o[0]], p[o[1]] = -1.0, u, v
            want.append((0, a, k, p))
    # critical points of the pair other than w: coordinate along w -1/2, then
    # 1/2; the other two equal to minus it
    for w in range(3):
        for k, t in enumerate([-h, h]):
            p = np.full(3, -t)
            p[w] = t
            want.append((1, w, k, p))
    for i, (kd, a, k, p) in enumerate(want):
        assert (r["kind"][i], r["axis"][i], r["root"][i]) == (kd, a, k), i
        assert np.allclose(r["loc"][i], p, atol=1e-14), (i, r["loc"][i], p)


def _random_cubes(n, seed):
    rng = np.random.default_rng(seed)
    c = 1.0
    out = []
    while len(out) < n:
        f = c + rng.normal(scale=1.0, size=8) * rng.choice([0.05, 0.5, 2.0])
        if f.min() < c < f.max():
            out.append(f)
    return c, out


def test_points_satisfy_their_equations():
    c, cubes = _random_cubes(3000, 7)
    npts = 0
    for f in cubes:
        r, margin, ndeg, mis = records(f, c)
        assert ndeg == 0 and mis == 0
        scale = np.abs(f - c).max()
        for kd, a, loc in zip(r["kind"], r["axis"], r["loc"]):
            npts += 1
            assert np.all(np.abs(loc) <= 1.0)
            if kd == 0:
                assert loc[a] == -1.0
                hi = loc.copy()
                hi[a] = 1.0
                # both ends on the surface, the derivative along a zero there
                assert abs(g_eval(f, loc)[0] - c) <= 1e-11 * scale
                assert abs(g_eval(f, hi)[0] - c) <= 1e-11 * scale
                assert abs(dg(f, loc, a)[0]) <= 1e-11 * scale
            else:
                assert abs(g_eval(f, loc)[0] - c) <= 1e-11 * scale
                for b in range(3):
                    if b != a:
                        assert abs(dg(f, loc, b)[0]) <= 1e-11 * scale
    assert npts > 1000


def _count_folds_scan(f, c, a, ns=4001):
    """Fold lines along a by a scan: for u on a fine grid, v(u) solves
    dg/da = 0 (dg/da is linear in v, so two samples give its root), then the
    sign changes of g - c along the part of that curve inside the square."""
    o = [i for i in range(3) if i != a]
    u = np.linspace(-1.0, 1.0, ns)
    P = np.zeros((ns, 3))
    P[:, o[0]] = u
    P0, P1 = P.copy(), P.copy()
    P0[:, o[1]], P1[:, o[1]] = 0.0, 1.0
    H0, H1 = dg(f, P0, a), dg(f, P1, a)
    with np.errstate(divide="ignore", invalid="ignore"):
        v = -H0 / (H1 - H0)
    inside = np.isfinite(v) & (np.abs(v) <= 1.0)
    P[:, o[1]] = np.where(inside, v, 0.0)
    G = g_eval(f, P) - c
    return int(np.sum(inside[:-1] & inside[1:] & (np.sign(G[:-1]) != np.sign(G[1:]))))


def _count_critical_scan(f, c, w, ns=4001):
    """Critical points of the pair other than w by a scan along x_w: in each
    slice g is bilinear, its stationary point is where both (linear)
    derivatives vanish; sign changes of g - c there, inside the square."""
    o = [i for i in range(3) if i != w]
    t = np.linspace(-1.0, 1.0, ns)
    base = np.zeros((ns, 3))
    base[:, w] = t
    # dg/dx_o0 is linear in x_o1 and independent of x_o0: root in x_o1
    A0, A1 = base.copy(), base.copy()
    A1[:, o[1]] = 1.0
    da0, da1 = dg(f, A0, o[0]), dg(f, A1, o[0])
    B0, B1 = base.copy(), base.copy()
    B1[:, o[0]] = 1.0
    db0, db1 = dg(f, B0, o[1]), dg(f, B1, o[1])
    with np.errstate(divide="ignore", invalid="ignore"):
        x1 = -da0 / (da1 - da0)
        x0 = -db0 / (db1 - db0)
    inside = np.isfinite(x0) & np.isfinite(x1) & (np.abs(x0) <= 1) & (np.abs(x1) <= 1)
    P = base.copy()
    P[:, o[0]] = np.where(inside, x0, 0.0)
    P[:, o[1]] = np.where(inside, x1, 0.0)
    G = g_eval(f, P) - c
    return int(np.sum(inside[:-1] & inside[1:] & (np.sign(G[:-1]) != np.sign(G[1:]))))


def test_solution_counts_match_a_scan():
    c, cubes = _random_cubes(300, 11)
    checked = 0
    tot = 0
    for f in cubes:
        r, margin, ndeg, mis = records(f, c)
        if margin < 1e-3:
            continue  # near a tangency or the cube boundary: a scan cannot tell
        checked += 1
        for a in range(3):
            n_or = int(np.sum((r["kind"] == 0) & (r["axis"] == a)))
            assert n_or == _count_folds_scan(f, c, a), (f, a)
            tot += n_or
            n_or = int(np.sum((r["kind"] == 1) & (r["axis"] == a)))
            assert n_or == _count_critical_scan(f, c, a), (f, a)
            tot += n_or
    assert checked > 180 and tot > 80


def test_invariances():
    c, cubes = _random_cubes(300, 13)
    for f in cubes:
        r, margin, _, _ = records(f, c)
        if margin < 1e-6:
            continue
        # scaling values and isovalue together
        r2, _, _, _ = records(3.0 * f, 3.0 * c)
        assert np.array_equal(r["kind"], r2["kind"]) and np.array_equal(r["axis"], r2["axis"])
        assert np.allclose(r["loc"], r2["loc"], atol=1e-12)
        # a permutation of the axes (new axis i is old axis perm[i]): the new
        # cube's value at q is the old one at p, p[perm[i]] = q[i]
        perm = (2, 0, 1)
        fp = np.zeros(8)
        for vn in range(8):
            po = np.zeros(3)
            for i in range(3):
                po[perm[i]] = CORNERS[vn][i]
            fp[vn] = f[int(sum(((po[i] + 1) // 2) * (1 << i) for i in range(3)))]
        rp, _, _, _ = records(fp, c)
        old = {}
        for k, a, l in zip(r["kind"], r["axis"], r["loc"]):
            old.setdefault((int(k), int(a)), []).append(l)
        assert len(rp["kind"]) == len(r["kind"])
        for k, a, l in zip(rp["kind"], rp["axis"], rp["loc"]):
            lo = np.zeros(3)
            for i in range(3):
                lo[perm[i]] = l[i]
            assert any(np.allclose(lo, x, atol=1e-12) for x in old[(int(k), perm[int(a)])])
        # mirror x -> -x: folds along x keep their (y, z); others mirror in x
        fm = f[[v ^ 1 for v in range(8)]]
        rm, _, _, _ = records(fm, c)
        assert len(rm["kind"]) == len(r["kind"])
        for k, a, l in zip(rm["kind"], rm["axis"], rm["loc"]):
            lm = l.copy()
            if not (k == 0 and a == 0):
                lm[0] = -lm[0]
            assert any(np.allclose(lm, x, atol=1e-12) for x in old[(int(k), int(a))])


def test_single_atom_has_no_folds():
    # one atom: phi depends on each coordinate through (x_a - x_i,a)^2 alone,
    # so along an axis every edge of a cube not centred on the atom changes
    # phi with the same sign, dg/da keeps one sign in the cube, and the
    # trilinear surface has neither fold segments nor critical points
    D, c = 0.9, 0.6
    atom = np.array([[0.3, -0.2, 0.45, 1.7]])
    res = oracle.partition(atom, D, c=c, tau=1e-3)
    s2 = oracle.stage2_of(res, c)
    assert np.sum(res.cls == oracle.CLS_SURFACE) > 100
    assert len(s2.pts) == 0 and s2.n_degenerate == 0
    # centred on a mid-plane x = const of the finest cubes: the cubes cut by
    # that plane see equal values at both ends of every x edge, so g does not
    # depend on x there (degenerate: every point of the patch is a fold point
    # along x); still no isolated points
    atom = np.array([[0.125, -0.2, 0.45, 1.7]])
    res = oracle.partition(atom, D, c=c, tau=1e-3)
    s2 = oracle.stage2_of(res, c)
    assert len(s2.pts) == 0 and s2.n_degenerate > 0
