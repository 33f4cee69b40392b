"""Pins for the oracle's estimator variants (Section 2.2): the 1-D series of
degree n = 1, 2 (the paper fixes n = 3, Section 2.2.1) and the child tensor
written from the parent's polynomial (eq. childtensor, Section 2.2.3) instead
of projected from the atoms again.  Each check compares the oracle with
something it does not compute itself: closed forms derived by hand, scipy
quadrature, evaluation identities, or a small brute-force refinement built
from those closed forms.  CPU only."""
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest
from scipy.integrate import quad

import oracle
from paper_1611_03474_amd import synth


def _series(a, t):
    return npleg.legval(t, a)


def _factor(D, lo, hi, xi):
    m, s = 0.5 * (lo + hi), 0.5 * (hi - lo)
    return lambda t: np.exp(-D * (m + s * t - xi) ** 2)


CASES = [(0.9, 0.0, 2.0, 0.3), (0.5, -1.0, 1.0, 2.5), (1.5, 3.0, 3.25, 3.1),
         (0.9, -4.0, -2.0, 0.7), (1.2, 0.5, 1.0, -3.0)]


# --------------------------------------------------------------------------
# degree n (eqs. poly3, condition1, alpha)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("case", CASES)
def test_degree_n_matches_ends(n, case):
    # eq. condition1: the corrected series equals the factor at both ends
    D, lo, hi, xi = case
    f = _factor(D, lo, hi, xi)
    a = oracle.project(D, lo, hi, xi, degree=n)
    assert np.all(a[n + 1:] == 0.0)
    for t in (-1.0, 1.0):
        assert abs(_series(a, t) - f(t)) <= 1e-15 * max(1.0, abs(f(t)))


@pytest.mark.parametrize("case", CASES)
def test_degree_closed_forms(case):
    # With the least-squares coefficients a_j = (2j+1)/2 int f L_j (scipy),
    # the endpoint conditions fix the corrected series of every degree:
    #   n = 1: the chord, (f(1) + f(-1))/2, (f(1) - f(-1))/2;
    #   n = 2: a0, (f(1) - f(-1))/2, (f(1) + f(-1))/2 - a0;
    #   n = 3: a0, a1, (f(1) + f(-1))/2 - a0, (f(1) - f(-1))/2 - a1.
    D, lo, hi, xi = case
    f = _factor(D, lo, hi, xi)
    a0 = 0.5 * quad(f, -1, 1, epsabs=1e-15, epsrel=1e-14)[0]
    a1 = 1.5 * quad(lambda t: f(t) * t, -1, 1, epsabs=1e-15, epsrel=1e-14)[0]
    fp, fm = f(1.0), f(-1.0)
    ev, od = 0.5 * (fp + fm), 0.5 * (fp - fm)
    want = {1: [ev, od, 0, 0], 2: [a0, od, ev - a0, 0], 3: [a0, a1, ev - a0, od - a1]}
    for n, w in want.items():
        got = oracle.project(D, lo, hi, xi, degree=n)
        assert np.allclose(got, w, atol=2e-14, rtol=0), (n, got, w)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_degree_n_reproduces_polynomials(n):
    # a polynomial of degree <= n is its own corrected series (no correction)
    rng = np.random.default_rng(10 + n)
    for _ in range(5):
        c = np.zeros(4)
        c[:n + 1] = rng.normal(size=n + 1)
        got = oracle.project_fn(lambda t: float(npleg.legval(t, c)), degree=n)
        assert np.allclose(got, c, atol=1e-14, rtol=0)


def test_degree_one_partition_stops_at_level_one():
    # n = 1 leaves no entry of degree above one: E = 0, so every child of a
    # kept root is a trilinear leaf (Step 3) and nothing is refined further
    atoms = synth.globule(120, 1001)
    r = oracle.partition(atoms, 0.9, tau=1e-3, degree=1)
    assert r.n_leaves > 0
    assert r.level.max() == 1
    assert np.all(r.reason[r.level == 1] == oracle.REASON_CONVERGED)
    assert r.n_refine[1] == 0 and r.n_est[2] == 0


# --------------------------------------------------------------------------
# child tensor (eq. childtensor)
# --------------------------------------------------------------------------

def _halfmap(s):
    # coefficient of L_j(t) in L_i((t + s)/2), derived by hand from
    # L2(u) = (3u^2 - 1)/2, L3(u) = (5u^3 - 3u)/2 and t^2 = (2 L2 + 1)/3,
    # t^3 = (2 L3 + 3 L1)/5; rows j, columns i
    return np.array([[1.0, s / 2, 0.0, -s / 8],
                     [0.0, 0.5, 3 * s / 4, 3 / 8],
                     [0.0, 0.0, 0.25, 5 * s / 8],
                     [0.0, 0.0, 0.0, 1 / 8]])


def _child_closed(A, o):
    M = [_halfmap(1.0 if (o >> a) & 1 else -1.0) for a in range(3)]
    return np.einsum("ja,kb,lc,abc->jkl", M[0], M[1], M[2], A)


@pytest.mark.parametrize("octant", range(8))
def test_child_tensor_evaluates_as_parent(octant):
    rng = np.random.default_rng(octant)
    A = rng.normal(size=(4, 4, 4))
    C = oracle.child_tensor(A, octant)
    s = np.array([1.0 if (octant >> a) & 1 else -1.0 for a in range(3)])
    for t in rng.uniform(-1, 1, size=(40, 3)):
        u = 0.5 * (t + s)
        assert abs(oracle.tensor_eval(C, *t) - oracle.tensor_eval(A, *u)) <= 1e-14 * np.abs(A).sum()


@pytest.mark.parametrize("octant", range(8))
def test_child_tensor_closed_form(octant):
    rng = np.random.default_rng(100 + octant)
    A = rng.normal(size=(4, 4, 4))
    assert np.allclose(oracle.child_tensor(A, octant), _child_closed(A, octant),
                       atol=1e-14, rtol=0)
    # lower-degree tensors stay lower-degree
    B = np.zeros((4, 4, 4))
    B[:3, :3, :3] = rng.normal(size=(3, 3, 3))
    Cb = oracle.child_tensor(B, octant)
    assert np.all(np.abs(Cb[3, :, :]) <= 1e-15) and np.all(np.abs(Cb[:, 3, :]) <= 1e-15)
    assert np.all(np.abs(Cb[:, :, 3]) <= 1e-15)


def test_child_tensor_composes():
    # two halvings = one quartering: child o2 of child o1 evaluates as the
    # parent on the quarter interval
    rng = np.random.default_rng(7)
    A = rng.normal(size=(4, 4, 4))
    for o1 in (0, 3, 5, 6):
        for o2 in (1, 2, 4, 7):
            C = oracle.child_tensor(oracle.child_tensor(A, o1), o2)
            s1 = np.array([1.0 if (o1 >> a) & 1 else -1.0 for a in range(3)])
            s2 = np.array([1.0 if (o2 >> a) & 1 else -1.0 for a in range(3)])
            for t in rng.uniform(-1, 1, size=(10, 3)):
                u = 0.5 * (0.5 * (t + s2) + s1)
                assert abs(oracle.tensor_eval(C, *t) - oracle.tensor_eval(A, *u)) <= 1e-13


def _reexpand_reference(atoms, D, c, tau, h0, h_min):
    """Brute-force refinement with re-expanded child tensors: root tensors
    from the oracle's projection, children from the hand-derived closed-form
    change of basis, Steps 2 and 3 as stated (Section 2.2)."""
    r = oracle.partition(atoms, D, c=c, tau=tau, h0=h0, h_min=h_min)
    K, o, dims = r.K, r.origin, r.dims
    rc2 = r.rc2
    leaves = set()
    ties = 0

    def visit(A, lev, ijk):
        nonlocal ties
        E = oracle.higher_mass(A)
        if lev >= 1 and 2.0 * E <= tau:
            leaves.add((lev, *ijk, oracle.REASON_CONVERGED))
            return
        L, U, _, _, tie = oracle.bound(A)
        if min(abs(L - c), abs(U - c)) < 1e-9 * np.abs(A).sum() or tie < 1e-9:
            ties += 1
        if c < L or c > U:
            return
        if lev == K:
            leaves.add((lev, *ijk, oracle.REASON_HMIN))
            return
        for oc in range(8):
            child = (2 * ijk[0] + (oc & 1), 2 * ijk[1] + ((oc >> 1) & 1), 2 * ijk[2] + ((oc >> 2) & 1))
            visit(_child_closed(A, oc), lev + 1, child)

    for z in range(dims[2]):
        for y in range(dims[1]):
            for x in range(dims[0]):
                lo = o + np.array([x, y, z]) * h0
                A, nn = oracle.cube_tensor(atoms, D, lo, lo + h0)
                if nn == 0:
                    continue
                visit(A, 0, (x, y, z))
    return leaves, ties


@pytest.mark.parametrize("tau", [0.05, 0.3])
def test_reexpand_partition_matches_brute_force(tau):
    atoms = synth.globule(40, 1011)
    D, c, h0, h_min = 0.9, 1.0, 2.0, 0.5
    ref, ties = _reexpand_reference(atoms, D, c, tau, h0, h_min)
    r = oracle.partition(atoms, D, c=c, tau=tau, h0=h0, h_min=h_min, reexpand=True)
    got = {(int(l), int(i), int(j), int(k), int(e))
           for l, (i, j, k), e in zip(r.level, r.ijk, r.reason)}
    print("leaves %d, near ties %d" % (len(got), ties))
    assert ties == 0 and r.tie_cube == 0
    assert len(got) == r.n_leaves == len(ref)
    assert got == ref
    # no atom loop below the roots: the pairs are those of the roots alone
    r0 = oracle.partition(atoms, D, c=c, tau=tau, h0=h0, h_min=h0)
    assert r.n_pairs == r0.n_pairs


def test_reexpand_invariants():
    # translation by root multiples and atom order leave the re-expanded
    # refinement unchanged (the root tensors and their children do not move)
    atoms = synth.globule(150, 1012)
    kw = dict(tau=0.1, reexpand=True)
    r0 = oracle.partition(atoms, 0.9, **kw)
    a = atoms.copy()
    a[:, :3] += np.array([4.0, -6.0, 2.0])
    r1 = oracle.partition(a, 0.9, **kw)
    perm = np.random.default_rng(3).permutation(len(atoms))
    r2 = oracle.partition(atoms[perm], 0.9, **kw)
    assert r0.tie_cube == 0
    for r in (r1, r2):
        assert np.array_equal(r.level, r0.level) and np.array_equal(r.ijk, r0.ijk)
        assert np.array_equal(r.reason, r0.reason) and np.array_equal(r.vkey, r0.vkey)
    # the roots' decisions are those of the projected variant
    rp = oracle.partition(atoms, 0.9, tau=0.1)
    assert r0.n_est[0] == rp.n_est[0] and r0.n_refine[0] == rp.n_refine[0]
    assert r0.n_disc[0] == rp.n_disc[0]
