"""Pins of the oracle's adjoint (derivative of eq. Gaussian1 and of the edge
points of eq. intersection) against central finite differences of the
oracle's own forward values, and against the forward gradient through
translation invariance."""
import numpy as np
import pytest

import oracle
from paper_1611_03474_amd import synth


def _cloud(n, seed, spread=6.0):
    rng = np.random.default_rng(seed)
    a = np.zeros((n, 4))
    a[:, :3] = rng.uniform(-spread, spread, (n, 3))
    a[:, 3] = rng.uniform(1.2, 1.7, n)
    a[0, 3] = 1.8   # the largest radius sits on atom 0, which is never perturbed
    return a


def test_phi_adjoint_matches_finite_differences():
    D = 0.9
    a = _cloud(40, 7)
    rng = np.random.default_rng(8)
    pts = rng.uniform(-8, 8, (300, 3))
    wbar = rng.normal(size=300)
    g = oracle.phi_adjoint(a, D, pts, wbar)

    def f(b):
        return float(np.dot(wbar, oracle.phi(b, D, pts)))

    h = 1e-5
    for i in (1, 5, 17, 33):
        for k in range(4):
            bp, bm = a.copy(), a.copy()
            bp[i, k] += h
            bm[i, k] -= h
            fd = (f(bp) - f(bm)) / (2 * h)
            assert abs(fd - g[i, k]) <= 1e-6 * max(1.0, abs(g[i, k])), (i, k, fd, g[i, k])


def test_phi_adjoint_translation_identity():
    # moving every atom by e moves phi like moving the points by -e, so
    # sum_i dL/dx_i = -sum_p wbar_p grad phi(p)
    D = 1.5
    a = _cloud(60, 9)
    rng = np.random.default_rng(10)
    pts = rng.uniform(-8, 8, (500, 3))
    wbar = rng.normal(size=500)
    g = oracle.phi_adjoint(a, D, pts, wbar)
    _, gp = oracle.phi(a, D, pts, grad=True)
    lhs = g[:, :3].sum(0)
    rhs = -(wbar[:, None] * gp).sum(0)
    scale = np.abs(wbar[:, None] * gp).sum(0)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale + 1e-14)


def test_phi_adjoint_single_atom_radius():
    # one atom: d phi/d r = 2 D r phi at every point
    D = 0.5
    a = np.array([[0.3, -0.2, 0.1, 1.6]])
    pts = np.array([[1.0, 0.5, -0.7], [2.5, 0.0, 0.0], [0.0, 3.0, 1.0]])
    for k in range(3):
        w = np.zeros(3)
        w[k] = 1.0
        g = oracle.phi_adjoint(a, D, pts, w)
        ph = oracle.phi(a, D, pts[k:k + 1])[0]
        assert g[0, 3] == pytest.approx(2 * D * 1.6 * ph, rel=1e-14)
        assert np.allclose(g[0, :3], 2 * D * (pts[k] - a[0, :3]) * ph, rtol=1e-14, atol=0)


def _central(f, a, i, k, h):
    """Central difference with a Richardson step (h and h/2), which removes
    the h^2 term: edges with a small phi1 - phi0 make t strongly curved."""
    def d(hh):
        bp, bm = a.copy(), a.copy()
        bp[i, k] += hh
        bm[i, k] -= hh
        return (f(bp) - f(bm)) / (2 * hh)
    return (4.0 * d(h / 2) - d(h)) / 3.0


def _frozen_loss(b, D, c, aux):
    ph = oracle.phi(b, D, aux["pts"])
    keys = aux["keys"]
    i0 = np.searchsorted(keys, aux["k0"])
    i1 = np.searchsorted(keys, aux["k1"])
    t = (c - ph[i0]) / (ph[i1] - ph[i0])
    return oracle.surface_loss(ph, c, t, aux["h"])


@pytest.mark.parametrize("D", [0.9, 1.5])
def test_surface_loss_grad_matches_finite_differences(D):
    # structure (leaves, masks, edges) held fixed; central differences with a
    # 1e-4 A step on coordinates and radii
    a = synth.globule(200, 1001)
    c = 1.0
    res = oracle.partition(a, D, c=c, tau=0.1)
    assert res.n_vert > 100
    L, g, aux = oracle.surface_loss_grad(a, D, c, res)
    assert L == pytest.approx(_frozen_loss(a, D, c, aux), rel=1e-13)
    rmax = a[:, 3].max()
    cand = [i for i in np.argsort(-np.abs(g[:, :3]).sum(1)) if a[i, 3] < rmax][:6]
    for i in cand:
        for k in range(4):
            fd = _central(lambda b: _frozen_loss(b, D, c, aux), a, i, k, 1e-4)
            scale = np.abs(g[i]).max()
            assert abs(fd - g[i, k]) <= 2e-6 * scale, (i, k, fd, g[i, k], scale)


def test_surface_loss_vertex_term_alone():
    # the vertex fold on its own: the gradient of sum ((t - 1/2) h)^2 equals
    # phi_adjoint of the folded corner weights, against finite differences
    a = synth.globule(200, 1001)
    D, c = 0.9, 1.0
    res = oracle.partition(a, D, c=c, tau=0.1)
    _, _, aux = oracle.surface_loss_grad(a, D, c, res)
    keys = aux["keys"]
    i0 = np.searchsorted(keys, aux["k0"])
    i1 = np.searchsorted(keys, aux["k1"])
    f0, f1 = aux["phi"][i0], aux["phi"][i1]
    t = (c - f0) / (f1 - f0)
    dldt = 2.0 * (t - 0.5) * aux["h"] ** 2
    w = np.zeros(len(keys))
    np.add.at(w, i0, dldt * (t - 1.0) / (f1 - f0))
    np.add.at(w, i1, dldt * (-t) / (f1 - f0))
    g = oracle.phi_adjoint(a, D, aux["pts"], w)

    def lv(b):
        ph = oracle.phi(b, D, aux["pts"])
        tt = (c - ph[i0]) / (ph[i1] - ph[i0])
        return float(np.sum(((tt - 0.5) * aux["h"]) ** 2))

    i = int(np.argmax(np.abs(g[:, 0])))
    for k in range(4):
        fd = _central(lv, a, i, k, 1e-4)
        assert abs(fd - g[i, k]) <= 2e-6 * np.abs(g[i]).max(), (k, fd, g[i, k])
