"""Whole-pass properties of the oracle that the paper's mathematics fixes:
translation by whole root cubes, atom order and the D = 1 rescaling of
Section 2.2.1 leave the refinement unchanged; the leaf set tiles the
surface; counts are consistent.  The refinement structure itself has no
printed reference values in the paper (parity of the level structure is
pinned only through these invariants).  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_1611_03474_amd import synth


def _leafset(r):
    return list(zip(r.level.tolist(), map(tuple, r.ijk.tolist()), r.reason.tolist(),
                    r.mask.tolist(), r.cls.tolist()))


@pytest.fixture(scope="module")
def glob200():
    return synth.globule(200, 1001)


@pytest.mark.parametrize("tau", [1e-3, 0.1, 0.3])
def test_translation_by_root_multiples(glob200, tau):
    r0 = oracle.partition(glob200, 0.9, tau=tau)
    a = glob200.copy()
    a[:, :3] += np.array([2.0 * 3, -2.0 * 5, 2.0 * 7])
    r1 = oracle.partition(a, 0.9, tau=tau)
    assert r0.tie_cube == 0 and r0.tie_corner == 0
    assert np.allclose(r1.origin - r0.origin, [6.0, -10.0, 14.0], atol=0)
    assert _leafset(r0) == _leafset(r1)
    assert np.array_equal(r0.vkey, r1.vkey)
    assert np.allclose(r0.vt, r1.vt, atol=1e-12)


def test_atom_permutation(glob200):
    r0 = oracle.partition(glob200, 0.9, tau=0.1)
    perm = np.random.default_rng(0).permutation(len(glob200))
    r1 = oracle.partition(glob200[perm], 0.9, tau=0.1)
    assert _leafset(r0) == _leafset(r1)
    assert np.array_equal(r0.vkey, r1.vkey)
    assert np.allclose(r0.vt, r1.vt, atol=1e-12)


@pytest.mark.parametrize("D", [0.5, 1.5])
def test_D_rescaling_identity(glob200, D):
    # Section 2.2.1: the case D != 1 is the case D = 1 after scaling every
    # length by sqrt(D); the refinement must not change.
    s = math.sqrt(D)
    r0 = oracle.partition(glob200, D, tau=0.1)
    r1 = oracle.partition(glob200 * s, 1.0, tau=0.1, h0=2.0 * s, h_min=0.25 * s, pad=3.0 * s)
    assert np.allclose(r1.origin, r0.origin * s, rtol=1e-14)
    assert _leafset(r0) == _leafset(r1)
    assert np.array_equal(r0.vkey, r1.vkey)
    assert np.allclose(r0.vt, r1.vt, atol=1e-9)


@pytest.mark.parametrize("tau", [1e-3, 0.1, 0.3])
def test_counts_consistent(glob200, tau):
    r = oracle.partition(glob200, 0.9, tau=tau)
    K = r.K
    assert K == 3
    for lev in range(K + 1):
        assert r.n_est[lev] == r.n_disc[lev] + r.n_refine[lev] + r.n_conv[lev] + r.n_hmin[lev]
        if lev < K:
            assert r.n_est[lev + 1] == 8 * r.n_refine[lev]
    assert r.n_refine[K] == 0 and r.n_hmin[:K].sum() == 0 and r.n_conv[0] == 0
    assert r.n_leaves == r.n_conv.sum() + r.n_hmin.sum()
    # leaves are listed level by level
    assert np.all(np.diff(r.level.astype(int)) >= 0)
    # no two leaves overlap: map each leaf to its finest-lattice box
    boxes = set()
    for lev, ijk in zip(r.level, r.ijk):
        sh = K - int(lev)
        base = np.array(ijk) << sh
        for dz in range(1 << sh):
            for dy in range(1 << sh):
                for dx in range(1 << sh):
                    key = (base[0] + dx, base[1] + dy, base[2] + dz)
                    assert key not in boxes
                    boxes.add(key)
    if tau >= 0.1:
        assert r.n_conv[1:].sum() > 0  # converged leaves do occur


def test_surface_cubes_all_kept(glob200):
    # every finest-lattice cube that the uniform-grid method at h_min flags as
    # surface-crossing (corner signs differ) must lie inside some kept leaf of
    # the adaptive pass: a discarded cube has c outside [L, U], an enclosure
    # of the polynomial, so corner values (which equal phi there up to
    # truncation) cannot straddle c by more than the approximation error.
    ra = oracle.partition(glob200, 0.9, tau=1e-3)
    ru = oracle.partition(glob200, 0.9, uniform=True, h0=0.25)
    sh = ra.K
    covered = set()
    off = np.round((ru.origin - ra.origin) / 0.25).astype(int)
    for lev, ijk in zip(ra.level, ra.ijk):
        s = sh - int(lev)
        base = np.array(ijk) << s
        for dz in range(1 << s):
            for dy in range(1 << s):
                for dx in range(1 << s):
                    covered.add((base[0] + dx, base[1] + dy, base[2] + dz))
    miss = 0
    for ijk, cls in zip(ru.ijk, ru.cls):
        if cls == oracle.CLS_SURFACE:
            k = tuple((np.array(ijk) + off).tolist())
            if k not in covered:
                miss += 1
    assert miss == 0


def test_uniform_mode_counts(glob200):
    r = oracle.partition(glob200, 0.9, uniform=True, h0=0.5)
    assert r.n_leaves == int(np.prod(r.dims))
    assert r.n_corners == int(np.prod(r.dims + 1))
    assert set(np.unique(r.reason)) == {oracle.REASON_UNIFORM}
    # every sign-change edge yields one vertex, shared edges once
    assert r.n_vert > 0 and len(set(r.vkey.tolist())) == r.n_vert


def test_invalid_inputs_rejected():
    a = synth.globule(20, 1)
    with pytest.raises(ValueError):
        oracle.partition(a, -1.0)
    with pytest.raises(ValueError):
        oracle.partition(a, 0.9, h_min=0.3)
    b = a.copy()
    b[3, 3] = 0.0
    with pytest.raises(ValueError):
        oracle.partition(b, 0.9)
    b = a.copy()
    b[2, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.partition(b, 0.9)


def test_empty_atom_set():
    r = oracle.partition(np.zeros((0, 4)), 0.9)
    assert r.n_leaves == 0 and r.n_vert == 0 and r.cubes_estimated == 0
