"""Estimator variants on the HIP path against the oracle (Section 2.2):

* degree n = 1, 2 of the 1-D Legendre series (Section 2.2.1 uses n = 3): the
  HIP projections zero the entries above n and correct L_{n-1}, L_n;
* child tensors re-expanded from the parent's polynomial (eq. childtensor)
  instead of projected from the atoms again: only the roots loop over atoms.

Leaf lists, masks, classes and vertex keys bit-exact; corner values and t
to the precision's bar (tests/parity_util.py); oracle near ties excluded.
"""
import numpy as np
import pytest

import oracle
from paper_1611_03474_amd import synth, tms, workloads
from parity_util import compare

pytestmark = pytest.mark.gpu

PRECS = [tms.PREC_FP64, tms.PREC_FP32_GUARD]
PIDS = ["fp64", "fp32g"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = tms.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def glob1000():
    return synth.globule(1000, 1006)


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
@pytest.mark.parametrize("degree", [1, 2])
@pytest.mark.parametrize("tau", [1e-3, 0.1])
def test_degree_parity(ctx, glob1000, prec, degree, tau):
    ref = oracle.partition(glob1000, 0.9, tau=tau, degree=degree)
    got, _ = compare(ctx, glob1000, prec, 0.9, ref=ref, label="degree %d tau %g" % (degree, tau),
                     tau=tau, degree=degree)
    if degree == 1:  # no entry above degree one: nothing is refined below level 1
        assert got["leaves"]["level"].max() <= 1


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
@pytest.mark.parametrize("tau", [1e-3, 0.1, 0.3])
def test_reexpand_parity(ctx, glob1000, prec, tau):
    ref = oracle.partition(glob1000, 0.9, tau=tau, reexpand=True)
    got, _ = compare(ctx, glob1000, prec, 0.9, ref=ref, label="re-expanded tau %g" % tau,
                     tau=tau, child_tensor=tms.CHILD_REEXPAND)
    st = got["stats"]
    # no atom loop below the roots
    assert st["n_pairs_lvl"][0] == st["n_pairs"] > 0
    assert ref.n_pairs == st["n_pairs"]


def test_reexpand_degree2_globule5k(ctx):
    # both variants together at the 5,000-atom size, FP32+guard
    w = workloads.GLOBULE5K[0.9]
    atoms = workloads.atoms(w)
    ref = oracle.partition(atoms, w.D, tau=1e-3, degree=2, reexpand=True)
    compare(ctx, atoms, tms.PREC_FP32_GUARD, w.D, ref=ref, label="globule5k degree 2 re-expanded",
            tau=1e-3, degree=2, child_tensor=tms.CHILD_REEXPAND)


def test_reexpand_batch_equals_single(ctx):
    # a batch with both variants: each conformation's leaves and corner values
    # bit-identical to its own pass, and that pass equal to the oracle
    confs = [synth.globule(n, 2200 + k) for k, n in enumerate([300, 700, 150])]
    kw = dict(D=0.9, tau=0.1, degree=2, child_tensor=tms.CHILD_REEXPAND)
    p = tms.make_params(precision=tms.PREC_FP32_GUARD, **kw)
    cells = ctx.build_cells_batch(confs, p)
    leaves, cphi, _ = ctx.partition_estimate(cells)
    L = tms.leaves_to_numpy(leaves)
    cp = cphi.cpu().numpy()
    ctx.free_cells(cells)
    start = 0
    for b, atoms in enumerate(confs):
        c1 = ctx.build_cells(atoms, p)
        l1, cp1, _ = ctx.partition_estimate(c1)
        l1 = tms.leaves_to_numpy(l1)
        ctx.free_cells(c1)
        n = len(l1)
        seg = L[start:start + n]
        assert np.all(seg["conf"] == b)
        for f in ("ix", "iy", "iz", "level", "reason", "mask", "cls"):
            assert np.array_equal(seg[f], l1[f]), (b, f)
        assert np.array_equal(cp[start:start + n], cp1.cpu().numpy())
        ref = oracle.partition(atoms, 0.9, tau=0.1, degree=2, reexpand=True)
        compare(ctx, atoms, tms.PREC_FP32_GUARD, ref=ref, label="batch conformation %d" % b, **kw)
        start += n
    assert start == len(L)


def test_variant_params_checked(ctx):
    for bad in (dict(degree=4), dict(degree=-1), dict(child_tensor=2)):
        rc, msg = tms.check_params(tms.make_params(**bad))
        assert rc == tms.TMS_E_INVALID and msg
    # degree 0 means the paper's 3
    a = synth.globule(200, 1001)
    outs = []
    for d in (0, 3):
        cells = ctx.build_cells(a, tms.make_params(D=0.9, tau=0.1, degree=d))
        leaves, cphi, _ = ctx.partition_estimate(cells)
        outs.append((leaves.cpu().numpy(), cphi.cpu().numpy()))
        ctx.free_cells(cells)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_capture_refuses_reexpand(ctx):
    a = synth.globule(200, 1001)
    cells = ctx.build_cells(a, tms.make_params(D=0.9, tau=0.1, child_tensor=tms.CHILD_REEXPAND))
    leaves, cphi, _ = ctx.partition_estimate(cells)
    ctx.extract(cells, leaves, cphi)
    with pytest.raises(tms.TmsError) as ei:
        ctx.graph_capture(cells)
    assert ei.value.code == tms.TMS_E_INVALID
    ctx.free_cells(cells)
