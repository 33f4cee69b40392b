"""Parity with the FP64 oracle at the real sizes of the adaptive workloads,
element by element (leaf list, levels, reasons, masks, classes bit-exact;
corner values, vertex keys, t and positions within the bars of
``parity_util``), near-tie subtrees excluded and counted:

* the 5,000-atom globule at D = 0.5, 0.9 and 1.5 (h0 = 2 -> h_min = 0.25,
  tau = 1e-3) in FP32+guard, and at D = 0.9 in FP64 too;
* the 22,009-atom slice of the 110,000-atom assembly (its first four
  globules with their hydrogens) in FP32+guard.
"""
import pytest

import oracle
from paper_1611_03474_amd import tms, workloads
from parity_util import compare

pytestmark = pytest.mark.gpu

_REF = {}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = tms.Context(0)
    yield c
    c.close()


def _ref(key, atoms, w):
    if key not in _REF:
        _REF[key] = oracle.partition(atoms, w.D, c=w.c, tau=w.tau, h0=w.h0, h_min=w.h_min,
                                     pad=w.pad, eps_cut=w.eps_cut)
    return _REF[key]


def _wkw(w):
    return dict(c=w.c, tau=w.tau, h0=w.h0, h_min=w.h_min, pad=w.pad, eps_cut=w.eps_cut)


@pytest.mark.parametrize("prec,D", [(tms.PREC_FP32_GUARD, 0.5), (tms.PREC_FP32_GUARD, 0.9),
                                    (tms.PREC_FP32_GUARD, 1.5), (tms.PREC_FP64, 0.9)],
                         ids=["fp32g-D0.5", "fp32g-D0.9", "fp32g-D1.5", "fp64-D0.9"])
def test_globule5k_parity(ctx, prec, D):
    w = workloads.GLOBULE5K[D]
    atoms = workloads.atoms(w)
    ref = _ref(w.name, atoms, w)
    got, _ = compare(ctx, atoms, prec, D=w.D, ref=ref, label=w.name, **_wkw(w))
    assert len(got["leaves"]) > 500_000


def test_assembly_slice_parity(ctx):
    w = workloads.ASSEMBLY110K
    atoms = workloads.assembly_slice(workloads.atoms(w), 4)
    assert len(atoms) == 22009
    ref = _ref("assembly_slice4", atoms, w)
    got, _ = compare(ctx, atoms, tms.PREC_FP32_GUARD, D=w.D, ref=ref, label="assembly slice",
                     **_wkw(w))
    assert len(got["leaves"]) > 2_000_000


@pytest.mark.parametrize("prec", [tms.PREC_FP64, tms.PREC_FP32_GUARD], ids=["fp64", "fp32g"])
def test_tile_sizes_bit_identical_globule5k_D05(ctx, prec):
    # 32-atom tiles hold up to 85 atoms for a chunk of one 2 x 2 x 2 block
    # (six intervals in all); at D = 0.5 (R_c = 7 A) such chunks see more
    # than 64 atoms, so a tile's weights must be staged beyond one wavefront
    w = workloads.GLOBULE5K[0.5]
    atoms = workloads.atoms(w)
    cells = ctx.build_cells(atoms, w.params(prec))
    base = ctx.get_tuning().as_dict()
    try:
        ref = None
        for ch in (8, 16, 32):
            ctx.set_tuning(tile_atoms=ch)
            leaves, cphi, st = ctx.partition_estimate(cells)
            got = (leaves.cpu().numpy().tobytes(), cphi.cpu().numpy().tobytes(),
                   list(st["n_est"]), st["n_bound"])
            if ref is None:
                ref = got
            assert got == ref, ch
    finally:
        ctx.set_tuning(**base)
        ctx.free_cells(cells)
