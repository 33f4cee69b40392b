"""phi at the unique leaf corners: the staged corner kernel against the
per-point kernel.

The corner kernel shares the atom loads of a wavefront's points but sums each
point over exactly the atoms within R_c, in ascending atom order, with the
operations of the per-point sum (eq. Gaussian1); so

* in FP64, every corner value of a partition equals tms_eval_phi at the same
  lattice point bit for bit;
* under every corner-kernel setting (per-point, one to eight spatial groups
  per wavefront, narrow to wide reach) the partition's leaves and corner values
  are bit-identical, in FP64 and in FP32+guard, for one conformation and for
  a batch whose wavefronts straddle conformations.
"""
import numpy as np
import pytest

from paper_1611_03474_amd import synth, tms

pytestmark = pytest.mark.gpu

SETTINGS = [(1, 48), (2, 8), (2, 2), (4, 8), (8, 4), (2, 24), (2, 64)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = tms.Context(0)
    yield c
    c.close()


def _corner_points(L, origin, hmin, K):
    v = np.arange(8)
    off = np.stack([v & 1, (v >> 1) & 1, (v >> 2) & 1], 1)          # [8, 3]
    ijk = np.stack([L["ix"], L["iy"], L["iz"]], 1).astype(np.int64)  # [n, 3]
    sh = (K - L["level"].astype(np.int64))[:, None, None]
    lat = (ijk[:, None, :] + off[None]) << sh                         # [n, 8, 3]
    return origin[None, None, :] + lat.astype(np.float64) * hmin


def test_corner_values_equal_eval_phi_fp64(ctx):
    atoms = synth.globule(1500, 1011)
    p = tms.make_params(D=0.9, c=1.0, tau=1e-3, precision=tms.PREC_FP64)
    cells = ctx.build_cells(atoms, p)
    ctx.set_tuning(corner_groups=2, corner_reach=48)
    leaves, cphi, st = ctx.partition_estimate(cells)
    L = tms.leaves_to_numpy(leaves)
    hmin = p.h0 / 2.0 ** cells.K
    pts = _corner_points(L, cells.origin, hmin, cells.K).reshape(-1, 3)
    ref = ctx.eval_phi(cells, pts)[0].cpu().numpy()
    got = cphi.cpu().numpy().reshape(-1)
    print("leaves %d, corner values %d, unique %d" % (len(L), len(got), st["n_corners"]))
    assert len(L) > 10_000
    assert np.array_equal(got, ref)
    ctx.free_cells(cells)


def _run(ctx, cells, groups, reach):
    ctx.set_tuning(corner_groups=groups, corner_reach=reach)
    leaves, cphi, st = ctx.partition_estimate(cells)
    return leaves.cpu().numpy(), cphi.cpu().numpy(), st["guard_points"]


@pytest.mark.parametrize("prec", [tms.PREC_FP64, tms.PREC_FP32_GUARD], ids=["fp64", "fp32g"])
@pytest.mark.parametrize("batch", [False, True], ids=["single", "batch"])
def test_corner_settings_bit_identical(ctx, prec, batch):
    p = tms.make_params(D=0.9, c=1.0, tau=1e-3, precision=prec)
    if batch:
        confs = []
        for k, n in enumerate([300, 0, 700, 150, 500]):
            g = synth.globule(n, 3000 + k) if n else np.zeros((0, 4))
            confs.append(g)
        cells = ctx.build_cells_batch(confs, p)
    else:
        cells = ctx.build_cells(synth.globule(2000, 1012), p)
    try:
        base = _run(ctx, cells, 0, 8)
        assert len(base[0]) > 1000
        for g, r in SETTINGS:
            got = _run(ctx, cells, g, r)
            assert np.array_equal(got[0], base[0]), (g, r)
            assert np.array_equal(got[1], base[1]), (g, r)
            assert got[2] == base[2], (g, r)
    finally:
        ctx.set_tuning(corner_groups=2, corner_reach=48)
        ctx.free_cells(cells)


def test_corner_tuning_range(ctx):
    with pytest.raises(tms.TmsError):
        ctx.set_tuning(corner_groups=9)
    with pytest.raises(tms.TmsError):
        ctx.set_tuning(corner_reach=0)
    t = ctx.get_tuning()
    assert t.corner_groups == 2 and t.corner_reach == 48
