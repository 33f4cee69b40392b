"""Stage-two points (Section 2.3: eqs. curve, fold1, critical) of the HIP path
against the oracle.

* Identical inputs: a seeded leaf list with corner values -- random values
  around c, exact trilinear saddles s (x - x0)(y - y0) + k (z - z0) in random
  axis orders, the twelve-point function c + 1/4 + xy + yz + zx, cubes whose
  values do not depend on x (degenerate), and INSIDE/OUTSIDE leaves -- fed to
  tms_stage2_points and to the oracle.  Records (leaf, kind, axis, root)
  must match exactly and points within 1e-10 of the leaf edge, outside the
  leaves whose oracle decision margin is below 1e-9 (a near tangency or a
  point on the cube boundary, where two FP64 codes may differ).
* End to end in FP64: each side's own partition of the same atoms, then its
  own stage-two points; the leaf lists are bit-identical, so records are
  matched by leaf index; leaves with an oracle margin below 1e-6 are
  excluded (the corner values agree to 1e-12 relative) and counted, points
  within 1e-8 of the leaf edge.
"""
import numpy as np
import pytest

import oracle
from paper_1611_03474_amd import synth, tms, workloads

pytestmark = pytest.mark.gpu

CORNERS = np.array([[2 * (v & 1) - 1, 2 * ((v >> 1) & 1) - 1, 2 * ((v >> 2) & 1) - 1]
                    for v in range(8)], dtype=np.float64)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = tms.Context(0)
    yield c
    c.close()


def _classes(cp, c):
    mask = np.zeros(len(cp), dtype=np.uint8)
    for v in range(8):
        mask |= (cp[:, v] >= c).astype(np.uint8) << np.uint8(v)
    cls = np.where(mask == 0xFF, tms.CLS_INSIDE, np.where(mask == 0, tms.CLS_OUTSIDE,
                                                         tms.CLS_SURFACE)).astype(np.uint8)
    return mask, cls


def _synthetic_leaves(n, dims, K, c, seed):
    rng = np.random.default_rng(seed)
    level = rng.integers(0, K + 1, n).astype(np.uint8)
    ijk = np.stack([rng.integers(0, dims[a] << level) for a in range(3)], 1).astype(np.int32)
    cp = np.empty((n, 8))
    kind = rng.choice(5, n, p=[0.55, 0.2, 0.05, 0.05, 0.15])
    for q in range(n):
        if kind[q] == 0:      # random values around c
            cp[q] = c + rng.normal(size=8) * rng.choice([0.01, 0.3, 2.0])
        elif kind[q] == 1:    # a trilinear saddle, axes in random order
            x0, y0, z0 = rng.uniform(-1.2, 1.2, 3)
            s, k = rng.uniform(0.2, 2.0, 2) * rng.choice([-1, 1], 2)
            pa = rng.permutation(3)
            P = CORNERS[:, pa]
            cp[q] = c + s * (P[:, 0] - x0) * (P[:, 1] - y0) + k * (P[:, 2] - z0)
        elif kind[q] == 2:    # twelve points
            X, Y, Z = CORNERS.T
            cp[q] = c + rng.uniform(0.2, 3.0) * (0.25 + X * Y + Y * Z + Z * X)
        elif kind[q] == 3:    # independent of x: degenerate along x
            half = c + rng.normal(size=4) * 0.5
            cp[q] = half[np.arange(8) >> 1]
        else:                 # one side of c (no points)
            cp[q] = c + np.abs(rng.normal(size=8)) * rng.choice([-1.0, 1.0])
    mask, cls = _classes(cp, c)
    L = np.zeros(n, dtype=tms.LEAF_DTYPE)
    L["ix"], L["iy"], L["iz"] = ijk[:, 0], ijk[:, 1], ijk[:, 2]
    L["level"], L["mask"], L["cls"] = level, mask, cls
    return L, cp


def _gpu_stage2(ctx, cells, L, cp):
    import torch
    lt = torch.as_tensor(np.frombuffer(L.tobytes(), dtype=np.uint8).reshape(-1, 20)).to(ctx.device)
    ct = torch.as_tensor(cp).to(ctx.device).contiguous()
    recs, ndeg = ctx.stage2_points(cells, lt, ct)
    return tms.s2_to_numpy(recs), ndeg


def _compare(R_g, R_o, margin, h_leaf, thr, tol):
    bad = margin < thr
    keep_g = ~bad[R_g["leaf"]]
    keep_o = ~bad[R_o["leaf"]]
    g, o = R_g[keep_g], R_o[keep_o]
    print("records %d (oracle %d); leaves excluded as near ties %d; compared %d"
          % (len(R_g), len(R_o), bad.sum(), len(g)))
    assert len(g) == len(o)
    for f in ("leaf", "kind", "axis", "root"):
        assert np.array_equal(g[f], o[f]), f
    h = h_leaf[g["leaf"]]
    err = np.max(np.abs(np.stack([g["x"] - o["x"], g["y"] - o["y"], g["z"] - o["z"]], 1))
                 / h[:, None], initial=0.0)
    print("max point error %.3e of the leaf edge" % err)
    assert err <= tol
    return len(g)


def test_stage2_identical_inputs(ctx):
    D, c = 0.9, 1.0
    atoms = synth.globule(200, 1001)
    ref = oracle.partition(atoms, D, c=c, uniform=True, h0=2.0, h_min=2.0)
    cells = ctx.build_cells(atoms, tms.make_params(D=D, c=c, tau=1e-3))
    assert np.array_equal(cells.origin, ref.origin)
    L, cp = _synthetic_leaves(120_000, cells.dims, cells.K, c, 99)
    R_g, nd_g = _gpu_stage2(ctx, cells, L, cp)
    ijk = np.stack([L["ix"], L["iy"], L["iz"]], 1)
    so = oracle.stage2_points(ijk, L["level"], L["cls"], cp, c, ref.origin, 2.0)
    print("degenerate: gpu %d oracle %d; fold %d critical %d"
          % (nd_g, so.n_degenerate, np.sum(so.pts["kind"] == 0), np.sum(so.pts["kind"] == 1)))
    assert so.n_mismatch == 0
    assert nd_g == so.n_degenerate and nd_g >= 1000
    h_leaf = 2.0 * 2.0 ** -L["level"].astype(np.float64)
    n = _compare(R_g, so.pts, so.leaf_margin, h_leaf, 1e-9, 1e-10)
    assert n > 100_000
    # every record is a leaf of the SURFACE class, in leaf order
    assert np.all(L["cls"][R_g["leaf"]] == tms.CLS_SURFACE)
    assert np.all(np.diff(R_g["leaf"]) >= 0)
    ctx.free_cells(cells)


def test_stage2_capacity(ctx):
    import torch
    atoms = synth.globule(200, 1001)
    cells = ctx.build_cells(atoms, tms.make_params(D=0.9))
    L, cp = _synthetic_leaves(2000, cells.dims, cells.K, 1.0, 5)
    lt = torch.as_tensor(np.frombuffer(L.tobytes(), dtype=np.uint8).reshape(-1, 20)).to(ctx.device)
    ct = torch.as_tensor(cp).to(ctx.device).contiguous()
    full, _ = ctx.stage2_points(cells, lt, ct)
    with pytest.raises(tms.TmsError) as ei:
        ctx.stage2_points(cells, lt, ct, cap=len(full) - 1)
    assert ei.value.code == tms.TMS_E_CAPACITY
    again, _ = ctx.stage2_points(cells, lt, ct, cap=len(full) + 10)
    assert torch.equal(full, again)
    empty, nd = ctx.stage2_points(cells, lt[:0], ct[:0])
    assert len(empty) == 0 and nd == 0
    ctx.free_cells(cells)


@pytest.mark.parametrize("which", ["globule1000", "globule5k_D0.9"])
def test_stage2_end_to_end_fp64(ctx, which):
    if which == "globule1000":
        atoms, D = synth.globule(1000, 1006), 0.9
    else:
        w = workloads.GLOBULE5K[0.9]
        atoms, D = workloads.atoms(w), w.D
    c = 1.0
    cells = ctx.build_cells(atoms, tms.make_params(D=D, c=c, tau=1e-3,
                                                   precision=tms.PREC_FP64))
    leaves, cphi, _ = ctx.partition_estimate(cells)
    recs, nd_g = ctx.stage2_points(cells, leaves, cphi)
    R_g = tms.s2_to_numpy(recs)
    L = tms.leaves_to_numpy(leaves)
    ref = oracle.partition(atoms, D, c=c, tau=1e-3)
    same = (len(L) == ref.n_leaves
            and np.array_equal(np.stack([L["ix"], L["iy"], L["iz"]], 1), ref.ijk)
            and np.array_equal(L["level"], ref.level) and np.array_equal(L["cls"], ref.cls))
    # the partition parity tests allow differences only inside oracle near-tie
    # subtrees; records are matched by leaf index, which needs equal lists
    assert same or ref.tie_cube + ref.tie_corner > 0
    if not same:
        pytest.skip("a near-tie subtree changed the leaf list: records cannot be matched by index")
    so = oracle.stage2_of(ref, c)
    print("%s: %d surface leaves, fold %d, critical %d, degenerate gpu %d oracle %d"
          % (which, np.sum(L["cls"] == tms.CLS_SURFACE), np.sum(so.pts["kind"] == 0),
             np.sum(so.pts["kind"] == 1), nd_g, so.n_degenerate))
    assert so.n_mismatch == 0 and nd_g == so.n_degenerate
    h_leaf = 2.0 * 2.0 ** -L["level"].astype(np.float64)
    n = _compare(R_g, so.pts, so.leaf_margin, h_leaf, 1e-6, 1e-8)
    assert n > 0
    ctx.free_cells(cells)
