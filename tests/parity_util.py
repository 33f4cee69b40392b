"""Element-by-element comparison of HIP-path results with the FP64 oracle.

Shared by the GPU parity tests.  Bars:
  * discrete results -- leaf list, levels, reasons, masks, classes, vertex
    keys -- bit-exact, in order;
  * corner values: FP64 path 1e-12 relative, FP32+guard path 1e-5 relative;
  * vertex t: FP64 path 1e-11 absolute, FP32+guard path 1e-5 absolute;
  * vertex positions: 2e-12 / 2e-5 absolute (t times an edge of <= 2).
Cubes the oracle reports as near ties (a decision margin below 1e-9
relative, where two FP64 codes may legitimately differ) are excluded with
their whole subtree, and so are leaves touching a near-tie corner; the
counts are printed.
"""
import numpy as np

import oracle
from paper_1611_03474_amd import tms

PNAME = {tms.PREC_FP64: "fp64", tms.PREC_FP32_GUARD: "fp32g"}


def phi_tol(prec):
    return 1e-12 if prec == tms.PREC_FP64 else 1e-5


def taint(level, ijk, K, tie_cubes, tie_corner_keys):
    """Boolean mask of leaves inside an oracle near-tie cube or touching a
    near-tie corner."""
    bad = np.zeros(len(level), dtype=bool)
    if len(level) == 0:
        return bad
    sh = K - level.astype(np.int64)
    lo = ijk.astype(np.int64) << sh[:, None]
    hi = (ijk.astype(np.int64) + 1) << sh[:, None]
    for lev, x, y, z in tie_cubes:
        s = K - int(lev)
        tlo = np.array([x, y, z], dtype=np.int64) << s
        thi = (np.array([x, y, z], dtype=np.int64) + 1) << s
        bad |= np.all((lo < thi) & (hi > tlo), axis=1)
    for key in tie_corner_keys:
        p = np.array([(int(key) >> 32) & 0xFFFF, (int(key) >> 16) & 0xFFFF, int(key) & 0xFFFF])
        bad |= np.all((lo <= p) & (hi >= p), axis=1)
    return bad


def run_gpu(ctx, atoms, prec, **kw):
    p = tms.make_params(precision=prec, **kw)
    cells = ctx.build_cells(atoms, p)
    leaves, cphi, st = ctx.partition_estimate(cells)
    verts = ctx.extract(cells, leaves, cphi)
    out = dict(origin=np.array(cells.origin), dims=np.array(cells.dims),
               leaves=tms.leaves_to_numpy(leaves), cphi=cphi.cpu().numpy(),
               verts=tms.vertices_to_numpy(verts), stats=st)
    ctx.free_cells(cells)
    return out


def compare_lists(L, cphi, V, ref, prec, label="", n_est=None):
    """Full comparison of one conformation's GPU leaves L (LEAF_DTYPE),
    corner values cphi [n][8] and vertices V (VERTEX_DTYPE) with an oracle
    result.  Returns the number of excluded (near-tie) GPU leaves."""
    ijk = np.stack([L["ix"], L["iy"], L["iz"]], axis=1)
    bad_g = taint(L["level"], ijk, ref.K, ref.tie_cubes, ref.tie_corner_keys)
    bad_r = taint(ref.level, ref.ijk, ref.K, ref.tie_cubes, ref.tie_corner_keys)
    print("%s %s: leaves %d (oracle %d), vertices %d (oracle %d), near-tie cubes %d corners %d,"
          " excluded leaves %d/%d"
          % (label, PNAME[prec], len(L), ref.n_leaves, len(V), ref.n_vert, ref.tie_cube,
             ref.tie_corner, bad_g.sum(), bad_r.sum()))
    if n_est is not None and ref.tie_cube == 0:
        assert np.array_equal(np.asarray(n_est)[:ref.K + 1], ref.n_est[:ref.K + 1])
    g_keep, r_keep = ~bad_g, ~bad_r
    assert g_keep.sum() == r_keep.sum()
    for f_g, f_r in [(L["level"], ref.level), (L["ix"], ref.ijk[:, 0]), (L["iy"], ref.ijk[:, 1]),
                     (L["iz"], ref.ijk[:, 2]), (L["reason"], ref.reason), (L["mask"], ref.mask),
                     (L["cls"], ref.cls)]:
        assert np.array_equal(np.asarray(f_g)[g_keep].astype(np.int64),
                              np.asarray(f_r)[r_keep].astype(np.int64))
    cg, cr = cphi[g_keep], ref.corner_phi[r_keep]
    tol = phi_tol(prec)
    if len(cr):
        rel = np.max(np.abs(cg - cr) / np.maximum(np.abs(cr), 1e-300))
        print("  max relative corner-value error %.3e" % rel)
    assert np.all(np.abs(cg - cr) <= tol * np.maximum(np.abs(cr), 1e-300) + 1e-300)
    if bad_r.any() or bad_g.any():
        # near ties present: compare t on the shared edge keys; the keys that
        # differ must come from the excluded subtrees (12 edges per leaf)
        common, ig, ir = np.intersect1d(V["edge_key"], ref.vkey, return_indices=True)
        tg, tr = V["t"][ig], ref.vt[ir]
        assert len(V) - len(common) <= 12 * bad_g.sum()
        assert ref.n_vert - len(common) <= 12 * bad_r.sum()
    else:
        assert np.array_equal(V["edge_key"], ref.vkey)
        tg, tr = V["t"], ref.vt
        assert np.allclose(np.stack([V["x"], V["y"], V["z"]], 1), ref.vxyz, rtol=0,
                           atol=(1e-12 if prec == tms.PREC_FP64 else 1e-5) * 2.0)
    ttol = 1e-11 if prec == tms.PREC_FP64 else 1e-5
    print("  max vertex t error %.3e" % np.max(np.abs(tg - tr), initial=0.0))
    assert np.max(np.abs(tg - tr), initial=0.0) <= ttol
    return int(bad_g.sum())


def compare(ctx, atoms, prec, D=0.9, ref=None, label="", **kw):
    """Run the HIP path and the oracle on the same atoms and compare."""
    okw = {k: v for k, v in kw.items() if k in ("c", "tau", "h0", "h_min", "pad", "eps_cut")}
    uniform = kw.get("mode", tms.MODE_ADAPTIVE) == tms.MODE_UNIFORM
    if ref is None:
        ref = oracle.partition(atoms, D, uniform=uniform, **okw)
    got = run_gpu(ctx, atoms, prec, D=D, **kw)
    assert np.array_equal(got["origin"], ref.origin)
    assert np.array_equal(got["dims"], ref.dims)
    print("%s guard cubes %d points %d" % (label, got["stats"]["guard_cubes"],
                                           got["stats"]["guard_points"]))
    compare_lists(got["leaves"], got["cphi"], got["verts"], ref, prec, label=label,
                  n_est=got["stats"]["n_est"])
    return got, ref
