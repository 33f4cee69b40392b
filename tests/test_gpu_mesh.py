"""The Stage-2 mesh (Section 2.3) of the HIP path's partitions, with and
without closing open faces, against the oracle.

* Unclosed: tms_mesh_build on the device partition gives the same triangles
  (vertex indices, leaf of each triangle) as tms_mesh_build_host on the
  oracle's partition of the same atoms (FP64: identical leaf lists and
  vertex keys), and positions within 2e-12.
* Closed: the cubes the library adds across open faces are exactly the
  oracle's (oracle/mesh.close_open_faces over the oracle's partition, phi of
  the oracle at the new corners), their corner values within the parity bar;
  the closed mesh has no open face, and the library's check report equals
  the oracle checker's on it with no defect of (a), (b) or (c).
* A sphere whose unclosed mesh has holes closes into a sphere (Euler
  characteristic 2, area within 1 % of the closed form); the 5,000-atom
  globule and the 110,000-atom assembly in FP32+guard close into manifolds
  with no defect of (a), (b) or (c); the added cubes' corner values are the
  oracle's phi (1e-5 relative, the FP32+guard bar).
* SURFACE leaves of two levels (loose tolerances): the finest cubes that
  replace the coarser leaves, and the closing cubes after them, equal the
  oracle's; the mesh has no defect.
* The mesh's extreme points on leaf faces are the ends of the fold segments
  the GPU's Stage-2 kernel writes for the same partition.
* Vertex density scales as 1 / h_min^2 (about 2.3 per square angstrom at
  h_min = 1, 1.5 of them edge points).
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from oracle import mesh as om
from paper_1611_03474_amd import synth, tms, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = tms.Context(0)
    yield c
    c.close()


def _gpu_meshes(ctx, atoms, prec, **kw):
    p = tms.make_params(precision=prec, **kw)
    cells = ctx.build_cells(atoms, p)
    try:
        leaves, cphi, _ = ctx.partition_estimate(cells)
        verts = ctx.extract(cells, leaves, cphi)
        open_m = ctx.mesh_build(cells, leaves, cphi, verts, close=False)
        closed = ctx.mesh_build(cells, leaves, cphi, verts, close=True)
        L = tms.leaves_to_numpy(leaves)
    finally:
        ctx.free_cells(cells)
    return L, open_m, closed


def _oracle_host_mesh(r, c, h0):
    L = np.zeros(r.n_leaves, dtype=tms.LEAF_DTYPE)
    L["ix"], L["iy"], L["iz"] = r.ijk[:, 0], r.ijk[:, 1], r.ijk[:, 2]
    L["level"], L["reason"], L["mask"], L["cls"] = r.level, r.reason, r.mask, r.cls
    V = np.zeros(r.n_vert, dtype=tms.VERTEX_DTYPE)
    V["edge_key"], V["t"] = r.vkey, r.vt
    V["x"], V["y"], V["z"] = r.vxyz[:, 0], r.vxyz[:, 1], r.vxyz[:, 2]
    return tms.mesh_build_host(L, r.corner_phi, V, c, r.K, h0)


def _oracle_closure(r, atoms, D, c, h0):
    surf = r.cls == oracle.CLS_SURFACE
    lev = int(r.level[surf][0]) if surf.any() else r.K
    h = h0 / (1 << lev)
    dims = tuple(int(d) << lev for d in r.dims)

    def phi_at(P):
        return oracle.phi(atoms, D, r.origin + P * h)

    same = r.level == lev
    return om.close_open_faces(r.ijk[same], r.corner_phi[same], surf[same], c, dims, phi_at)


# atoms and seeds whose oracle partition has no near tie; the first two and
# the 200-atom globule of seed 1002 have open faces before closing
CASES = {
    "sphere_with_holes": (np.array([[-2.8735, -1.1366, 2.6300, 1.6307]]), 0.9),
    "sphere_with_holes2": (np.array([[2.8824, 0.0931, 0.1270, 1.9172]]), 0.9),
    "globule200_open": (synth.globule(200, 1002), 0.9),
    "globule200": (synth.globule(200, 1001), 0.9),
    "globule1000": (synth.globule(1000, 1006), 0.9),
}


@pytest.mark.parametrize("name", list(CASES))
def test_mesh_parity_fp64(ctx, name):
    atoms, D = CASES[name]
    c, h0 = 1.0, 2.0
    print("case", name, flush=True)
    L, mo, mc = _gpu_meshes(ctx, atoms, tms.PREC_FP64, D=D)
    r = oracle.partition(atoms, D, c=c, tau=1e-3, h0=h0, h_min=0.25)
    assert r.tie_cube == 0 and r.tie_corner == 0, "near ties: pick another seed"
    ref = _oracle_host_mesh(r, c, h0)
    # unclosed: same triangles as the host mesher on the oracle's partition
    assert np.array_equal(mo.tri, ref.tri) and np.array_equal(mo.tri_leaf, ref.tri_leaf)
    assert np.max(np.abs(mo.xyz - ref.xyz), initial=0.0) < 2e-12
    assert mo.info["open_faces"] == ref.info["open_faces"] and len(mo.added) == 0
    # closed: the oracle's closure of its own partition
    keys, aphi = _oracle_closure(r, atoms, D, c, h0)
    got = sorted(zip(mc.added["ix"].tolist(), mc.added["iy"].tolist(), mc.added["iz"].tolist()))
    print("open faces %d, added cubes: library %d, oracle %d"
          % (mo.info["open_faces"], len(got), len(keys)))
    assert got == keys
    order = np.lexsort((mc.added["iz"], mc.added["iy"], mc.added["ix"]))
    if len(keys):
        assert np.max(np.abs(mc.added_phi[order] - aphi) / np.abs(aphi)) < 1e-12
        assert np.all(mc.added["reason"] == tms.REASON_CLOSED)
        assert np.all(mc.added["cls"] == tms.CLS_SURFACE)
    if name in ("sphere_with_holes", "sphere_with_holes2", "globule200_open"):
        assert mo.info["open_faces"] > 0 and len(keys) > 0
    assert mc.info["open_faces"] == 0
    assert np.all(mc.tri_leaf < len(L) + len(mc.added))
    rep = mc.check()
    oref = om.check_mesh(mc.xyz, mc.tri, cell=0.5)
    print(rep)
    for k in ("boundary_edges", "nonmanifold_edges", "misoriented_edges", "nonmanifold_vertices",
              "intersecting_pairs", "components", "euler"):
        assert rep[k] == oref[k], k
    assert rep["boundary_edges"] == rep["nonmanifold_vertices"] == rep["intersecting_pairs"] == 0
    assert rep["misoriented_edges"] == rep["nonmanifold_edges"] == 0
    assert rep["euler"] % 2 == 0 and rep["volume"] > 0
    if name.startswith("sphere"):
        R = atoms[0, 3]  # c = 1: phi = 1 on the sphere of radius r_i
        assert rep["euler"] == 2 and rep["components"] == 1
        assert abs(rep["area"] / (4 * np.pi * R * R) - 1) < 0.01


def test_face_points_equal_gpu_stage2_fold_ends(ctx):
    # two implementations of eq. curve on one device partition: the host
    # mesher's extreme points on the leaves' faces, and the ends of the fold
    # segments tms_stage2_points writes on the GPU (the stored lower end on
    # the face axis = -1, the upper end one leaf edge along the axis)
    atoms, D = CASES["globule200"]
    cells = ctx.build_cells(atoms, tms.make_params(precision=tms.PREC_FP64, D=D))
    try:
        leaves, cphi, _ = ctx.partition_estimate(cells)
        verts = ctx.extract(cells, leaves, cphi)
        m = ctx.mesh_build(cells, leaves, cphi, verts, close=False)
        recs, ndeg = ctx.stage2_points(cells, leaves, cphi)
        R = tms.s2_to_numpy(recs)
        L = tms.leaves_to_numpy(leaves)
        nv, h0 = verts.shape[0], cells.params.h0
    finally:
        ctx.free_cells(cells)
    assert ndeg == 0 and len(m.added) == 0
    F = m.xyz[nv:len(m.xyz) - m.info["n_fallback"]]
    f = R[R["kind"] == tms.S2_FOLD]
    lo = np.stack([f["x"], f["y"], f["z"]], 1)
    hi = lo.copy()
    hi[np.arange(len(f)), f["axis"]] += h0 * 2.0 ** (-L["level"][f["leaf"]].astype(np.float64))
    O = np.concatenate([lo, hi])
    print("face points %d, GPU fold ends %d" % (len(F), len(O)))
    assert len(F) == len(O) > 0
    assert cKDTree(O).query(F)[0].max() < 1e-9
    assert cKDTree(F).query(O)[0].max() < 1e-9


def test_closed_mesh_globule5k_fp32g(ctx):
    w = workloads.GLOBULE5K[0.9]
    atoms = workloads.atoms(w)
    print("case globule5k fp32g", flush=True)
    L, mo, mc = _gpu_meshes(ctx, atoms, tms.PREC_FP32_GUARD, D=w.D, tau=1e-3)
    rep = mc.check()
    print(mo.info, rep)
    assert mc.info["open_faces"] == 0
    assert rep["boundary_edges"] == rep["nonmanifold_vertices"] == rep["intersecting_pairs"] == 0
    assert rep["misoriented_edges"] == rep["nonmanifold_edges"] == 0
    assert rep["unused_vertices"] == 0 and rep["euler"] % 2 == 0 and rep["volume"] > 0
    # the added cubes straddle c and touch the surface through a crossing face
    a = mc.added
    assert np.all(a["cls"] == tms.CLS_SURFACE)
    assert np.all((mc.added_phi >= 1.0).any(1) & (mc.added_phi < 1.0).any(1))


def test_closed_mesh_assembly110k(ctx):
    # the benchmark's workload at full size (FP32+guard, default launch
    # shapes): the closed mesh meets all three conditions, including (c)
    # over every pair of triangles of touching leaves; the corner values of
    # a sample of the added cubes are phi of the oracle at those points
    w = workloads.ASSEMBLY110K
    atoms = workloads.atoms(w)
    print("case assembly110k fp32g", flush=True)
    cells = ctx.build_cells(atoms, w.params(tms.PREC_FP32_GUARD))
    try:
        leaves, cphi, _ = ctx.partition_estimate(cells)
        verts = ctx.extract(cells, leaves, cphi)
        m = ctx.mesh_build(cells, leaves, cphi, verts, close=True)
        origin, K = np.array(cells.origin), cells.K
    finally:
        ctx.free_cells(cells)
    rep = m.check(intersections=True)
    print(rep)
    assert rep["n_triangles"] > 10_000_000 and rep["open_faces"] == 0
    assert rep["boundary_edges"] == rep["nonmanifold_edges"] == rep["misoriented_edges"] == 0
    assert rep["nonmanifold_vertices"] == rep["intersecting_pairs"] == 0
    assert rep["unused_vertices"] == 0 and rep["euler"] % 2 == 0 and rep["volume"] > 0
    a, ap = m.added, m.added_phi
    assert np.all(a["reason"] == tms.REASON_CLOSED) and np.all(a["level"] == K)
    rng = np.random.default_rng(12)
    pick = rng.choice(len(a), min(50, len(a)), replace=False)
    h = w.h0 / (1 << K)
    off = np.array([[v & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)])
    ijk = np.stack([a["ix"], a["iy"], a["iz"]], 1)[pick]
    pts = origin + ((ijk[:, None, :] + off[None]) * h).reshape(-1, 3)
    ref = oracle.phi(atoms, w.D, pts).reshape(-1, 8)
    assert np.max(np.abs(ap[pick] - ref) / ref) < 1e-5


def test_vertex_density_follows_h_min(ctx):
    # the mesh's vertices are edge points of the finest lattice and extreme
    # points on its faces, so the density per unit area scales as
    # 1 / h_min^2 (Section 3.1 tunes it to 1 and 2 vertices per square
    # angstrom; h_min = 1 gives about 2.3, 1.5 of them edge points); every
    # level's closed mesh has no defect
    w = workloads.GLOBULE5K[0.9]
    atoms = workloads.atoms(w)
    dens = {}
    for h_min in (1.0, 0.5, 0.25):
        print("case globule5k h_min %g" % h_min, flush=True)
        p = tms.make_params(D=w.D, tau=1e-3, h0=2.0, h_min=h_min,
                            precision=tms.PREC_FP32_GUARD)
        cells = ctx.build_cells(atoms, p)
        try:
            leaves, cphi, _ = ctx.partition_estimate(cells)
            verts = ctx.extract(cells, leaves, cphi)
            m = ctx.mesh_build(cells, leaves, cphi, verts, close=True)
        finally:
            ctx.free_cells(cells)
        rep = m.check(intersections=True)
        print(h_min, rep)
        assert rep["open_faces"] == 0 and rep["boundary_edges"] == 0
        assert rep["nonmanifold_vertices"] == rep["intersecting_pairs"] == 0
        assert rep["misoriented_edges"] == rep["nonmanifold_edges"] == 0
        dens[h_min] = rep["density"]
    assert 1.0 < dens[1.0] < 3.0
    for a, b in ((1.0, 0.5), (0.5, 0.25)):
        assert 3.0 < dens[b] / dens[a] < 5.0


SPLIT_CASES = {
    # loose tolerances stop some straddling cubes above the finest level
    "globule600_D0.5_tau0.1": (synth.globule(600, 1011), 0.5, 0.1),
    "globule600_D0.9_tau0.3": (synth.globule(600, 1012), 0.9, 0.3),
}


@pytest.mark.parametrize("name", list(SPLIT_CASES))
def test_mixed_levels_fp64(ctx, name):
    # SURFACE leaves of two levels: the library meshes the coarser ones
    # through their straddling cubes of the finest level; those cubes, and
    # then the cubes added across open faces, equal the oracle's (from its
    # own partition and phi), and the mesh has no defect
    atoms, D, tau = SPLIT_CASES[name]
    c, h0 = 1.0, 2.0
    print("case", name, flush=True)
    p = tms.make_params(D=D, tau=tau, precision=tms.PREC_FP64)
    cells = ctx.build_cells(atoms, p)
    try:
        leaves, cphi, _ = ctx.partition_estimate(cells)
        verts = ctx.extract(cells, leaves, cphi)
        m = ctx.mesh_build(cells, leaves, cphi, verts, close=True)
        V = tms.vertices_to_numpy(verts)
    finally:
        ctx.free_cells(cells)
    r = oracle.partition(atoms, D, c=c, tau=tau, h0=h0, h_min=0.25)
    assert r.tie_cube == 0 and r.tie_corner == 0
    K = r.K
    surf = r.cls == oracle.CLS_SURFACE
    assert (r.level[surf] < K).any()
    h = h0 / (1 << K)

    def phi_at(P):
        return oracle.phi(atoms, D, r.origin + P * h)

    sk, sv = om.straddling(om.split_coarse(r.ijk, r.level, r.corner_phi, surf, K, phi_at), c)
    a = m.added
    ijk = np.stack([a["ix"], a["iy"], a["iz"]], 1)
    sp = a["reason"] == tms.REASON_SPLIT
    got = sorted(map(tuple, ijk[sp].tolist()))
    print("split cubes: library %d, oracle %d" % (len(got), len(sk)))
    assert got == sk
    o = np.lexsort((ijk[sp, 2], ijk[sp, 1], ijk[sp, 0]))
    assert np.max(np.abs(m.added_phi[sp][o] - sv) / np.abs(sv)) < 1e-12
    # closing over the finest SURFACE leaves and the split cubes
    fine = surf & (r.level == K)
    keys, _ = om.close_open_faces(np.vstack([r.ijk[fine], np.array(sk)]),
                                  np.vstack([r.corner_phi[fine], sv]),
                                  np.ones(int(fine.sum()) + len(sk), bool), c,
                                  tuple(int(d) << K for d in r.dims), phi_at)
    cl = a["reason"] == tms.REASON_CLOSED
    assert sorted(map(tuple, ijk[cl].tolist())) == keys
    rep = m.check(intersections=True)
    print(rep)
    assert rep["open_faces"] == 0 and rep["boundary_edges"] == 0
    assert rep["nonmanifold_edges"] == rep["misoriented_edges"] == 0
    assert rep["nonmanifold_vertices"] == rep["intersecting_pairs"] == 0
    # the coarse leaves' own edge points are the only unused vertices
    assert rep["unused_vertices"] == int((((V["edge_key"] >> 50) & 7) < K).sum())


def test_empty_partition_and_bad_flags(ctx):
    # no atoms: no leaves, an empty mesh; unknown flags are refused
    p = tms.make_params(precision=tms.PREC_FP64)
    cells = ctx.build_cells(np.zeros((0, 4)), p)
    try:
        leaves, cphi, _ = ctx.partition_estimate(cells)
        verts = ctx.extract(cells, leaves, cphi)
        assert leaves.shape[0] == 0 and verts.shape[0] == 0
        m = ctx.mesh_build(cells, leaves, cphi, verts)
        rep = m.check()
        assert rep["n_triangles"] == rep["n_vertices"] == 0 and len(m.added) == 0
        import ctypes as C
        h = C.c_void_p()
        rc = ctx.lib.tms_mesh_build(ctx.h, cells.handle, None, 0, None, None, 0, 2, C.byref(h))
        assert rc == tms.TMS_E_INVALID
    finally:
        ctx.free_cells(cells)


def test_batch_conformations_mesh_as_single_passes(ctx):
    # each conformation of a batch meshed from its ranges of the batch's
    # leaves and vertices (the closing cubes evaluated for that conformation)
    # equals the mesh of its own single pass; a range spanning two
    # conformations is refused
    confs = [synth.globule(200, 1002), synth.globule(300, 1013), synth.globule(200, 1001)]
    p = tms.make_params(D=0.9, tau=1e-3, precision=tms.PREC_FP32_GUARD)
    cells = ctx.build_cells_batch(confs, p)
    try:
        leaves, cphi, _ = ctx.partition_estimate(cells)
        verts = ctx.extract(cells, leaves, cphi)
        lo, vo = ctx.batch_counts(cells)
        meshes = [ctx.mesh_build(cells, leaves[lo[b]:lo[b + 1]], cphi[lo[b]:lo[b + 1]],
                                 verts[vo[b]:vo[b + 1]]) for b in range(len(confs))]
        with pytest.raises(tms.TmsError):
            ctx.mesh_build(cells, leaves[lo[0]:lo[2]], cphi[lo[0]:lo[2]], verts[vo[0]:vo[2]])
    finally:
        ctx.free_cells(cells)
    n_added = 0
    for b, atoms in enumerate(confs):
        L, mo, ms = _gpu_meshes(ctx, atoms, tms.PREC_FP32_GUARD, D=0.9, tau=1e-3)
        mb = meshes[b]
        assert np.array_equal(mb.tri, ms.tri) and np.array_equal(mb.tri_leaf, ms.tri_leaf)
        assert np.array_equal(mb.xyz, ms.xyz)
        assert np.array_equal(mb.added_phi, ms.added_phi)
        for f in ("ix", "iy", "iz", "level", "reason", "mask", "cls"):
            assert np.array_equal(mb.added[f], ms.added[f])
        assert np.all(mb.added["conf"] == b)
        assert mb.check() == ms.check()
        n_added += len(mb.added)
    assert n_added > 0  # the first globule has open faces
