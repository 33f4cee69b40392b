"""The captured pass (one HIP graph, every size on the device) against the
eager pass of the same cells: bit-identical leaves, corner values, vertices,
per-conformation offsets and counters, over several replays with eager work
in between."""
import numpy as np
import pytest

from paper_1611_03474_amd import synth, tms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = tms.Context(0)
    yield c
    c.close()


def _eager(ctx, cells):
    leaves, cphi, st = ctx.partition_estimate(cells)
    verts = ctx.extract(cells, leaves, cphi)
    return leaves.clone(), cphi.clone(), verts.clone(), st


def _check_replays(ctx, cells, n_conf, reps=3, bound=False):
    import torch
    L0, C0, V0, st0 = _eager(ctx, cells)
    lo0 = vo0 = None
    if n_conf > 1:
        lo0, vo0 = ctx.batch_counts(cells)
    if bound:
        # the graph writes straight into these (no copies on replay)
        lcap, vcap = ctx.graph_capacity(cells, margin=1.25)
        assert lcap >= L0.shape[0] and vcap >= V0.shape[0]
        lb = torch.empty((lcap, 20), dtype=torch.uint8, device="cuda:0")
        cb = torch.empty((lcap, 8), dtype=torch.float64, device="cuda:0")
        vb = torch.empty((vcap, 40), dtype=torch.uint8, device="cuda:0")
        ctx.graph_capture(cells, margin=1.25, leaves=lb, cphi=cb, verts=vb)
        # a bound buffer below the capacity is refused, and the capture stays
        with pytest.raises(tms.TmsError):
            ctx.graph_capture(cells, margin=1.25, leaves=lb[:lcap - 1], cphi=cb[:lcap - 1],
                              verts=vb)
        with pytest.raises(tms.TmsError):
            ctx.graph_capture(cells, margin=1.25, verts=vb[:vcap - 1])
    else:
        ctx.graph_capture(cells, margin=1.25)
        lb = torch.empty((L0.shape[0] + 100, 20), dtype=torch.uint8, device="cuda:0")
        cb = torch.empty((L0.shape[0] + 100, 8), dtype=torch.float64, device="cuda:0")
        vb = torch.empty((V0.shape[0] + 100, 40), dtype=torch.uint8, device="cuda:0")
    for r in range(reps):
        lb.fill_(0)
        vb.fill_(0)
        nl, nv, st, (lo, vo) = ctx.graph_launch(cells, lb, cb, vb, offsets=True)
        assert nl == L0.shape[0] and nv == V0.shape[0], r
        assert torch.equal(lb[:nl], L0) and torch.equal(cb[:nl], C0) and torch.equal(vb[:nv], V0), r
        for k in ("n_est", "n_disc", "n_refine", "n_conv", "n_hmin", "n_leaves", "n_surface",
                  "n_corners", "n_bound", "guard_cubes", "guard_points", "n_pairs"):
            assert st[k] == st0[k], (r, k, st[k], st0[k])
        if n_conf > 1:
            assert np.array_equal(lo, lo0) and np.array_equal(vo, vo0)
        # eager work on the same context between replays
        ctx.eval_phi(cells, torch.zeros((5, 3), dtype=torch.float64, device="cuda:0")) \
            if n_conf == 1 else ctx.partition_estimate(cells)
        torch.cuda.synchronize()
    if bound:
        # a replay into other buffers copies the results there
        l2, c2, v2 = torch.zeros_like(L0), torch.zeros_like(C0), torch.zeros_like(V0)
        nl, nv, _ = ctx.graph_launch(cells, l2, c2, v2)
        assert nl == L0.shape[0] and nv == V0.shape[0]
        assert torch.equal(l2, L0) and torch.equal(c2, C0) and torch.equal(v2, V0)


@pytest.mark.parametrize("prec", [tms.PREC_FP64, tms.PREC_FP32_GUARD], ids=["fp64", "fp32g"])
def test_graph_single(ctx, prec):
    atoms = synth.globule(1000, 1006)
    cells = ctx.build_cells(atoms, tms.make_params(D=0.9, tau=0.1, precision=prec))
    _check_replays(ctx, cells, 1)
    ctx.free_cells(cells)


@pytest.mark.parametrize("n_conf", [1, 4], ids=["single", "batch"])
def test_graph_bound_outputs(ctx, n_conf):
    confs = [synth.globule(n, 3100 + k) for k, n in enumerate([600, 150, 400, 250][:n_conf])]
    p = tms.make_params(D=0.9, tau=0.1, precision=tms.PREC_FP32_GUARD)
    cells = ctx.build_cells(confs[0], p) if n_conf == 1 else ctx.build_cells_batch(confs, p)
    _check_replays(ctx, cells, n_conf, bound=True)
    ctx.free_cells(cells)


@pytest.mark.parametrize("proj_table,half,tml", [(1, 0, 1), (0, 0, 1), (1, 1, 1), (1, 2, 1),
                                                  (1, 0, 0)],
                         ids=["table", "in_place", "half_chunks", "half_level2", "grouped_level0"])
def test_graph_batch_sliced(ctx, proj_table, half, tml):
    # a batch, with queue slices far smaller than the levels so the slicing
    # of the captured pass is exercised too
    confs = [synth.globule(n, 3000 + k) for k, n in enumerate([300, 120, 500, 220])]
    cells = ctx.build_cells_batch(confs, tms.make_params(D=0.9, tau=1e-3,
                                                         precision=tms.PREC_FP32_GUARD))
    base = ctx.get_tuning().as_dict()
    ctx.set_tuning(slice_cubes=4096, proj_table=proj_table, tiled_half=half,
                   tiled_min_level=tml)
    try:
        _check_replays(ctx, cells, len(confs))
    finally:
        ctx.set_tuning(**base)
    ctx.free_cells(cells)


def test_graph_rejects_without_eager_pass(ctx):
    atoms = synth.globule(200, 1001)
    cells = ctx.build_cells(atoms, tms.make_params(tau=0.1))
    with pytest.raises(tms.TmsError):
        ctx.graph_capture(cells)
    with pytest.raises(tms.TmsError):
        ctx.graph_capacity(cells)
    ctx.partition_estimate(cells)
    with pytest.raises(tms.TmsError):  # the extraction is missing too
        ctx.graph_capacity(cells)
    ctx.free_cells(cells)


def test_graph_replay_on_rebuilt_cells(ctx):
    # the captured pass replayed on cells rebuilt in place from slightly moved
    # atoms (same geometry): the counts shift against the capture's (queues,
    # chunks per slice, leaves, corners, vertices), so the replay either
    # matches an eager pass on the new cells bit for bit or reports the
    # exceeded capacity -- never a wrong result
    import torch
    confs = [synth.globule(n, 4000 + k) for k, n in enumerate([400, 250, 600])]
    p = tms.make_params(D=0.9, tau=1e-3, precision=tms.PREC_FP32_GUARD)
    base = ctx.get_tuning().as_dict()
    ctx.set_tuning(slice_cubes=4096)
    try:
        cells = ctx.build_cells_batch(confs, p)
        L0, _, V0, _ = _eager(ctx, cells)
        ctx.graph_capture(cells, margin=1.25)
        nlc, nvc = 2 * L0.shape[0] + 1024, 2 * V0.shape[0] + 1024
        replayed = 0
        for seed in range(4):
            rng = np.random.default_rng(50 + seed)
            moved = []
            for c in confs:
                m = np.array(c, dtype=np.float64)
                m[:, :3] += rng.normal(0.0, 0.02, size=(len(m), 3))
                moved.append(m)
            ctx.build_cells_batch(moved, p, cells)
            lb = torch.zeros((nlc, 20), dtype=torch.uint8, device="cuda:0")
            cb = torch.zeros((nlc, 8), dtype=torch.float64, device="cuda:0")
            vb = torch.zeros((nvc, 40), dtype=torch.uint8, device="cuda:0")
            try:
                nl, nv, st = ctx.graph_launch(cells, lb, cb, vb)
            except tms.TmsError as e:
                assert e.code in (tms.TMS_E_CAPACITY, tms.TMS_E_INVALID), e
                print("seed %d: replay refused (%s)" % (seed, e))
                continue
            L1, C1, V1, st1 = _eager(ctx, cells)
            assert nl == L1.shape[0] and nv == V1.shape[0], seed
            assert torch.equal(lb[:nl], L1) and torch.equal(cb[:nl], C1), seed
            assert torch.equal(vb[:nv], V1), seed
            assert st["n_est"] == st1["n_est"], seed
            replayed += 1
        print("replays on rebuilt cells that matched the eager pass: %d of 4" % replayed)
        assert replayed >= 1
        ctx.free_cells(cells)
    finally:
        ctx.set_tuning(**base)


def test_graph_refuses_rebuild_with_other_atom_count(ctx):
    # cells first built with one atom more, then rebuilt in place without it
    # and captured: a rebuild back to the larger set keeps the geometry (the
    # extra atom sits inside the box, with the smallest radius) and the
    # buffers (they only grow), but the captured launches and the projection
    # table's rows were sized by the smaller atom count, so the replay is
    # refused; the captured set itself replays
    atoms = synth.globule(400, 4100)
    extra = np.concatenate([atoms, [[*atoms[:, :3].mean(axis=0), atoms[:, 3].min()]]], axis=0)
    p = tms.make_params(D=0.9, tau=1e-3, precision=tms.PREC_FP32_GUARD)
    cells = ctx.build_cells(extra, p)
    cells = ctx.build_cells(atoms, p, cells)
    L0, _, V0, _ = _eager(ctx, cells)
    ctx.graph_capture(cells, margin=1.25)
    nl, nv, _ = ctx.graph_launch(cells)
    assert nl == L0.shape[0] and nv == V0.shape[0]
    big = ctx.build_cells(extra, p, cells)
    assert np.array_equal(big.origin, cells.origin) and np.array_equal(big.dims, cells.dims)
    with pytest.raises(tms.TmsError) as ei:
        ctx.graph_launch(cells)
    assert ei.value.code == tms.TMS_E_INVALID and "atom count" in str(ei.value)
    ctx.free_cells(cells)
