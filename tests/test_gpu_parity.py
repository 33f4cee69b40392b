"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars:
  * discrete results -- leaf list, levels, reasons, masks, classes, vertex
    keys -- bit-exact, in order;
  * phi, corner values, vertex t: FP64 path 1e-12 relative; FP32+guard path
    1e-5 relative (phi) and 1e-5 absolute in t;
  * grad phi: 1e-5 of the gradient scale 2 D R_c phi (FP32), 1e-12 (FP64).
Cubes that the oracle reports as near ties (a decision margin below 1e-9
relative, where both FP64 codes may legitimately differ) are excluded with
their whole subtree; the count is printed.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
from paper_1611_03474_amd import synth, tms
from parity_util import compare as _compare, phi_tol as _phi_tol, run_gpu as _run_gpu

pytestmark = pytest.mark.gpu

PRECS = [tms.PREC_FP64, tms.PREC_FP32_GUARD]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = tms.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def g200():
    return synth.globule(200, 1001)


@pytest.fixture(scope="module")
def g1000():
    return synth.globule(1000, 1006)


@pytest.mark.parametrize("prec", PRECS)
def test_phi_and_grad_parity(ctx, g200, prec):
    D = 0.9
    rng = np.random.default_rng(17)
    lo, hi = g200[:, :3].min(0) - 8, g200[:, :3].max(0) + 8
    pts = rng.uniform(lo, hi, size=(20000, 3))
    pts[:2000] = g200[rng.integers(0, len(g200), 2000), :3] + rng.normal(scale=1.0, size=(2000, 3))
    p = tms.make_params(D=D, precision=prec)
    cells = ctx.build_cells(g200, p)
    phi, grad, ng = ctx.eval_phi(cells, pts, grad=True)
    phi, grad = phi.cpu().numpy(), grad.cpu().numpy()
    rphi, rgrad = oracle.phi(g200, D, pts, grad=True)
    tol = _phi_tol(prec)
    rel = np.abs(phi - rphi) / np.maximum(rphi, 1e-300)
    print("max relative phi error %.3e" % rel.max())
    assert np.all(np.abs(phi - rphi) <= tol * rphi + 1e-300)
    if prec == tms.PREC_FP32_GUARD:
        # single-precision exponentials: relative error within the design
        # bound kFastExpErr = 1.5e-7 of every term (plus double rounding)
        assert rel.max() <= 1.5e-7 + 1e-13
    scale = 2 * D * math.sqrt(cells.rc2) * rphi
    assert np.all(np.abs(grad - rgrad) <= tol * scale[:, None] + 1e-300)
    assert np.array_equal(phi >= 1.0, rphi >= 1.0)
    print("guard points", ng)
    ctx.free_cells(cells)


@pytest.mark.parametrize("prec", PRECS)
def test_tensor_parity(ctx, g200, prec):
    D = 0.9
    p = tms.make_params(D=D, precision=prec)
    cells = ctx.build_cells(g200, p)
    rng = np.random.default_rng(5)
    cubes = []
    for lev in range(4):
        n = cells.dims << lev
        for _ in range(40):
            # cubes near atoms, plus a few empty ones
            a = g200[rng.integers(0, len(g200)), :3] + rng.normal(scale=2.0, size=3)
            i = np.floor((a - cells.origin) / (2.0 / 2 ** lev)).astype(int)
            i = np.clip(i, 0, n - 1)
            cubes.append([lev, *i])
    cubes = np.array(cubes, dtype=np.int32)
    A, EA = ctx.debug_tensor(cells, cubes, precision=prec, with_scale=True)
    A, EA = A.cpu().numpy(), EA.cpu().numpy()
    A64 = ctx.debug_tensor(cells, cubes, precision=tms.PREC_FP64).cpu().numpy()
    worst = 0.0
    for row, (lev, ix, iy, iz) in enumerate(cubes):
        h = 2.0 / 2 ** lev
        lo = cells.origin + np.array([ix, iy, iz]) * h
        R, _ = oracle.cube_tensor(g200, D, lo, lo + h)
        R = R.reshape(64)
        scale = max(np.abs(R).sum(), 1e-300)
        if prec == tms.PREC_FP64:
            assert EA[row] == 0.0
            assert np.abs(A[row] - R).sum() <= 1e-12 * scale
        else:
            # the kernel's own a-posteriori l1 bound covers the difference
            # to the exact-exponential tensor
            err = np.abs(A[row] - A64[row]).sum()
            assert err <= EA[row] + 1e-13 * scale
            assert np.abs(A[row] - R).sum() <= EA[row] + 1e-12 * scale
            if EA[row] > 0:
                worst = max(worst, err / EA[row])
    print("max actual/bound tensor error ratio %.3f" % worst)
    ctx.free_cells(cells)


def test_fast_exp_error_bound(ctx):
    # the guard band of the FP32+guard path assumes |exp_fast(x)/exp(x) - 1|
    # <= 1.5e-7 for every x <= 0; sweep the range the kernels use densely
    x = -np.concatenate([np.linspace(0.0, 60.0, 4_000_001),
                         np.random.default_rng(3).uniform(0.0, 60.0, 2_000_000)])
    y = ctx.debug_fast_exp(x).cpu().numpy()
    rel = np.abs(y / np.exp(x) - 1.0)
    print("fast exp max relative error %.3e" % rel.max())
    assert rel.max() <= 1.5e-7


def test_bound_parity(ctx, g200):
    D = 0.9
    rng = np.random.default_rng(6)
    As, refs = [], []
    for lev in range(4):
        h = 2.0 / 2 ** lev
        for _ in range(60):
            a = g200[rng.integers(0, len(g200)), :3] + rng.normal(scale=2.5, size=3)
            lo = np.floor(a / h) * h
            A, _ = oracle.cube_tensor(g200, D, lo, lo + h)
            As.append(A.reshape(64))
            refs.append(oracle.bound(A))
    # synthetic tensors: trilinear, rank one, zero
    A = np.zeros((4, 4, 4))
    A[:2, :2, :2] = rng.normal(size=(2, 2, 2))
    As.append(A.reshape(64))
    refs.append(oracle.bound(A))
    As.append(np.zeros(64))
    refs.append(oracle.bound(np.zeros(64)))
    out = ctx.debug_bound(np.array(As)).cpu().numpy()
    assert out.shape[1] == 6
    refs = np.array(refs)
    for k in range(len(As)):
        scale = max(np.abs(As[k]).sum(), 1e-300)
        if refs[k, 4] < 1e-6:
            continue  # near-degenerate singular values: bound not unique
        assert out[k, 3] == refs[k, 3]
        assert abs(out[k, 0] - refs[k, 0]) <= 1e-10 * scale
        assert abs(out[k, 1] - refs[k, 1]) <= 1e-10 * scale


@pytest.mark.parametrize("prec", PRECS)
def test_uniform_grid_parity(ctx, g200, prec):
    # the plain method: every cube of a uniform h = 0.5 grid
    _compare(ctx, g200, prec, D=0.9, mode=tms.MODE_UNIFORM, h0=0.5, h_min=0.5)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("tau", [1e-3, 0.1, 0.3])
def test_adaptive_parity_small(ctx, g200, prec, tau):
    _compare(ctx, g200, prec, D=0.9, tau=tau)


@pytest.mark.parametrize("prec", PRECS, ids=["fp64", "fp32g"])
@pytest.mark.parametrize("h0,h_min,tau", [(1.5, 0.1875, 0.1), (2.0, 0.125, 0.1),
                                          (2.0, 0.125, 1e-3)],
                         ids=["h0_1.5", "K4_tau0.1", "K4_tau1e-3"])
def test_adaptive_parity_lattices(ctx, g200, prec, h0, h_min, tau):
    # h0 not a power of two (cell and table coordinates by division rather
    # than exact scaling) and a fourth level (per-thread estimate from a wider
    # projection table)
    _compare(ctx, g200, prec, D=0.9, tau=tau, h0=h0, h_min=h_min)


@pytest.mark.parametrize("D", [0.5, 0.9, 1.5])
def test_adaptive_parity_1000(ctx, g1000, D):
    _compare(ctx, g1000, tms.PREC_FP32_GUARD, D=D, tau=1e-3)


def test_fp32_guard_equals_fp64(ctx, g1000):
    a = _run_gpu(ctx, g1000, tms.PREC_FP64, D=0.9, tau=0.1)
    b = _run_gpu(ctx, g1000, tms.PREC_FP32_GUARD, D=0.9, tau=0.1)
    assert np.array_equal(a["leaves"], b["leaves"])
    assert np.array_equal(a["verts"]["edge_key"], b["verts"]["edge_key"])
    assert a["stats"]["n_est"] == b["stats"]["n_est"]


def test_deterministic(ctx, g1000):
    a = _run_gpu(ctx, g1000, tms.PREC_FP32_GUARD, D=0.9)
    b = _run_gpu(ctx, g1000, tms.PREC_FP32_GUARD, D=0.9)
    assert a["leaves"].tobytes() == b["leaves"].tobytes()
    assert a["cphi"].tobytes() == b["cphi"].tobytes()
    assert a["verts"].tobytes() == b["verts"].tobytes()


def test_empty_atom_set(ctx):
    got = _run_gpu(ctx, np.zeros((0, 4)), tms.PREC_FP64)
    assert len(got["leaves"]) == 0 and len(got["verts"]) == 0


@pytest.mark.parametrize("prec", PRECS)
def test_single_atom(ctx, prec):
    atom = np.array([[0.3, -0.2, 0.45, 1.7]])
    _compare(ctx, atom, prec, D=0.9, tau=1e-3)
    _compare(ctx, atom, prec, D=0.9, mode=tms.MODE_UNIFORM, h0=0.25, h_min=0.25)


def test_capacity_protocol(ctx, g200):
    p = tms.make_params(D=0.9)
    cells = ctx.build_cells(g200, p)
    leaves, cphi, st = ctx.partition_estimate(cells)
    n = len(leaves)
    small = ctx.partition_estimate(cells, cap=10)[0]  # retries via tms_get_leaves
    assert len(small) == n
    import torch
    buf = torch.empty((5, 20), dtype=torch.uint8, device=ctx.device)
    cb = torch.empty((5, 8), dtype=torch.float64, device=ctx.device)
    with pytest.raises(tms.TmsError) as ei:
        ctx.partition_into(cells, buf, cb)
    assert ei.value.code == tms.TMS_E_CAPACITY and ei.value.required == n
    v = ctx.extract(cells, leaves, cphi, cap=3)
    assert len(v) == len(ctx.extract(cells, leaves, cphi))
    ctx.free_cells(cells)


def test_direct_delivery(ctx, g200):
    # buffers that hold the result receive it directly (bit-identical to the
    # kept copy); ctx then keeps none, and the get calls say so
    import torch
    p = tms.make_params(D=0.9, tau=0.1, precision=tms.PREC_FP32_GUARD)
    cells = ctx.build_cells(g200, p)
    leaves, cphi, _ = ctx.partition_estimate(cells)        # kept, then copied
    verts = ctx.extract(cells, leaves, cphi)
    lb = torch.zeros((len(leaves) + 7, 20), dtype=torch.uint8, device=ctx.device)
    cb = torch.zeros((len(leaves) + 7, 8), dtype=torch.float64, device=ctx.device)
    nl, _ = ctx.partition_into(cells, lb, cb)                # written in place
    assert nl == len(leaves)
    assert torch.equal(lb[:nl], leaves) and torch.equal(cb[:nl], cphi)
    n = ctypes.c_int64()
    with pytest.raises(tms.TmsError) as ei:
        ctx._check(ctx.lib.tms_get_leaves(ctx.h, tms._VP(lb.data_ptr()), None, lb.shape[0],
                                          ctypes.byref(n)))
    assert ei.value.code == tms.TMS_E_INVALID
    ctx._check(ctx.lib.tms_get_leaves(ctx.h, None, None, 0, ctypes.byref(n)))
    assert n.value == nl                                     # the count stays
    vb = torch.zeros((len(verts) + 7, 40), dtype=torch.uint8, device=ctx.device)
    nv = ctx.extract_into(cells, lb, nl, cb, vb)
    assert nv == len(verts) and torch.equal(vb[:nv], verts)
    with pytest.raises(tms.TmsError) as ei:
        ctx.get_vertices()
    assert ei.value.code == tms.TMS_E_INVALID
    # a count-only pass keeps its result again
    leaves2, cphi2, _ = ctx.partition_estimate(cells)
    assert torch.equal(leaves2, leaves) and torch.equal(cphi2, cphi)
    ctx.free_cells(cells)


def test_invalid_input_rejected(ctx):
    p = tms.make_params()
    a = np.array([[0.0, 0.0, 0.0, 1.7], [1.0, np.nan, 0.0, 1.5]])
    with pytest.raises(tms.TmsError) as ei:
        ctx.build_cells(a, p)
    assert ei.value.code == tms.TMS_E_INVALID
    a = np.array([[0.0, 0.0, 0.0, -1.0]])
    with pytest.raises(tms.TmsError):
        ctx.build_cells(a, p)


def test_extract_recomputes_corners(ctx, g200):
    p = tms.make_params(D=0.9)
    cells = ctx.build_cells(g200, p)
    leaves, cphi, _ = ctx.partition_estimate(cells)
    a = tms.vertices_to_numpy(ctx.extract(cells, leaves, cphi))
    b = tms.vertices_to_numpy(ctx.extract(cells, leaves, None))
    assert a.tobytes() == b.tobytes()
    ctx.free_cells(cells)


def test_phi_pair_count(ctx, g200):
    # the pairs phi sums: (point, atom) with |p - x_i|^2 <= R_c^2, counted by
    # brute force over every pair
    rng = np.random.default_rng(23)
    pts = g200[rng.integers(0, len(g200), 3000), :3] + rng.normal(scale=3.0, size=(3000, 3))
    p = tms.make_params(D=0.9)
    cells = ctx.build_cells(g200, p)
    rc2 = oracle.cutoff2(g200, 0.9)
    d2 = ((pts[:, None, :] - g200[None, :, :3]) ** 2).sum(-1)
    assert ctx.debug_phi_pairs(cells, pts) == int((d2 <= rc2).sum())
    ctx.free_cells(cells)


def test_extract_exact_on_trilinear_field(ctx):
    # corner values of a trilinear field (dyadic coefficients: exact inputs)
    # on leaves of two levels, fed to tms_extract_cube_vertices and to the
    # oracle's edge step: the same edges, t equal to the last bits
    import torch
    from test_oracle_extract import leaves_and_values
    c = 0.883
    atoms = np.array([[-5.0, -3.0, -1.0, 1.5], [1.0, 3.0, 5.0, 1.5]])
    cells = ctx.build_cells(atoms, tms.make_params(D=0.9, c=c))
    origin, h0, K = np.array([-8.0, -6.0, -4.0]), 2.0, 3
    assert np.array_equal(cells.origin, origin) and cells.K == K  # reading R9
    coef = [3 / 4, 1 / 8, -1 / 16, 1 / 32, 3 / 64, -1 / 64, 1 / 128, 1 / 256]
    _, ijk, level, cp = leaves_and_values(coef, origin, h0, K)
    ref = oracle.extract(ijk, level, cp, c, origin, h0, K, conf=0)
    L = np.zeros(len(ijk), dtype=tms.LEAF_DTYPE)
    L["ix"], L["iy"], L["iz"], L["level"] = ijk[:, 0], ijk[:, 1], ijk[:, 2], level
    L["mask"], L["cls"] = ref.mask, ref.cls
    lt = torch.as_tensor(np.frombuffer(L.tobytes(), dtype=np.uint8).reshape(-1, 20)).to(ctx.device)
    V = tms.vertices_to_numpy(ctx.extract(cells, lt, torch.as_tensor(cp).to(ctx.device)))
    assert ref.n_vert > 100
    assert np.array_equal(V["edge_key"], ref.vkey)
    ulp = np.spacing(np.maximum(np.abs(ref.vt), 1e-300))
    assert np.all(np.abs(V["t"] - ref.vt) <= ulp)
    assert np.allclose(np.stack([V["x"], V["y"], V["z"]], 1), ref.vxyz, rtol=0, atol=1e-14)
    ctx.free_cells(cells)
