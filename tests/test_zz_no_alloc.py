"""The allocation-free phi entry point (tms_eval_phi_noalloc) against
tms_eval_phi, through the C ABI: same phi, gradient and guard count, bit for
bit, on two calls in a row (the second with fewer points, so that the static
scratch still holds the first call's guard flags and list), in both
precisions; sizes beyond its maximum are refused."""
import numpy as np
import pytest

from paper_1611_03474_amd import synth, tms

pytestmark = pytest.mark.gpu

MAX_POINTS = 1 << 22


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = tms.Context(0)
    yield c
    c.close()


def _points(atoms, m, seed):
    rng = np.random.default_rng(seed)
    lo, hi = atoms[:, :3].min(0) - 6, atoms[:, :3].max(0) + 6
    pts = rng.uniform(lo, hi, size=(m, 3))
    k = m // 2
    pts[:k] = atoms[rng.integers(0, len(atoms), k), :3] + rng.normal(scale=1.2, size=(k, 3))
    return pts


def _isolated_atoms():
    # 64 atoms 20 A apart (beyond twice the cut-off radius at D = 0.9), so
    # that on the sphere |p - x_i| = r_i phi is 1 = c up to rounding
    g = np.stack(np.meshgrid(*[np.arange(4) * 20.0] * 3, indexing="ij"), -1).reshape(-1, 3)
    return np.concatenate([g, np.full((len(g), 1), 1.7)], axis=1)


def _sphere_points(atoms, m, seed):
    rng = np.random.default_rng(seed)
    pts = _points(atoms, m, seed)
    k = (2 * m) // 5
    d = rng.normal(size=(k, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    i = rng.integers(0, len(atoms), k)
    pts[m - k:] = atoms[i, :3] + d * atoms[i, 3:4]
    return pts


@pytest.mark.parametrize("prec", [tms.PREC_FP32_GUARD, tms.PREC_FP64], ids=["fp32g", "fp64"])
def test_noalloc_equals_eval_phi(ctx, prec):
    import torch
    atoms = _isolated_atoms()
    cells = ctx.build_cells(atoms, tms.make_params(D=0.9, precision=prec))
    for m, seed, with_grad in [(600_000, 1, True), (70_001, 2, True), (5_003, 3, False)]:
        pts = torch.as_tensor(_sphere_points(atoms, m, seed), device=ctx.device).contiguous()
        phi_a, grad_a, ng_a = ctx.eval_phi(cells, pts, grad=with_grad)
        phi_b = torch.full((m,), float("nan"), dtype=torch.float64, device=ctx.device)
        grad_b = (torch.full((m, 3), float("nan"), dtype=torch.float64, device=ctx.device)
                  if with_grad else None)
        ng_b = ctx.eval_phi_noalloc(cells, pts, phi_b, grad_b)
        print("m=%d guard points %d / %d" % (m, ng_a, ng_b))
        assert not torch.isnan(phi_b).any()
        assert ng_a == ng_b
        if prec == tms.PREC_FP32_GUARD:
            assert ng_a > 0
        assert torch.equal(phi_a, phi_b)
        if with_grad:
            assert torch.equal(grad_a, grad_b)
    ctx.free_cells(cells)


def test_noalloc_refuses_too_many_points(ctx):
    import torch
    atoms = synth.globule(200, 1001)
    cells = ctx.build_cells(atoms, tms.make_params(D=0.9, precision=tms.PREC_FP32_GUARD))
    m = MAX_POINTS + 1
    pts = torch.zeros((m, 3), dtype=torch.float64, device=ctx.device)
    phi = torch.empty(m, dtype=torch.float64, device=ctx.device)
    with pytest.raises(tms.TmsError) as ei:
        ctx.eval_phi_noalloc(cells, pts, phi)
    assert ei.value.code == tms.TMS_E_INVALID
    assert "maximum" in str(ei.value)
    # the largest allowed size runs
    pts = torch.as_tensor(_points(atoms, MAX_POINTS, 4), device=ctx.device).contiguous()
    phi_a, _, ng_a = ctx.eval_phi(cells, pts)
    phi_b = torch.empty(MAX_POINTS, dtype=torch.float64, device=ctx.device)
    assert ctx.eval_phi_noalloc(cells, pts, phi_b[:MAX_POINTS]) == ng_a
    assert torch.equal(phi_a, phi_b)
    ctx.free_cells(cells)
