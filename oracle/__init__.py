"""FP64 CPU oracle for the Gaussian-surface partition/estimation method
(Liu, Chen & Lu, arXiv:1611.03474).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP implementation in ``paper_1611_03474_amd`` and never imports it.

The numerical work lives in ``tms_oracle.c`` (plain C, double precision,
OpenMP over independent cubes/points); this module compiles it with gcc when
needed and wraps it with ctypes.  Each wrapper cites the passage of the paper
that the C function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tms_oracle.c")
_LIB = os.path.join(_HERE, "libtms_oracle.so")

OR_MAXLEV = 8
REASON_UNIFORM, REASON_CONVERGED, REASON_HMIN = 0, 1, 2
CLS_OUTSIDE, CLS_SURFACE, CLS_INSIDE = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile ``tms_oracle.c`` into ``libtms_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("D", C.c_double), ("c", C.c_double), ("tau", C.c_double),
                ("h0", C.c_double), ("h_min", C.c_double), ("pad", C.c_double),
                ("eps_cut", C.c_double), ("uniform", C.c_int32),
                ("nthreads", C.c_int32), ("conf", C.c_int32), ("gl_nodes", C.c_int32),
                ("degree", C.c_int32), ("reexpand", C.c_int32)]


_I64A = C.c_int64 * OR_MAXLEV


class _Result(C.Structure):
    _fields_ = [("n_leaves", C.c_int64), ("ijk", C.POINTER(C.c_int32)),
                ("level", C.POINTER(C.c_uint8)), ("reason", C.POINTER(C.c_uint8)),
                ("mask", C.POINTER(C.c_uint8)), ("cls", C.POINTER(C.c_uint8)),
                ("corner_phi", C.POINTER(C.c_double)), ("n_vert", C.c_int64),
                ("vkey", C.POINTER(C.c_uint64)), ("vt", C.POINTER(C.c_double)),
                ("vxyz", C.POINTER(C.c_double)), ("origin", C.c_double * 3),
                ("dims", C.c_int64 * 3), ("K", C.c_int32), ("status", C.c_int32),
                ("rc2", C.c_double), ("n_est", _I64A), ("n_disc", _I64A),
                ("n_refine", _I64A), ("n_conv", _I64A), ("n_hmin", _I64A),
                ("n_pairs", C.c_int64), ("n_corners", C.c_int64),
                ("tie_cube", C.c_int64), ("tie_corner", C.c_int64),
                ("n_tie_list", C.c_int64), ("tie_list", C.c_int32 * (4 * 1024)),
                ("tie_corner_keys", C.c_uint64 * 1024)]


class _S2Pt(C.Structure):
    _fields_ = [("leaf", C.c_int32), ("kind", C.c_uint8), ("axis", C.c_uint8),
                ("root", C.c_uint8), ("pad", C.c_uint8), ("p", C.c_double * 3)]


class _S2Result(C.Structure):
    _fields_ = [("n", C.c_int64), ("pts", C.POINTER(_S2Pt)),
                ("leaf_margin", C.POINTER(C.c_double)), ("n_degenerate", C.c_int64),
                ("n_mismatch", C.c_int64)]


S2_DTYPE = np.dtype([("leaf", "<i4"), ("kind", "u1"), ("axis", "u1"), ("root", "u1"),
                     ("pad", "u1"), ("x", "<f8"), ("y", "<f8"), ("z", "<f8")])
S2_FOLD, S2_CRITICAL = 0, 1

_lib = None
_DP = C.POINTER(C.c_double)
_FUN1 = C.CFUNCTYPE(C.c_double, C.c_double, C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.or_gauss_legendre.argtypes = [C.c_int, _DP, _DP]
        L.or_project_fn.argtypes = [_FUN1, C.c_void_p, C.c_int, _DP]
        L.or_project.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, _DP]
        L.or_project_deg.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                     C.c_int, _DP]
        L.or_project_fn_deg.argtypes = [_FUN1, C.c_void_p, C.c_int, C.c_int, _DP]
        L.or_child_tensor.argtypes = [_DP, C.c_int, _DP]
        L.or_cutoff2.argtypes = [_DP, C.c_int64, C.c_double, C.c_double]
        L.or_cutoff2.restype = C.c_double
        L.or_phi.argtypes = [_DP, C.c_int64, C.c_double, C.c_double, _DP, C.c_int64, _DP, _DP,
                             C.c_int]
        L.or_phi_adjoint.argtypes = [_DP, C.c_int64, C.c_double, C.c_double, _DP, C.c_int64,
                                     _DP, _DP, C.c_int]
        L.or_cube_tensor.argtypes = [_DP, C.c_int64, C.c_double, C.c_double, C.c_int, _DP, _DP,
                                     _DP, C.POINTER(C.c_int64)]
        L.or_tensor_eval.argtypes = [_DP, C.c_double, C.c_double, C.c_double]
        L.or_tensor_eval.restype = C.c_double
        L.or_higher_mass.argtypes = [_DP]
        L.or_higher_mass.restype = C.c_double
        L.or_svd.argtypes = [C.c_int, C.c_int, _DP, _DP, _DP, _DP]
        L.or_cubic_range.argtypes = [_DP, _DP, _DP]
        L.or_bound.argtypes = [_DP, _DP]
        L.or_partition.argtypes = [_DP, C.c_int64, C.POINTER(Params)]
        L.or_partition.restype = C.POINTER(_Result)
        L.or_free.argtypes = [C.POINTER(_Result)]
        L.or_extract.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_uint8), _DP, C.c_int64,
                                 C.c_double, _DP, C.c_double, C.c_int, C.c_int]
        L.or_extract.restype = C.POINTER(_Result)
        _U8P = C.POINTER(C.c_uint8)
        L.or_stage2_cube.argtypes = [_DP, C.c_double, _DP, _U8P, _U8P, _U8P, _DP,
                                     C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.or_stage2_cube.restype = C.c_int
        L.or_stage2_points.argtypes = [C.POINTER(C.c_int32), _U8P, _U8P, _DP, C.c_int64,
                                       C.c_double, _DP, C.c_double, C.c_int]
        L.or_stage2_points.restype = C.POINTER(_S2Result)
        L.or_stage2_free.argtypes = [C.POINTER(_S2Result)]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _atoms(xyzr) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xyzr, dtype=np.float64).reshape(-1, 4))
    return a


# --------------------------------------------------------------------------
# Single-function wrappers (used by the pinning tests)
# --------------------------------------------------------------------------

def gauss_legendre(n: int):
    t = np.zeros(n)
    w = np.zeros(n)
    lib().or_gauss_legendre(n, _dp(t), _dp(w))
    return t, w


def project(D, lo, hi, xi, nodes=0, degree=3):
    """Degree-n Legendre projection (n = 1..3; the paper uses 3) with C0
    endpoint correction of the factor exp(-D (x - xi)^2) on [lo, hi]
    (Section 2.2.1, eqs. poly2_1, poly3, condition1, alpha); coefficients
    above n are zero."""
    a = np.zeros(4)
    lib().or_project_deg(float(D), float(lo), float(hi), float(xi), int(nodes), int(degree),
                         _dp(a))
    return a


def project_fn(f, nodes=0, degree=3):
    """The same projection applied to an arbitrary function f on [-1, 1]."""
    cb = _FUN1(lambda t, _ctx: float(f(t)))
    a = np.zeros(4)
    lib().or_project_fn_deg(cb, None, int(nodes), int(degree), _dp(a))
    return a


def child_tensor(A, octant):
    """The polynomial of tensor A written in the Legendre basis of child
    `octant` (bit 0: x, 1: y, 2: z; set = upper half) of its cube
    (Section 2.2.3, eq. childtensor)."""
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(64)
    out = np.zeros(64)
    lib().or_child_tensor(_dp(A), int(octant), _dp(out))
    return out.reshape(4, 4, 4)


def cutoff2(xyzr, D, eps_cut=1e-10):
    a = _atoms(xyzr)
    return lib().or_cutoff2(_dp(a), a.shape[0], float(D), float(eps_cut))


def phi(xyzr, D, pts, eps_cut=1e-10, grad=False, nthreads=0):
    """phi and its gradient at points (Section 1, eq. Gaussian1), truncated to
    the atoms within R_c of each point."""
    a = _atoms(xyzr)
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
    out = np.zeros(p.shape[0])
    g = np.zeros((p.shape[0], 3)) if grad else None
    lib().or_phi(_dp(a), a.shape[0], float(D), float(eps_cut), _dp(p), p.shape[0], _dp(out),
                 _dp(g) if grad else None, int(nthreads))
    return (out, g) if grad else out


def phi_adjoint(xyzr, D, pts, wbar, eps_cut=1e-10, nthreads=0):
    """sum_p wbar_p d phi(p)/d(x_i, y_i, z_i, r_i) for every atom i: the
    derivative of eq. Gaussian1 (Section 1), cut-off radius held fixed.
    Returns [n, 4]."""
    a = _atoms(xyzr)
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
    w = np.ascontiguousarray(np.asarray(wbar, dtype=np.float64).reshape(-1))
    assert w.shape[0] == p.shape[0]
    out = np.zeros((a.shape[0], 4))
    lib().or_phi_adjoint(_dp(a), a.shape[0], float(D), float(eps_cut), _dp(p), p.shape[0],
                         _dp(w), _dp(out), int(nthreads))
    return out


def cube_tensor(xyzr, D, lo, hi, eps_cut=1e-10, nodes=0):
    """Coefficient tensor A[j,k,l] of a cube (eqs. polynew, tensor1, tensor2)."""
    a = _atoms(xyzr)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    A = np.zeros(64)
    nn = C.c_int64(0)
    lib().or_cube_tensor(_dp(a), a.shape[0], float(D), float(eps_cut), int(nodes), _dp(lo),
                         _dp(hi), _dp(A), C.byref(nn))
    return A.reshape(4, 4, 4), nn.value


def tensor_eval(A, x, y, z):
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(64)
    return lib().or_tensor_eval(_dp(A), float(x), float(y), float(z))


def higher_mass(A):
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(64)
    return lib().or_higher_mass(_dp(A))


def svd(M):
    M = np.ascontiguousarray(M, dtype=np.float64)
    m, n = M.shape
    s = np.zeros(m)
    U = np.zeros((m, m))
    Vt = np.zeros((m, n))
    lib().or_svd(m, n, _dp(M), _dp(s), _dp(U), _dp(Vt))
    return U, s, Vt


def cubic_range(q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    lo = C.c_double(0)
    hi = C.c_double(0)
    lib().or_cubic_range(_dp(q), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def bound(A):
    """(L, U, rho, r, tie) of the nested-SVD bound (Section 2.2.2)."""
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(64)
    out = np.zeros(5)
    lib().or_bound(_dp(A), _dp(out))
    return out


# --------------------------------------------------------------------------
# Whole pass
# --------------------------------------------------------------------------

class Result:
    """Leaves, corner values, classes and edge vertices of one pass."""

    def __init__(self, r: _Result):
        n = r.n_leaves
        nv = r.n_vert
        self.status = r.status
        self.n_leaves = n
        self.ijk = np.ctypeslib.as_array(r.ijk, (max(n, 1), 3))[:n].copy()
        self.level = np.ctypeslib.as_array(r.level, (max(n, 1),))[:n].copy()
        self.reason = np.ctypeslib.as_array(r.reason, (max(n, 1),))[:n].copy()
        self.mask = np.ctypeslib.as_array(r.mask, (max(n, 1),))[:n].copy()
        self.cls = np.ctypeslib.as_array(r.cls, (max(n, 1),))[:n].copy()
        self.corner_phi = np.ctypeslib.as_array(r.corner_phi, (max(n, 1), 8))[:n].copy()
        self.n_vert = nv
        self.vkey = np.ctypeslib.as_array(r.vkey, (max(nv, 1),))[:nv].copy()
        self.vt = np.ctypeslib.as_array(r.vt, (max(nv, 1),))[:nv].copy()
        self.vxyz = np.ctypeslib.as_array(r.vxyz, (max(nv, 1), 3))[:nv].copy()
        self.origin = np.array(r.origin[:])
        self.dims = np.array(r.dims[:])
        self.K = r.K
        self.rc2 = r.rc2
        self.n_est = np.array(r.n_est[:])
        self.n_disc = np.array(r.n_disc[:])
        self.n_refine = np.array(r.n_refine[:])
        self.n_conv = np.array(r.n_conv[:])
        self.n_hmin = np.array(r.n_hmin[:])
        self.n_pairs = r.n_pairs
        self.n_corners = r.n_corners
        self.tie_cube = r.tie_cube
        self.tie_corner = r.tie_corner
        nt = min(r.n_tie_list, 1024)
        self.tie_cubes = np.array(r.tie_list[:4 * nt], dtype=np.int64).reshape(nt, 4)
        self.tie_corner_keys = np.array(r.tie_corner_keys[:min(r.tie_corner, 1024)],
                                        dtype=np.uint64)

    @property
    def cubes_estimated(self) -> int:
        return int(self.n_est.sum())


def partition(xyzr, D, c=1.0, tau=1e-3, h0=2.0, h_min=0.25, pad=3.0, eps_cut=1e-10,
              uniform=False, nthreads=0, conf=0, gl_nodes=0, degree=3,
              reexpand=False) -> Result:
    """Adaptive partition and estimation (Section 2.2, Steps 1-3) followed by
    leaf classification (eq. linear1) and edge intersections (eq. intersection).
    degree: the 1-D series degree n (1..3); reexpand: child tensors are the
    parent's polynomial in the child's basis (eq. childtensor) instead of new
    projections from the atoms."""
    a = _atoms(xyzr)
    P = Params(D=float(D), c=float(c), tau=float(tau), h0=float(h0), h_min=float(h_min),
               pad=float(pad), eps_cut=float(eps_cut), uniform=int(bool(uniform)),
               nthreads=int(nthreads), conf=int(conf), gl_nodes=int(gl_nodes),
               degree=int(degree), reexpand=int(bool(reexpand)))
    rp = lib().or_partition(_dp(a), a.shape[0], C.byref(P))
    try:
        res = Result(rp.contents)
    finally:
        lib().or_free(rp)
    if res.status != 0:
        raise ValueError("oracle rejected the input (status %d)" % res.status)
    res.h0 = float(h0)
    return res


def extract(ijk, level, corner_phi, c, origin, h0, K, conf=0) -> Result:
    """Edge intersection points (eq. intersection) of a caller's leaves with
    their corner values (masks and classes from eq. linear1); vertices in
    ascending key order."""
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    level = np.ascontiguousarray(level, dtype=np.uint8)
    cp = np.ascontiguousarray(corner_phi, dtype=np.float64).reshape(-1, 8)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    rp = lib().or_extract(ijk.ctypes.data_as(C.POINTER(C.c_int32)),
                          level.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(cp), ijk.shape[0],
                          float(c), _dp(o), float(h0), int(K), int(conf))
    try:
        res = Result(rp.contents)
    finally:
        lib().or_free(rp)
    res.h0 = float(h0)
    return res


# --------------------------------------------------------------------------
# Surface loss and its gradient (the adjoint workload)
# --------------------------------------------------------------------------

def corner_list(res: Result):
    """Unique leaf corners of a pass: finest-lattice keys X<<32 | Y<<16 | Z
    (ascending), their points and phi values.  Each corner value was
    evaluated once per unique point by the oracle, so any leaf that holds the
    corner gives the same value."""
    sh = (res.K - res.level.astype(np.int64))[:, None]
    keys, vals = [], []
    for v in range(8):
        d = np.array([v & 1, (v >> 1) & 1, (v >> 2) & 1], dtype=np.int64)
        X = (res.ijk.astype(np.int64) + d[None, :]) << sh
        keys.append((X[:, 0] << 32) | (X[:, 1] << 16) | X[:, 2])
        vals.append(res.corner_phi[:, v])
    keys = np.concatenate(keys)
    vals = np.concatenate(vals)
    uk, first = np.unique(keys, return_index=True)
    hmin = 2.0 ** -res.K * res.h0
    X = np.stack([(uk >> 32) & 0xFFFF, (uk >> 16) & 0xFFFF, uk & 0xFFFF], 1).astype(np.float64)
    pts = res.origin[None, :] + X * hmin
    return uk, pts, vals[first]


def vertex_edges(res: Result):
    """For every vertex: the keys of the lower and upper end of its edge and
    the edge length h (eq. intersection)."""
    k = res.vkey.astype(np.uint64)
    level = ((k >> np.uint64(50)) & np.uint64(7)).astype(np.int64)
    axis = ((k >> np.uint64(48)) & np.uint64(3)).astype(np.int64)
    X = np.stack([(k >> np.uint64(32)) & np.uint64(0xFFFF), (k >> np.uint64(16)) & np.uint64(0xFFFF),
                  k & np.uint64(0xFFFF)], 1).astype(np.int64)
    k0 = (X[:, 0] << 32) | (X[:, 1] << 16) | X[:, 2]
    step = np.int64(1) << (res.K - level)
    X1 = X.copy()
    X1[np.arange(len(X)), axis] += step
    k1 = (X1[:, 0] << 32) | (X1[:, 1] << 16) | X1[:, 2]
    h = res.h0 * 2.0 ** (-level.astype(np.float64))
    return k0, k1, h


def surface_loss(phi_c, c, t, h):
    """Loss of the adjoint workload: sum over unique leaf corners of
    (phi - c)^2 plus the squared distance of every edge point from its edge
    midpoint, ((t - 1/2) h)^2."""
    return float(np.sum((phi_c - c) ** 2) + np.sum(((t - 0.5) * h) ** 2))


def surface_loss_grad(xyzr, D, c, res: Result, eps_cut=1e-10, nthreads=0):
    """Loss and its gradient with respect to every atom's (x, y, z, r), with
    the discrete structure of the pass (leaves, masks, edges) held fixed.

    Chain: dL/dphi_p = 2 (phi_p - c) at every corner; every edge point adds
    dL/dt = 2 (t - 1/2) h^2 times dt/dphi0 = (t - 1)/(phi1 - phi0) at its
    lower end and dt/dphi1 = -t/(phi1 - phi0) at its upper end, since
    t = (c - phi0)/(phi1 - phi0) (eq. intersection); then phi_adjoint."""
    keys, pts, ph = corner_list(res)
    k0, k1, h = vertex_edges(res)
    i0 = np.searchsorted(keys, k0)
    i1 = np.searchsorted(keys, k1)
    assert np.all(keys[i0] == k0) and np.all(keys[i1] == k1)
    f0, f1 = ph[i0], ph[i1]
    t = (c - f0) / (f1 - f0)
    wbar = 2.0 * (ph - c)
    dldt = 2.0 * (t - 0.5) * h * h
    np.add.at(wbar, i0, dldt * (t - 1.0) / (f1 - f0))
    np.add.at(wbar, i1, dldt * (-t) / (f1 - f0))
    grad = phi_adjoint(xyzr, D, pts, wbar, eps_cut=eps_cut, nthreads=nthreads)
    return surface_loss(ph, c, t, h), grad, dict(keys=keys, pts=pts, phi=ph, wbar=wbar, t=t,
                                                 k0=k0, k1=k1, h=h)


# --------------------------------------------------------------------------
# Stage 2 points of the trilinear surface (Section 2.3)
# --------------------------------------------------------------------------

def stage2_cube(f, c):
    """Fold segments (eqs. curve, fold1) and critical points (eq. critical) of
    g = c on one cube [-1,1]^3 whose trilinear interpolant (eq. linear1) has
    corner values f[v], v = dx + 2 dy + 4 dz.  Returns (records in local
    coordinates as a dict of arrays, margin, degenerate count, count of fold
    segments whose two face extreme points disagree)."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(8)
    loc = np.zeros((12, 3))
    kind = np.zeros(12, dtype=np.uint8)
    axis = np.zeros(12, dtype=np.uint8)
    root = np.zeros(12, dtype=np.uint8)
    margin = C.c_double(0)
    nd = C.c_int(0)
    mis = C.c_int(0)
    U8 = C.POINTER(C.c_uint8)
    n = lib().or_stage2_cube(_dp(f), float(c), _dp(loc), kind.ctypes.data_as(U8),
                             axis.ctypes.data_as(U8), root.ctypes.data_as(U8), C.byref(margin),
                             C.byref(nd), C.byref(mis))
    return (dict(loc=loc[:n].copy(), kind=kind[:n].copy(), axis=axis[:n].copy(),
                 root=root[:n].copy()), margin.value, nd.value, mis.value)


class Stage2:
    """Stage 2 points of every SURFACE leaf of a pass: ``pts`` (S2_DTYPE,
    world coordinates, by leaf), ``leaf_margin`` per leaf, counts of
    degenerate configurations and of face mismatches."""

    def __init__(self, r):
        n = r.n
        raw = np.ctypeslib.as_array(C.cast(r.pts, C.POINTER(C.c_uint8)), (max(n, 1) * 32,))
        self.pts = np.frombuffer(raw[:n * 32].tobytes(), dtype=S2_DTYPE).copy()
        self.n_degenerate = r.n_degenerate
        self.n_mismatch = r.n_mismatch


def stage2_points(ijk, level, cls, corner_phi, c, origin, h0, nthreads=0):
    """Stage 2 points (Section 2.3: eqs. curve, fold1, critical) of the
    SURFACE leaves of a leaf list with its corner values."""
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    level = np.ascontiguousarray(level, dtype=np.uint8)
    cls = np.ascontiguousarray(cls, dtype=np.uint8)
    cp = np.ascontiguousarray(corner_phi, dtype=np.float64).reshape(-1, 8)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    n = ijk.shape[0]
    assert level.shape[0] == n and cls.shape[0] == n and cp.shape[0] == n
    U8 = C.POINTER(C.c_uint8)
    rp = lib().or_stage2_points(ijk.ctypes.data_as(C.POINTER(C.c_int32)), level.ctypes.data_as(U8),
                                cls.ctypes.data_as(U8), _dp(cp), n, float(c), _dp(o), float(h0),
                                int(nthreads))
    try:
        out = Stage2(rp.contents)
        out.leaf_margin = np.ctypeslib.as_array(rp.contents.leaf_margin, (max(n, 1),))[:n].copy()
    finally:
        lib().or_stage2_free(rp)
    return out


def stage2_of(res: Result, c, nthreads=0):
    """Stage 2 points of a partition result."""
    return stage2_points(res.ijk, res.level, res.cls, res.corner_phi, c, res.origin, res.h0,
                         nthreads=nthreads)
