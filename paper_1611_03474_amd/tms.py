"""Thin ctypes binding over ``libtms.so`` (the C ABI of ``include/tms.h``).

Only argument marshalling lives here: every step of the computation runs in
the library's HIP kernels.  PyTorch supplies device memory and the stream.
Importing this module does not touch the GPU; the first ``Context`` loads the
library and raises ``RuntimeError`` if it is missing (no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtms.so")

TMS_OK, TMS_E_INVALID, TMS_E_CAPACITY, TMS_E_DEVICE, TMS_E_OOM = 0, -1, -2, -3, -4
PREC_FP64, PREC_FP32_GUARD = 0, 1
MODE_ADAPTIVE, MODE_UNIFORM = 0, 1
CHILD_PROJECT, CHILD_REEXPAND = 0, 1
REASON_UNIFORM, REASON_CONVERGED, REASON_HMIN, REASON_CLOSED, REASON_SPLIT = 0, 1, 2, 3, 4
MESH_CLOSE = 1
CLS_OUTSIDE, CLS_SURFACE, CLS_INSIDE = 0, 1, 2
MAX_LEVELS = 8

LEAF_DTYPE = np.dtype([("ix", "<i4"), ("iy", "<i4"), ("iz", "<i4"), ("conf", "<i4"),
                       ("level", "u1"), ("reason", "u1"), ("mask", "u1"), ("cls", "u1")])
VERTEX_DTYPE = np.dtype([("edge_key", "<u8"), ("t", "<f8"), ("x", "<f8"), ("y", "<f8"),
                         ("z", "<f8")])
assert LEAF_DTYPE.itemsize == 20 and VERTEX_DTYPE.itemsize == 40


T_SLOTS = ["build", "estimate", "decide", "guard", "compact", "corner", "phi", "extract",
           "tiled", "backward", "table", "grouped", "stage2"]


class Timing(C.Structure):
    _fields_ = [("ms", C.c_double * len(T_SLOTS)), ("launches", C.c_int64 * len(T_SLOTS))]

    def as_dict(self) -> dict:
        return {k: {"ms": self.ms[i], "launches": int(self.launches[i])}
                for i, k in enumerate(T_SLOTS)}


class MeshReport(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n_vertices", "n_triangles", "n_loops", "n_fallback", "open_faces", "added_cubes",
        "boundary_edges",
        "nonmanifold_edges", "misoriented_edges", "nonmanifold_vertices", "intersecting_pairs",
        "components", "euler", "unused_vertices")] + [
        ("area", C.c_double), ("volume", C.c_double), ("density", C.c_double),
        ("min_angle", C.c_double), ("small_angles", C.c_int64), ("zero_area", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Mesh:
    """A host mesh of tms_mesh_build (Section 2.3): .xyz [nv, 3], .tri [nt, 3],
    .tri_leaf [nt] (numpy), counts in .info; .added (LEAF_DTYPE) and
    .added_phi [k, 8]: the cubes added across open faces."""

    def __init__(self, lib, handle):
        self.lib, self.h = lib, handle
        i64 = C.c_int64
        v = [i64() for _ in range(5)]
        lib.tms_mesh_info(handle, *[C.byref(x) for x in v])
        nv, nt = v[0].value, v[1].value
        self.info = dict(n_vertices=nv, n_triangles=nt, n_loops=v[2].value,
                         n_fallback=v[3].value, open_faces=v[4].value)
        self.xyz = np.zeros((nv, 3))
        self.tri = np.zeros((nt, 3), dtype=np.int32)
        self.tri_leaf = np.zeros(nt, dtype=np.int32)
        lib.tms_mesh_get(handle, self.xyz.ctypes.data_as(_VP), self.tri.ctypes.data_as(_VP),
                         self.tri_leaf.ctypes.data_as(_VP))
        k = i64()
        lib.tms_mesh_added(handle, None, None, 0, C.byref(k))
        self.added = np.zeros(k.value, dtype=LEAF_DTYPE)
        self.added_phi = np.zeros((k.value, 8))
        rc = lib.tms_mesh_added(handle, self.added.ctypes.data_as(_VP),
                                self.added_phi.ctypes.data_as(_VP), k.value, C.byref(k))
        if rc != TMS_OK:
            raise TmsError(rc, "tms_mesh_added")
        self.info["added_cubes"] = len(self.added)

    def check(self, intersections: bool = True) -> dict:
        r = MeshReport()
        rc = self.lib.tms_mesh_check(self.h, int(bool(intersections)), C.byref(r))
        if rc != TMS_OK:
            raise TmsError(rc, "tms_mesh_check")
        return r.as_dict()

    def write_off(self, path: str):
        rc = self.lib.tms_mesh_write_off(self.h, str(path).encode())
        if rc != TMS_OK:
            raise TmsError(rc, "cannot write %s" % path)

    def free(self):
        if self.h:
            self.lib.tms_mesh_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def mesh_build_host(leaves: np.ndarray, corner_phi: np.ndarray, verts: np.ndarray, c: float,
                    K: int, h0: float) -> Mesh:
    """tms_mesh_build_host on host arrays: leaves (LEAF_DTYPE), corner values
    [n, 8], vertices (VERTEX_DTYPE, ascending keys)."""
    L = load_library()
    lv = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
    cp = np.ascontiguousarray(corner_phi, dtype=np.float64).reshape(-1, 8)
    vv = np.ascontiguousarray(verts, dtype=VERTEX_DTYPE)
    assert len(lv) == len(cp)
    h = _VP()
    msg = C.create_string_buffer(256)
    rc = L.tms_mesh_build_host(lv.ctypes.data_as(_VP), len(lv), cp.ctypes.data_as(_VP),
                               vv.ctypes.data_as(_VP), len(vv), float(c), int(K), float(h0),
                               C.byref(h),
                               msg, 256)
    if rc != TMS_OK:
        raise TmsError(rc, msg.value.decode())
    return Mesh(L, h)


class Tuning(C.Structure):
    _fields_ = [("slice_cubes", C.c_int64), ("tiled_min_level", C.c_int32),
                ("tile_atoms", C.c_int32), ("proj_table", C.c_int32),
                ("tiled_persistent", C.c_int32), ("tiled_half", C.c_int32),
                ("corner_groups", C.c_int32), ("corner_reach", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class TmsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("tms error %d: %s" % (code, msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [("D", C.c_double), ("c", C.c_double), ("tau", C.c_double), ("h0", C.c_double),
                ("h_min", C.c_double), ("pad", C.c_double), ("eps_cut", C.c_double),
                ("precision", C.c_int32), ("mode", C.c_int32), ("degree", C.c_int32),
                ("child_tensor", C.c_int32)]


_I64L = C.c_int64 * MAX_LEVELS


class Stats(C.Structure):
    _fields_ = [("n_est", _I64L), ("n_disc", _I64L), ("n_refine", _I64L), ("n_conv", _I64L),
                ("n_hmin", _I64L), ("n_leaves", C.c_int64), ("n_surface", C.c_int64),
                ("n_corners", C.c_int64), ("n_bound", C.c_int64), ("guard_cubes", C.c_int64),
                ("guard_points", C.c_int64), ("n_pairs", C.c_int64), ("n_pairs_lvl", _I64L)]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, C.Array) else int(v)
        d["cubes_estimated"] = int(sum(self.n_est))
        return d


_lib = None
_VP = C.c_void_p


def load_library(path: str = LIB_PATH):
    """Load libtms.so; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libtms.so not found at %s: build it with "
                           "`python -m paper_1611_03474_amd.build`" % path)
    L = C.CDLL(path)
    i32, i64, dp = C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.tms_create.argtypes = [C.POINTER(_VP), i32, _VP]
    L.tms_destroy.argtypes = [_VP]
    L.tms_last_error.argtypes = [_VP]
    L.tms_last_error.restype = C.c_char_p
    L.tms_check_params.argtypes = [C.POINTER(Params), C.c_char_p, i64]
    L.tms_check_atoms_host.argtypes = [dp, i64, C.POINTER(Params), C.c_char_p, i64]
    L.tms_build_cells.argtypes = [_VP, _VP, i64, C.POINTER(Params), C.POINTER(_VP)]
    L.tms_cells_info.argtypes = [_VP, dp, C.POINTER(i64), C.POINTER(i32), dp, C.POINTER(i64)]
    L.tms_free_cells.argtypes = [_VP, _VP]
    L.tms_eval_phi.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, C.POINTER(i64)]
    L.tms_eval_phi_noalloc.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, C.POINTER(i64)]
    L.tms_stage2_points.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, i64, C.POINTER(i64),
                                    C.POINTER(i64)]
    L.tms_partition_estimate.argtypes = [_VP, _VP, _VP, i64, C.POINTER(i64), _VP,
                                         C.POINTER(Stats)]
    L.tms_get_leaves.argtypes = [_VP, _VP, _VP, i64, C.POINTER(i64)]
    L.tms_extract_cube_vertices.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, i64, C.POINTER(i64)]
    L.tms_get_vertices.argtypes = [_VP, _VP, i64, C.POINTER(i64)]
    L.tms_get_corners.argtypes = [_VP, _VP, _VP, i64, C.POINTER(i64)]
    L.tms_build_cells_batch.argtypes = [_VP, _VP, C.POINTER(i64), i32, C.POINTER(Params),
                                        C.POINTER(_VP)]
    L.tms_batch_counts.argtypes = [_VP, _VP, C.POINTER(i64), C.POINTER(i64)]
    L.tms_graph_capture.argtypes = [_VP, _VP, C.c_double]
    L.tms_graph_capacity.argtypes = [_VP, _VP, C.c_double, C.POINTER(i64), C.POINTER(i64)]
    L.tms_graph_capture_into.argtypes = [_VP, _VP, C.c_double, _VP, _VP, i64, _VP, i64]
    L.tms_graph_launch.argtypes = [_VP, _VP, _VP, _VP, i64, C.POINTER(i64), _VP, i64,
                                   C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                                   C.POINTER(Stats)]
    L.tms_set_tuning.argtypes = [_VP, C.POINTER(Tuning)]
    L.tms_get_tuning.argtypes = [_VP, C.POINTER(Tuning)]
    L.tms_autotune.argtypes = [_VP, _VP, C.POINTER(Tuning), C.POINTER(C.c_double),
                               C.POINTER(i32)]
    L.tms_backward.argtypes = [_VP, _VP, _VP, i64, _VP, i64, _VP]
    L.tms_set_timing.argtypes = [_VP, i32]
    L.tms_get_timing.argtypes = [_VP, C.POINTER(Timing), i32]
    L.tms_debug_tensor.argtypes = [_VP, _VP, _VP, i64, i32, _VP, _VP]
    L.tms_debug_bound.argtypes = [_VP, _VP, _VP, i64, _VP]
    L.tms_debug_fast_exp.argtypes = [_VP, _VP, i64, _VP]
    L.tms_debug_phi_pairs.argtypes = [_VP, _VP, _VP, i64, C.POINTER(i64)]
    L.tms_mesh_build.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, i64, i32, C.POINTER(_VP)]
    L.tms_mesh_build_host.argtypes = [_VP, i64, _VP, _VP, i64, C.c_double, i32, C.c_double,
                                      C.POINTER(_VP), C.c_char_p, i64]
    L.tms_mesh_info.argtypes = [_VP] + [C.POINTER(i64)] * 5
    L.tms_mesh_get.argtypes = [_VP, _VP, _VP, _VP]
    L.tms_mesh_added.argtypes = [_VP, _VP, _VP, i64, C.POINTER(i64)]
    L.tms_mesh_check.argtypes = [_VP, i32, C.POINTER(MeshReport)]
    L.tms_mesh_write_off.argtypes = [_VP, C.c_char_p]
    L.tms_mesh_free.argtypes = [_VP]
    for f in ("tms_mesh_build", "tms_mesh_build_host", "tms_mesh_info", "tms_mesh_get",
              "tms_mesh_added", "tms_mesh_check",
              "tms_mesh_write_off", "tms_mesh_free"):
        getattr(L, f).restype = i32
    for f in ("tms_create", "tms_destroy", "tms_check_params", "tms_check_atoms_host",
              "tms_build_cells", "tms_cells_info", "tms_free_cells", "tms_eval_phi",
              "tms_eval_phi_noalloc", "tms_stage2_points", "tms_debug_phi_pairs",
              "tms_partition_estimate", "tms_get_leaves", "tms_extract_cube_vertices",
              "tms_get_vertices", "tms_debug_tensor", "tms_debug_bound", "tms_set_timing",
              "tms_get_timing", "tms_debug_fast_exp", "tms_get_corners", "tms_backward",
              "tms_build_cells_batch", "tms_batch_counts", "tms_set_tuning", "tms_get_tuning",
              "tms_autotune", "tms_graph_capture", "tms_graph_capacity", "tms_graph_capture_into",
              "tms_graph_launch"):
        getattr(L, f).restype = i32
    _lib = L
    return L


def make_params(D=0.9, c=1.0, tau=1e-3, h0=2.0, h_min=0.25, pad=3.0, eps_cut=1e-10,
                precision=PREC_FP64, mode=MODE_ADAPTIVE, degree=3,
                child_tensor=CHILD_PROJECT) -> Params:
    return Params(D=float(D), c=float(c), tau=float(tau), h0=float(h0), h_min=float(h_min),
                  pad=float(pad), eps_cut=float(eps_cut), precision=int(precision),
                  mode=int(mode), degree=int(degree), child_tensor=int(child_tensor))


def check_params(p: Params):
    buf = C.create_string_buffer(256)
    rc = load_library().tms_check_params(C.byref(p), buf, 256)
    return rc, buf.value.decode()


def check_atoms_host(xyzr: np.ndarray, p: Params):
    a = np.ascontiguousarray(xyzr, dtype=np.float64).reshape(-1, 4)
    buf = C.create_string_buffer(256)
    rc = load_library().tms_check_atoms_host(a.ctypes.data_as(C.POINTER(C.c_double)),
                                             a.shape[0], C.byref(p), buf, 256)
    return rc, buf.value.decode()


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


@dataclass
class Cells:
    handle: C.c_void_p
    params: Params
    n_atoms: int
    origin: np.ndarray   # conformation 0
    dims: np.ndarray     # conformation 0
    K: int
    rc2: float           # conformation 0
    n_conf: int = 1


class Context:
    """A library context on one device and torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = _VP()
        rc = self.lib.tms_create(C.byref(h), int(device), _VP(stream.cuda_stream))
        if rc != TMS_OK:
            raise TmsError(rc, self.lib.tms_last_error(None).decode())
        self.h = h
        self._bound = None  # output tensors a capture writes into

    def close(self):
        if getattr(self, "h", None):
            self.lib.tms_destroy(self.h)
            self.h = None
        self._bound = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != TMS_OK:
            raise TmsError(rc, self.lib.tms_last_error(self.h).decode())

    # ---------------------------------------------------------------- cells
    def build_cells(self, xyzr, params: Params, cells: Cells | None = None) -> Cells:
        t = self._torch
        a = xyzr if isinstance(xyzr, t.Tensor) else t.as_tensor(np.asarray(xyzr))
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        assert a.dim() == 2 and a.shape[1] == 4
        h = cells.handle if cells is not None else _VP()
        self._check(self.lib.tms_build_cells(self.h, _VP(_ptr(a)), a.shape[0], C.byref(params),
                                             C.byref(h)))
        o = (C.c_double * 3)()
        d = (C.c_int64 * 3)()
        K = C.c_int32()
        rc2 = C.c_double()
        na = C.c_int64()
        self.lib.tms_cells_info(h, o, d, C.byref(K), C.byref(rc2), C.byref(na))
        return Cells(h, params, int(na.value), np.array(o[:]), np.array(d[:]), int(K.value),
                     float(rc2.value))

    def build_cells_batch(self, confs, params: Params, cells: Cells | None = None) -> Cells:
        """Cells of a batch: `confs` is a list of [N_b, 4] arrays/tensors, or a
        (concatenated [N, 4] tensor, offsets [n_conf + 1]) pair."""
        t = self._torch
        if isinstance(confs, tuple):
            a, off = confs
            off = np.asarray(off, dtype=np.int64)
        else:
            parts = [np.asarray(c.cpu() if isinstance(c, t.Tensor) else c, dtype=np.float64)
                     .reshape(-1, 4) for c in confs]
            off = np.zeros(len(parts) + 1, dtype=np.int64)
            off[1:] = np.cumsum([len(x) for x in parts])
            a = np.concatenate(parts, axis=0) if parts else np.zeros((0, 4))
        a = a if isinstance(a, t.Tensor) else t.as_tensor(np.asarray(a))
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        offc = np.ascontiguousarray(off, dtype=np.int64)
        h = cells.handle if cells is not None else _VP()
        self._check(self.lib.tms_build_cells_batch(
            self.h, _VP(_ptr(a)), offc.ctypes.data_as(C.POINTER(C.c_int64)), len(offc) - 1,
            C.byref(params), C.byref(h)))
        o = (C.c_double * 3)()
        d = (C.c_int64 * 3)()
        K = C.c_int32()
        rc2 = C.c_double()
        na = C.c_int64()
        self.lib.tms_cells_info(h, o, d, C.byref(K), C.byref(rc2), C.byref(na))
        return Cells(h, params, int(na.value), np.array(o[:]), np.array(d[:]), int(K.value),
                     float(rc2.value), n_conf=len(offc) - 1)

    def batch_counts(self, cells: Cells, vertices: bool = True):
        """(leaf offsets, vertex offsets or None) [n_conf + 1] of the kept results."""
        lo = np.zeros(cells.n_conf + 1, dtype=np.int64)
        vo = np.zeros(cells.n_conf + 1, dtype=np.int64)
        P = C.POINTER(C.c_int64)
        self._check(self.lib.tms_batch_counts(self.h, cells.handle, lo.ctypes.data_as(P),
                                              vo.ctypes.data_as(P) if vertices else None))
        return lo, (vo if vertices else None)

    def free_cells(self, cells: Cells):
        self._check(self.lib.tms_free_cells(self.h, cells.handle))

    # ------------------------------------------------------------------ phi
    def eval_phi(self, cells: Cells, pts, grad: bool = False):
        t = self._torch
        p = pts if isinstance(pts, t.Tensor) else t.as_tensor(np.asarray(pts))
        p = p.to(device=self.device, dtype=t.float64).contiguous()
        m = p.shape[0]
        phi = t.empty(m, dtype=t.float64, device=self.device)
        g = t.empty((m, 3), dtype=t.float64, device=self.device) if grad else None
        ng = C.c_int64()
        self._check(self.lib.tms_eval_phi(self.h, cells.handle, _VP(_ptr(p)), m, _VP(_ptr(phi)),
                                          _VP(_ptr(g)), C.byref(ng)))
        return phi, g, int(ng.value)

    def eval_phi_noalloc(self, cells: Cells, pts, phi, grad=None):
        """tms_eval_phi_noalloc: phi (and grad) at the points of a device
        [m, 3] float64 tensor into the caller's tensors; the library allocates
        nothing.  Returns the number of points recomputed in double precision."""
        ng = C.c_int64()
        self._check(self.lib.tms_eval_phi_noalloc(self.h, cells.handle, _VP(_ptr(pts)),
                                                  pts.shape[0], _VP(_ptr(phi)), _VP(_ptr(grad)),
                                                  C.byref(ng)))
        return int(ng.value)

    # ------------------------------------------------------------ partition
    def mesh_build(self, cells: Cells, leaves, cphi, verts, close: bool = True) -> "Mesh":
        """tms_mesh_build on device tensors from partition_estimate / extract;
        close: add the cubes across open faces (TMS_MESH_CLOSE)."""
        h = _VP()
        self._check(self.lib.tms_mesh_build(self.h, cells.handle, _VP(_ptr(leaves)),
                                            leaves.shape[0], _VP(_ptr(cphi)), _VP(_ptr(verts)),
                                            verts.shape[0], MESH_CLOSE if close else 0,
                                            C.byref(h)))
        return Mesh(self.lib, h)

    def partition_estimate(self, cells: Cells, cap: int | None = None):
        """Returns (leaves uint8 tensor [L, 20], corner_phi [L, 8], stats dict)."""
        t = self._torch
        st = Stats()
        n = C.c_int64()
        if cap is None:
            self._check(self.lib.tms_partition_estimate(self.h, cells.handle, None, 0,
                                                         C.byref(n), None, C.byref(st)))
            cap = n.value
            leaves = t.empty((max(cap, 1), 20), dtype=t.uint8, device=self.device)
            cphi = t.empty((max(cap, 1), 8), dtype=t.float64, device=self.device)
            self._check(self.lib.tms_get_leaves(self.h, _VP(_ptr(leaves)), _VP(_ptr(cphi)), cap,
                                                C.byref(n)))
        else:
            leaves = t.empty((max(cap, 1), 20), dtype=t.uint8, device=self.device)
            cphi = t.empty((max(cap, 1), 8), dtype=t.float64, device=self.device)
            rc = self.lib.tms_partition_estimate(self.h, cells.handle, _VP(_ptr(leaves)), cap,
                                                 C.byref(n), _VP(_ptr(cphi)), C.byref(st))
            if rc == TMS_E_CAPACITY:
                cap = n.value
                leaves = t.empty((max(cap, 1), 20), dtype=t.uint8, device=self.device)
                cphi = t.empty((max(cap, 1), 8), dtype=t.float64, device=self.device)
                rc = self.lib.tms_get_leaves(self.h, _VP(_ptr(leaves)), _VP(_ptr(cphi)), cap,
                                             C.byref(n))
            self._check(rc)
        L = n.value
        return leaves[:L], cphi[:L], st.as_dict()

    def partition_into(self, cells: Cells, leaves, cphi):
        """Partition into preallocated buffers; returns (L, stats) or raises
        TmsError(TMS_E_CAPACITY) with the required size in .required."""
        st = Stats()
        n = C.c_int64()
        rc = self.lib.tms_partition_estimate(self.h, cells.handle, _VP(_ptr(leaves)),
                                             leaves.shape[0], C.byref(n), _VP(_ptr(cphi)),
                                             C.byref(st))
        if rc == TMS_E_CAPACITY:
            e = TmsError(rc, self.lib.tms_last_error(self.h).decode())
            e.required = n.value
            raise e
        self._check(rc)
        return n.value, st

    def extract(self, cells: Cells, leaves, corner_phi=None, cap: int | None = None):
        """Returns vertex uint8 tensor [V, 40]."""
        t = self._torch
        n = C.c_int64()
        nl = leaves.shape[0]
        if cap is None:
            self._check(self.lib.tms_extract_cube_vertices(
                self.h, cells.handle, _VP(_ptr(leaves)), nl, _VP(_ptr(corner_phi)), None, 0,
                C.byref(n)))
            cap = n.value
            out = t.empty((max(cap, 1), 40), dtype=t.uint8, device=self.device)
            self._check(self.lib.tms_get_vertices(self.h, _VP(_ptr(out)), cap, C.byref(n)))
        else:
            out = t.empty((max(cap, 1), 40), dtype=t.uint8, device=self.device)
            rc = self.lib.tms_extract_cube_vertices(self.h, cells.handle, _VP(_ptr(leaves)), nl,
                                                    _VP(_ptr(corner_phi)), _VP(_ptr(out)), cap,
                                                    C.byref(n))
            if rc == TMS_E_CAPACITY:
                cap = n.value
                out = t.empty((max(cap, 1), 40), dtype=t.uint8, device=self.device)
                rc = self.lib.tms_get_vertices(self.h, _VP(_ptr(out)), cap, C.byref(n))
            self._check(rc)
        return out[:n.value]

    def stage2_points(self, cells: Cells, leaves, corner_phi, cap: int | None = None):
        """tms_stage2_points: fold segments and critical points (Section 2.3)
        of the SURFACE leaves.  Returns (records uint8 tensor [P, 32],
        degenerate count)."""
        t = self._torch
        n = leaves.shape[0]
        cnt = C.c_int64()
        nd = C.c_int64()
        if cap is None:
            self._check(self.lib.tms_stage2_points(self.h, cells.handle, _VP(_ptr(leaves)), n,
                                                   _VP(_ptr(corner_phi)), None, 0,
                                                   C.byref(cnt), C.byref(nd)))
            cap = cnt.value
        out = t.empty((max(cap, 1), 32), dtype=t.uint8, device=self.device)
        self._check(self.lib.tms_stage2_points(self.h, cells.handle, _VP(_ptr(leaves)), n,
                                               _VP(_ptr(corner_phi)), _VP(out.data_ptr()), cap,
                                               C.byref(cnt), C.byref(nd)))
        return out[:cnt.value], int(nd.value)

    def get_vertices(self):
        """Vertices [V, 40] of the last extraction."""
        t = self._torch
        n = C.c_int64()
        self._check(self.lib.tms_get_vertices(self.h, None, 0, C.byref(n)))
        out = t.empty((max(n.value, 1), 40), dtype=t.uint8, device=self.device)
        self._check(self.lib.tms_get_vertices(self.h, _VP(_ptr(out)), n.value, C.byref(n)))
        return out[:n.value]

    def extract_into(self, cells: Cells, leaves, nl: int, corner_phi, out):
        n = C.c_int64()
        rc = self.lib.tms_extract_cube_vertices(self.h, cells.handle, _VP(_ptr(leaves)), nl,
                                                _VP(_ptr(corner_phi)), _VP(_ptr(out)),
                                                out.shape[0], C.byref(n))
        if rc == TMS_E_CAPACITY:
            e = TmsError(rc, self.lib.tms_last_error(self.h).decode())
            e.required = n.value
            raise e
        self._check(rc)
        return n.value

    # --------------------------------------------------------------- adjoint
    def get_corners(self):
        """Unique corners of the last pass: (xyz [M, 3], phi [M])."""
        t = self._torch
        n = C.c_int64()
        self._check(self.lib.tms_get_corners(self.h, None, None, 0, C.byref(n)))
        m = n.value
        xyz = t.empty((max(m, 1), 3), dtype=t.float64, device=self.device)
        phi = t.empty(max(m, 1), dtype=t.float64, device=self.device)
        self._check(self.lib.tms_get_corners(self.h, _VP(_ptr(xyz)), _VP(_ptr(phi)), m,
                                             C.byref(n)))
        return xyz[:m], phi[:m]

    def backward(self, cells: Cells, dphi=None, dt=None, out=None):
        """dL/d(x, y, z, r) of every atom [N, 4] from dL/dphi at the kept corners
        and dL/dt at the kept edge points (either may be None)."""
        t = self._torch
        if out is None:
            out = t.empty((cells.n_atoms, 4), dtype=t.float64, device=self.device)
        assert out.dtype == t.float64 and out.is_contiguous() and out.shape == (cells.n_atoms, 4)
        for a in (dphi, dt):
            assert a is None or (a.dtype == t.float64 and a.is_contiguous() and a.dim() == 1)
        self._check(self.lib.tms_backward(self.h, cells.handle, _VP(_ptr(dphi)),
                                          0 if dphi is None else dphi.shape[0], _VP(_ptr(dt)),
                                          0 if dt is None else dt.shape[0], _VP(_ptr(out))))
        return out

    # --------------------------------------------------------- captured pass
    def graph_capacity(self, cells: Cells, margin: float = 1.25):
        """(leaf capacity, vertex capacity) of a capture with this margin: the
        sizes buffers bound by graph_capture must hold."""
        nl = C.c_int64()
        nv = C.c_int64()
        self._check(self.lib.tms_graph_capacity(self.h, cells.handle, float(margin),
                                                C.byref(nl), C.byref(nv)))
        return nl.value, nv.value

    def graph_capture(self, cells: Cells, margin: float = 1.25, leaves=None, cphi=None,
                      verts=None):
        """Record the pass (partition + corners + extraction) of `cells` into a
        HIP graph; needs an eager partition and extraction of them first.
        Tensors given for leaves (uint8 [cap, 20]), cphi (float64 [cap, 8]) or
        verts (uint8 [cap, 40]) are bound: the graph writes its results there
        (each must hold graph_capacity's figure), and the context keeps them
        alive while the capture stands."""
        if leaves is None and cphi is None and verts is None:
            self._check(self.lib.tms_graph_capture(self.h, cells.handle, float(margin)))
            self._bound = None
            return
        caps = [t.shape[0] for t in (leaves, cphi) if t is not None]
        self._check(self.lib.tms_graph_capture_into(
            self.h, cells.handle, float(margin), _VP(_ptr(leaves)), _VP(_ptr(cphi)),
            min(caps) if caps else 0, _VP(_ptr(verts)), 0 if verts is None else verts.shape[0]))
        self._bound = (leaves, cphi, verts)

    def graph_launch(self, cells: Cells, leaves=None, cphi=None, verts=None, offsets=False):
        """Replay the captured pass; returns (n_leaves, n_verts, stats dict
        [, (leaf offsets, vertex offsets)])."""
        nl = C.c_int64()
        nv = C.c_int64()
        st = Stats()
        lo = np.zeros(cells.n_conf + 1, dtype=np.int64) if offsets else None
        vo = np.zeros(cells.n_conf + 1, dtype=np.int64) if offsets else None
        P = C.POINTER(C.c_int64)
        self._check(self.lib.tms_graph_launch(
            self.h, cells.handle, _VP(_ptr(leaves)), _VP(_ptr(cphi)),
            0 if leaves is None else leaves.shape[0], C.byref(nl), _VP(_ptr(verts)),
            0 if verts is None else verts.shape[0], C.byref(nv),
            lo.ctypes.data_as(P) if offsets else None, vo.ctypes.data_as(P) if offsets else None,
            C.byref(st)))
        r = (nl.value, nv.value, st.as_dict())
        return r + ((lo, vo),) if offsets else r

    # ---------------------------------------------------------------- tuning
    def set_tuning(self, slice_cubes=None, tiled_min_level=None, tile_atoms=None,
                   proj_table=None, tiled_persistent=None, tiled_half=None,
                   corner_groups=None, corner_reach=None):
        t = self.get_tuning()
        if slice_cubes is not None:
            t.slice_cubes = int(slice_cubes)
        if tiled_min_level is not None:
            t.tiled_min_level = int(tiled_min_level)
        if tile_atoms is not None:
            t.tile_atoms = int(tile_atoms)
        if proj_table is not None:
            t.proj_table = int(proj_table)
        if tiled_persistent is not None:
            t.tiled_persistent = int(tiled_persistent)
        if tiled_half is not None:
            t.tiled_half = int(tiled_half)
        if corner_groups is not None:
            t.corner_groups = int(corner_groups)
        if corner_reach is not None:
            t.corner_reach = int(corner_reach)
        self._check(self.lib.tms_set_tuning(self.h, C.byref(t)))

    def get_tuning(self) -> Tuning:
        t = Tuning()
        self._check(self.lib.tms_get_tuning(self.h, C.byref(t)))
        return t

    def autotune(self, cells: Cells):
        """Runs the library's autotuner on `cells`; returns (tuning dict, best ms, passes)."""
        t = Tuning()
        ms = C.c_double()
        n = C.c_int32()
        self._check(self.lib.tms_autotune(self.h, cells.handle, C.byref(t), C.byref(ms),
                                          C.byref(n)))
        return t.as_dict(), ms.value, n.value

    # ---------------------------------------------------------------- timing
    def set_timing(self, enable: bool):
        self._check(self.lib.tms_set_timing(self.h, int(bool(enable))))

    def get_timing(self, reset: bool = False) -> dict:
        t = Timing()
        self._check(self.lib.tms_get_timing(self.h, C.byref(t), int(bool(reset))))
        return t.as_dict()

    # ----------------------------------------------------------------- debug
    def debug_tensor(self, cells: Cells, cubes, precision=PREC_FP64, with_scale=False):
        t = self._torch
        cb = t.as_tensor(np.asarray(cubes, dtype=np.int32)).to(self.device).contiguous()
        A = t.zeros((cb.shape[0], 64), dtype=t.float64, device=self.device)
        S = t.zeros(cb.shape[0], dtype=t.float64, device=self.device) if with_scale else None
        self._check(self.lib.tms_debug_tensor(self.h, cells.handle, _VP(_ptr(cb)), cb.shape[0],
                                              int(precision), _VP(_ptr(A)), _VP(_ptr(S))))
        return (A, S) if with_scale else A

    def debug_fast_exp(self, x):
        t = self._torch
        xx = t.as_tensor(np.asarray(x, dtype=np.float64)).to(self.device).contiguous()
        y = t.empty_like(xx)
        self._check(self.lib.tms_debug_fast_exp(self.h, _VP(_ptr(xx)), xx.shape[0],
                                                _VP(_ptr(y))))
        return y

    def debug_phi_pairs(self, cells: Cells, pts) -> int:
        """(point, atom) pairs within R_c over the points (phi's terms)."""
        t = self._torch
        p = pts if isinstance(pts, t.Tensor) else t.as_tensor(np.asarray(pts))
        p = p.to(device=self.device, dtype=t.float64).contiguous()
        n = C.c_int64()
        self._check(self.lib.tms_debug_phi_pairs(self.h, cells.handle, _VP(_ptr(p)), p.shape[0],
                                                 C.byref(n)))
        return int(n.value)

    def debug_bound(self, A, band=None):
        """Returns [n, 6]: L, U, rho, r, jump, amp."""
        t = self._torch
        a = t.as_tensor(np.asarray(A, dtype=np.float64)).reshape(-1, 64).to(self.device)
        a = a.contiguous()
        b = None
        if band is not None:
            b = t.as_tensor(np.asarray(band, dtype=np.float64)).to(self.device).contiguous()
        out = t.zeros((a.shape[0], 6), dtype=t.float64, device=self.device)
        self._check(self.lib.tms_debug_bound(self.h, _VP(_ptr(a)), _VP(_ptr(b)), a.shape[0],
                                             _VP(_ptr(out))))
        return out


def leaves_to_numpy(leaves) -> np.ndarray:
    return leaves.cpu().numpy().reshape(-1).view(LEAF_DTYPE)


S2_DTYPE = np.dtype([("leaf", "<i4"), ("kind", "u1"), ("axis", "u1"), ("root", "u1"),
                     ("pad", "u1"), ("x", "<f8"), ("y", "<f8"), ("z", "<f8")])
S2_FOLD, S2_CRITICAL = 0, 1


def s2_to_numpy(recs) -> np.ndarray:
    return np.frombuffer(recs.cpu().numpy().tobytes(), dtype=S2_DTYPE)


def vertices_to_numpy(verts) -> np.ndarray:
    return verts.cpu().numpy().reshape(-1).view(VERTEX_DTYPE)


def vertex_t(verts):
    """The t column of a vertex tensor [V, 40] (uint8) as float64 [V]."""
    return verts.view(-1).view(__import__("torch").float64).view(-1, 5)[:, 1]


def vertex_edge_h(verts, h0: float):
    """Edge length of every vertex's edge, from the level in its key."""
    import torch
    key = verts.view(-1).view(torch.int64).view(-1, 5)[:, 0]
    level = (key >> 50) & 7
    return h0 * torch.pow(torch.tensor(0.5, dtype=torch.float64, device=verts.device),
                          level.to(torch.float64))


def _surface_function():
    import torch

    class GaussianSurface(torch.autograd.Function):
        """Differentiable pass: atoms [N, 4] (x, y, z, r) -> (phi at the unique
        leaf corners [M], t of the edge points [V]).  The backward runs the
        library's adjoint kernels with the discrete structure of the forward
        pass held fixed."""

        @staticmethod
        def forward(fctx, xyzr, tctx, params):
            cells = tctx.build_cells(xyzr.detach(), params)
            leaves, cphi, st = tctx.partition_estimate(cells)
            verts = tctx.extract(cells, leaves, cphi)
            _, phi = tctx.get_corners()
            fctx.tctx = tctx
            fctx.cells = cells
            fctx.info = dict(leaves=leaves, verts=verts, stats=st)
            return phi, vertex_t(verts).clone()

        @staticmethod
        def backward(fctx, dphi, dt):
            tctx, cells = fctx.tctx, fctx.cells
            g = tctx.backward(cells, None if dphi is None else dphi.contiguous(),
                              None if dt is None else dt.contiguous())
            tctx.free_cells(cells)
            return g, None, None

    return GaussianSurface


_GS = None


def gaussian_surface(xyzr, tctx: Context, params: Params):
    """(phi at the unique leaf corners, t of the edge points), differentiable
    with respect to xyzr through the library's adjoint."""
    global _GS
    if _GS is None:
        _GS = _surface_function()
    return _GS.apply(xyzr, tctx, params)
