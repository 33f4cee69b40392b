"""Seeded synthetic atom sets shaped like the proteins the method is meant for.

This module only draws coordinates and radii; it contains none of the
method's arithmetic, and both the HIP path and the CPU oracle consume its
output.  The paper measures on a benchmark of real PQR structures (7 to about
1.08 M atoms); those structures are not reproduced here -- these generators
stand in for them with the same sizes and packing density.

Globule G(N, seed)
    Confinement radius R_g = (3N / (4 pi 0.05))^(1/3) (heavy-atom density
    0.05 per cubic angstrom).  Residues are one C-alpha plus 2..10 side atoms.
    The C-alphas follow a random walk with 3.8 A steps in uniformly random
    directions; a step is redrawn (up to 100 times) when it leaves the sphere
    of radius R_g - 1.5 or comes within 3.0 A of an earlier C-alpha, and after
    100 failures the walk restarts from a random earlier C-alpha (after every
    50 failed restarts the sphere grows by 10 %, which only happens for very
    small N).  Side atoms
    form a bonded branch: each sits at a distance drawn from U[1.2, 1.5] A
    from the previous atom of its residue and is redrawn (up to 100 times)
    when it comes within 2.0 A of any atom other than that parent; a branch
    that cannot grow ends early.  Elements are drawn C/N/O/S with
    probabilities 0.62/0.17/0.19/0.02 and radii 1.7/1.55/1.52/1.8 A.
Hydrogens
    1.0 A from a uniformly chosen heavy atom in a random direction, redrawn
    when within 1.5 A of another heavy atom; radius 1.2 A.
Assembly
    20 globules G(5000, seed + k) centred on the first 20 sites (in
    lexicographic order) of a 3x3x3 cubic lattice whose spacing is
    max_k 2 (rho_k + 1.8) + 2 A, rho_k the largest centre distance of
    globule k from its centroid, so bounding spheres keep a 2 A gap; plus
    hydrogens numbering 10 % of the heavy atoms.
Batch
    N_b = round(exp(U(ln 500, ln 20000))); conformation b is G(N_b, seed_b)
    plus iid N(0, 0.3^2) A noise on every coordinate.
"""
from __future__ import annotations

import math

import numpy as np

ELEM_P = np.array([0.62, 0.17, 0.19, 0.02])
ELEM_R = np.array([1.7, 1.55, 1.52, 1.8])
H_RADIUS = 1.2


class _Grid:
    """Spatial hash of placed atoms for the rejection tests."""

    def __init__(self, cell: float):
        self.cell = cell
        self.cells: dict = {}
        self.n = 0

    def add(self, p) -> int:
        idx = self.n
        self.n += 1
        x, y, z = float(p[0]), float(p[1]), float(p[2])
        c = self.cell
        key = (math.floor(x / c), math.floor(y / c), math.floor(z / c))
        self.cells.setdefault(key, []).append((idx, x, y, z))
        return idx

    def near(self, p, r: float, skip: int = -1) -> bool:
        px, py, pz = float(p[0]), float(p[1]), float(p[2])
        c = self.cell
        kx, ky, kz = math.floor(px / c), math.floor(py / c), math.floor(pz / c)
        r2 = r * r
        get = self.cells.get
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    lst = get((kx + dx, ky + dy, kz + dz))
                    if lst is None:
                        continue
                    for j, qx, qy, qz in lst:
                        ex, ey, ez = px - qx, py - qy, pz - qz
                        if ex * ex + ey * ey + ez * ez < r2 and j != skip:
                            return True
        return False


def _unit(rng):
    x, y, z = rng.normal(size=3).tolist()
    n = math.sqrt(x * x + y * y + z * z)
    return (x / n, y / n, z / n)


def _step(p, d, u):
    return (p[0] + d * u[0], p[1] + d * u[1], p[2] + d * u[2])


def globule(n: int, seed: int) -> np.ndarray:
    """G(n, seed): [n, 4] float64 array of (x, y, z, r)."""
    rng = np.random.default_rng(seed)
    rg = (3.0 * n / (4.0 * math.pi * 0.05)) ** (1.0 / 3.0)
    rwalk = max(rg - 1.5, 2.0)
    ca = _Grid(3.0)       # C-alphas only
    allg = _Grid(2.0)     # every atom
    pos = []
    cur = (0.0, 0.0, 0.0)
    ca_idx = []
    fails = 0
    while len(pos) < n:
        # next C-alpha
        if not ca_idx:
            p = (0.0, 0.0, 0.0)
        else:
            placed = False
            for _ in range(100):
                p = _step(cur, 3.8, _unit(rng))
                if math.sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) <= rwalk \
                        and not ca.near(p, 3.0):
                    placed = True
                    break
            if not placed:
                fails += 1
                if fails % 50 == 0:
                    rwalk *= 1.1  # too tight for the walk: loosen the sphere
                cur = pos[ca_idx[int(rng.integers(len(ca_idx)))]]
                continue
        ca.add(p)
        gi = allg.add(p)
        ca_idx.append(len(pos))
        pos.append(p)
        cur = p
        # side branch
        ns = int(rng.integers(2, 11))
        parent, pidx = p, gi
        for _ in range(ns):
            if len(pos) >= n:
                break
            ok = False
            for _ in range(100):
                d = rng.uniform(1.2, 1.5)
                q = _step(parent, d, _unit(rng))
                if not allg.near(q, 2.0, skip=pidx):
                    ok = True
                    break
            if not ok:
                break
            pidx = allg.add(q)
            pos.append(q)
            parent = q
    xyz = np.array(pos[:n], dtype=np.float64)
    el = rng.choice(4, size=n, p=ELEM_P)
    out = np.empty((n, 4))
    out[:, :3] = xyz
    out[:, 3] = ELEM_R[el]
    return out


def add_hydrogens(heavy: np.ndarray, frac: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    nh = int(round(frac * heavy.shape[0]))
    g = _Grid(1.5)
    for p in heavy[:, :3]:
        g.add(p)
    hs = []
    while len(hs) < nh:
        k = int(rng.integers(heavy.shape[0]))
        q = _step(tuple(heavy[k, :3].tolist()), 1.0, _unit(rng))
        if g.near(q, 1.5, skip=k):
            continue
        hs.append(q)
    h = np.empty((nh, 4))
    if nh:
        h[:, :3] = np.array(hs)
    h[:, 3] = H_RADIUS
    return np.concatenate([heavy, h], axis=0)


def assembly(n_glob: int = 20, n_each: int = 5000, seed: int = 1003,
             h_frac: float = 0.10) -> np.ndarray:
    globs = [globule(n_each, seed + k) for k in range(n_glob)]
    cents = [g[:, :3].mean(axis=0) for g in globs]
    rho = [float(np.max(np.linalg.norm(g[:, :3] - c, axis=1))) for g, c in zip(globs, cents)]
    spacing = max(2.0 * (r + 1.8) for r in rho) + 2.0
    sites = [(i, j, k) for i in range(3) for j in range(3) for k in range(3)][:n_glob]
    parts = []
    for g, c, s in zip(globs, cents, sites):
        h = g.copy()
        h[:, :3] += spacing * np.array(s, dtype=np.float64) - c
        parts.append(h)
    heavy = np.concatenate(parts, axis=0)
    return add_hydrogens(heavy, h_frac, seed + 1000)


def batch_sizes(n_conf: int = 256, seed: int = 1005, lo: int = 500, hi: int = 20000):
    rng = np.random.default_rng(seed * 10)
    return [int(round(math.exp(v))) for v in rng.uniform(math.log(lo), math.log(hi), n_conf)]


def batch(n_conf: int = 256, seed: int = 1005, sigma: float = 0.3, sizes=None):
    """List of [N_b, 4] arrays."""
    sizes = batch_sizes(n_conf, seed) if sizes is None else sizes
    out = []
    for b, nb in enumerate(sizes):
        g = globule(nb, seed + b)
        rng = np.random.default_rng((seed + b) * 7919)
        g[:, :3] += rng.normal(scale=sigma, size=(nb, 3))
        out.append(g)
    return out
