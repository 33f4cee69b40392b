"""Named synthetic workloads (sizes, seeds and surface parameters).

Pure data plus calls into ``synth``; no arithmetic of the method.  They stand
in for the paper's benchmark of PQR structures, whose files are not used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import synth


@dataclass(frozen=True)
class Workload:
    name: str
    description: str
    D: float
    c: float = 1.0
    tau: float = 1e-3
    h0: float = 2.0
    h_min: float = 0.25
    pad: float = 3.0
    eps_cut: float = 1e-10
    uniform: bool = False
    extra: dict = field(default_factory=dict)

    def params(self, precision: int):
        from .tms import MODE_ADAPTIVE, MODE_UNIFORM, make_params
        return make_params(D=self.D, c=self.c, tau=self.tau, h0=self.h0, h_min=self.h_min,
                           pad=self.pad, eps_cut=self.eps_cut, precision=precision,
                           mode=MODE_UNIFORM if self.uniform else MODE_ADAPTIVE)


GLOBULE200_UNIFORM = Workload(
    "globule200_uniform", "200-atom globule, plain method on a uniform h=0.5 grid",
    D=0.9, h0=0.5, h_min=0.5, uniform=True)
GLOBULE5K = {D: Workload("globule5k_D%g" % D, "5,000-atom globule, adaptive 2 -> 0.25, tau 1e-3",
                         D=D) for D in (0.5, 0.9, 1.5)}
GLOBULE20K_ADJOINT = Workload(
    "globule20k_adjoint",
    "20,000-atom globule, adaptive 2 -> 0.25, tau 1e-3; loss sum (phi - c)^2 over unique leaf "
    "corners + sum ((t - 1/2) h)^2 over edge points, gradient w.r.t. centres and radii", D=0.9)
BATCH256 = Workload(
    "batch256",
    "256 conformations, atom counts log-uniform in [500, 20000] (each its own globule plus "
    "N(0, 0.3^2) A coordinate noise), adaptive 2 -> 0.25, tau 1e-3, refined as one batch", D=0.9)
ASSEMBLY110K = Workload(
    "assembly110k",
    "110,000-atom assembly (20 globules of 5,000 atoms, 2 A gaps, plus 10% hydrogens r=1.2), "
    "adaptive 2 -> 0.25, tau 1e-3", D=0.9)


def atoms(w: Workload):
    if w.name == "globule200_uniform":
        return synth.globule(200, 1001)
    if w.name.startswith("globule5k"):
        return synth.globule(5000, 1002)
    if w.name == "globule20k_adjoint":
        return synth.globule(20000, 1004)
    if w.name == "batch256":
        return synth.batch(256, 1005)
    if w.name == "assembly110k":
        return synth.assembly(20, 5000, seed=1003, h_frac=0.10)
    raise KeyError(w.name)


def assembly_slice(atoms, n_glob: int = 4):
    """The first n_glob globules of the assembly with the hydrogens near
    them (every atom within a globule's largest centre distance + 1.05 A of
    its centroid): a bounded sample of the assembly workload that the FP64
    oracle finishes in seconds to tens of seconds.  Selection only."""
    import numpy as np
    sel = np.zeros(len(atoms), dtype=bool)
    for k in range(n_glob):
        heavy = atoms[5000 * k:5000 * (k + 1)]
        cen = heavy[:, :3].mean(axis=0)
        rho = np.max(np.linalg.norm(heavy[:, :3] - cen, axis=1))
        sel |= np.linalg.norm(atoms[:, :3] - cen, axis=1) <= rho + 1.05
    return atoms[sel]


ALL = {w.name: w for w in [GLOBULE200_UNIFORM, *GLOBULE5K.values(), GLOBULE20K_ADJOINT,
                           BATCH256, ASSEMBLY110K]}
