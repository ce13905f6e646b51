"""The synthetic workloads: meshes, fields, rules and coefficient laws.

Each workload is a plain description (mesh sizes, quadrature degree,
coefficient laws) plus generators; both the library under test and the CPU
reference receive the same arrays. Coefficient laws are given as data:
  ("const", value)           -> s = value
  ("poly2", a0, a1, a2)      -> s = a0 + a1*u + a2*u^2   with u = u_h at the q-point
  ("exp", a0, a1)            -> s = exp(a0 + a1*u)
Matrix naming follows the paper: the mass coefficient m, the conductivity
coefficient c (called k in the workload descriptions).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fields as F
from .mesh import structured_mesh
from .quadrature import rule


@dataclass
class Workload:
    name: str
    cfg_id: int
    dim: int
    order: int
    N: int
    jitter: float
    quad_degree: int
    mass_law: tuple
    stiff_law: tuple
    field_kind: str = "none"        # none | sinusoids8 | grf64 | heat
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_elem(self):
        return (2 * self.N ** 2) if self.dim == 2 else (6 * self.N ** 3)

    @property
    def n_nodes(self):
        return (self.order * self.N + 1) ** self.dim


# The named workloads (sizes of the full configurations).
WORKLOADS = {
    "p1_2d_64": Workload("p1_2d_64", 1, 2, 1, 64, 0.0, 2, ("const", 1.0), ("const", 1.0), "none",
                          "2D P1 unit square 64x64x2 triangles, 3-point rule, m=c=1"),
    "p2_3d_32": Workload("p2_3d_32", 2, 3, 2, 32, 0.2, 4, ("const", 1.0), ("poly2", 1.0, 0.0, 0.5), "sinusoids8",
                          "3D P2 Kuhn tets on 32^3 cube (196,608 elements), jitter 0.2h, 11-point rule, "
                          "c(u)=1+0.5u^2, u = sum of 8 random-phase sinusoids"),
    "p3_2d_1024": Workload("p3_2d_1024", 3, 2, 3, 1024, 0.25, 6, ("const", 1.0), ("exp", 0.0, 1.0), "grf64",
                            "2D P3 triangles on 1024^2 square (2,097,152 elements), jitter 0.25h, 12-point rule, "
                            "c(x)=exp(g(x)), g a unit-variance smooth Gaussian random field"),
    "p1_3d_96_heat": Workload("p1_3d_96_heat", 4, 3, 1, 96, 0.2, 2, ("poly2", 1.0, 0.1, 0.0), ("poly2", 1.0, 0.0, 1.0),
                               "heat", "3D P1 Kuhn tets on 96^3 cube (5,308,416 elements), c(u)=1+u^2, "
                               "m(u)=1+0.1u, 20 reassemblies with smooth increments of size 0.05"),
    # the 3D P3 shape (16-element tiles, Q^T read from L2): its precision forms and fix-up share
    "p3_3d_36": Workload("p3_3d_36", 6, 3, 3, 36, 0.2, 6, ("const", 1.0), ("poly2", 1.0, 0.0, 0.5), "sinusoids8",
                          "3D P3 Kuhn tets on 36^3 cube (279,936 elements), jitter 0.2h, 24-point rule, "
                          "c(u)=1+0.5u^2, u = sum of 8 random-phase sinusoids"),
}


def scaled(name: str, N: int) -> Workload:
    """The same workload on a smaller (or larger) mesh."""
    w = WORKLOADS[name]
    return Workload(w.name + f"@N{N}", w.cfg_id, w.dim, w.order, N, w.jitter, w.quad_degree,
                    w.mass_law, w.stiff_law, w.field_kind, w.description, dict(w.extra))


def make_inputs(w: Workload, stream: int = 0):
    """Mesh, quadrature rule and nodal field of a workload (all host numpy arrays)."""
    mesh = structured_mesh(w.dim, w.order, w.N, w.jitter, seed=[2204, w.cfg_id, 1000 + stream])
    pts, wts = rule(w.dim, w.quad_degree)
    rng = F.rng_for(w.cfg_id, stream)
    if w.field_kind == "none":
        u = np.zeros(mesh["n_nodes"])
    elif w.field_kind == "sinusoids8":
        u = F.random_sinusoids(mesh["coords"], 8, rng)
    elif w.field_kind == "grf64":
        u = F.gaussian_random_field(mesh["coords"], 64, rng, length=0.1)
    elif w.field_kind == "grf16":
        u = F.gaussian_random_field(mesh["coords"], 16, rng, length=0.1)
    elif w.field_kind == "heat":
        u = F.random_sinusoids(mesh["coords"], 8, rng, amplitude=1.0 / np.sqrt(8.0))
    else:
        raise ValueError(w.field_kind)
    return mesh, (pts, wts), u


def heat_increment(w: Workload, mesh, step: int):
    """Smooth increment delta_s with |delta_s| <= 1 for reassembly step s."""
    rng = F.rng_for(w.cfg_id, 100 + step)
    return 0.05 * F.random_sinusoids(mesh["coords"], 4, rng, amplitude=0.25)
