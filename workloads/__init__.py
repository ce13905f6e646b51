"""Seeded synthetic inputs (meshes, nodal fields, quadrature rules).

Shared by the library's tests, the benchmark and the CPU reference; holds no
part of the assembly arithmetic.
"""
from .mesh import structured_mesh, local_alpha, n_local, boundary_mask, nnz_closed_form  # noqa: F401
from .quadrature import rule, rule_degree, simplex_moment  # noqa: F401
from .configs import WORKLOADS, Workload, make_inputs, scaled, heat_increment  # noqa: F401
