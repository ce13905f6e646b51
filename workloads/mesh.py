"""Seeded structured simplex meshes standing in for the paper's unit-square meshes.

The paper's experiments use Gmsh meshes of the unit square (Section 6,
Experiment 1) that are not available; these generators produce meshes of the
same domain and element types with a chosen element count. Nothing here
computes any part of the assembly method: only node positions, connectivity
and the local node layout (which is a mesh-format convention, Section 3
step 3 defers the basis to textbooks).

Conventions (one mesh format shared by every consumer):
  * ``coords``: float64 SoA array [dim, n_nodes]; ``conn``: int32 SoA [n_p, n_elem].
  * Local node order: the d+1 vertices first, then P-1 equispaced nodes on each
    edge (2D edges (0,1),(1,2),(2,0); 3D edges (0,1),(1,2),(2,0),(0,3),(1,3),(2,3)),
    each running from the first to the second listed vertex, then for P3 one
    node per face (2D: the centroid; 3D: faces opposite vertex 3, 0, 1, 2).
    Local node i sits at barycentric coordinates alpha_i / P.
  * Global numbering: the (P*N+1)^d lattice of the P-refined grid, x fastest.
  * 2D cells split along the (i,j)->(i+1,j+1) diagonal; 3D cells split into the
    6 Kuhn tetrahedra along (0,0,0)->(1,1,1), one per axis permutation.
  * Jitter moves interior vertices by independent U(-a*h, a*h) per coordinate;
    higher-order nodes are then placed at their affine positions (straight
    sided elements, the affine map of Section 3 step 3).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def n_local(dim: int, order: int) -> int:
    return math.comb(order + dim, dim)


def local_alpha(dim: int, order: int) -> np.ndarray:
    """Barycentric multi-indices (|alpha| = order) of the local nodes, shape [n_p, dim+1]."""
    P = order
    rows = []
    for k in range(dim + 1):
        a = [0] * (dim + 1)
        a[k] = P
        rows.append(a)
    edges = [(0, 1), (1, 2), (2, 0)] if dim == 2 else [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]
    for (a_, b_) in edges:
        for t in range(1, P):
            a = [0] * (dim + 1)
            a[a_] = P - t
            a[b_] = t
            rows.append(a)
    if P == 3:
        if dim == 2:
            rows.append([1, 1, 1])
        else:
            for opp in (3, 0, 1, 2):
                rows.append([0 if k == opp else 1 for k in range(4)])
    if P > 3:
        raise ValueError("orders 1..3 only")
    out = np.array(rows, dtype=np.int64)
    assert out.shape[0] == n_local(dim, order)
    return out


def _cell_simplices(dim):
    """Vertex offsets (in cell units) of the simplices splitting one cell."""
    if dim == 2:
        return [[(0, 0), (1, 0), (1, 1)], [(0, 0), (1, 1), (0, 1)]]
    out = []
    for perm in itertools.permutations(range(3)):
        v = [0, 0, 0]
        verts = [tuple(v)]
        for ax in perm:
            v[ax] += 1
            verts.append(tuple(v))
        out.append(verts)
    return out


def structured_mesh(dim: int, order: int, N: int, jitter: float = 0.0, seed=None):
    """Unit square/cube, N cells per side, simplices of the given Lagrange order.

    Returns a dict with coords [dim, n_nodes] float64, conn [n_p, n_elem] int32,
    vertex_mask [n_nodes] bool, h, and sizes.
    """
    P = order
    h = 1.0 / N
    L = P * N + 1  # lattice points per side
    n_nodes = L ** dim
    alpha = local_alpha(dim, order)              # [n_p, dim+1]
    simp = np.array(_cell_simplices(dim), dtype=np.int64)  # [n_s, dim+1, dim]
    n_s = simp.shape[0]
    # cells, x fastest
    grids = np.meshgrid(*([np.arange(N)] * dim), indexing="ij")
    cell = np.stack([g.reshape(-1) for g in grids], axis=1)  # ij indexing -> first axis slowest
    # reorder so that x (axis 0) is fastest: sort by (z, y, x)
    keys = tuple(cell[:, k] for k in range(dim))  # lexsort uses last key as primary
    order_idx = np.lexsort(keys)
    cell = cell[order_idx]
    n_cells = cell.shape[0]
    # vertex lattice coords (cell units) of every simplex: [n_cells, n_s, dim+1, dim]
    vc = cell[:, None, None, :] + simp[None, :, :, :]
    vc = vc.reshape(n_cells * n_s, dim + 1, dim)
    # refined-lattice coordinate of each local node: sum_k alpha_k * vc_k
    node_lat = np.einsum("pk,ekd->epd", alpha, vc)       # [n_e, n_p, dim]
    strides = np.array([L ** k for k in range(dim)], dtype=np.int64)
    node_id = node_lat @ strides                          # [n_e, n_p]
    conn = np.ascontiguousarray(node_id.T).astype(np.int32)

    # vertex positions with jitter
    lat = np.stack(np.meshgrid(*([np.arange(L)] * dim), indexing="ij"), axis=0).reshape(dim, -1)
    # lattice id with x fastest: id = ix + L*iy + L^2*iz ; meshgrid 'ij' gives ix slowest, so remap
    ids = (lat * strides[:, None]).sum(axis=0)
    lat_by_id = np.empty_like(lat)
    lat_by_id[:, ids] = lat
    vertex_mask = np.all(lat_by_id % P == 0, axis=0)
    pos = lat_by_id.astype(np.float64) * (h / P)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        interior = vertex_mask & np.all((lat_by_id > 0) & (lat_by_id < L - 1), axis=0)
        idx = np.nonzero(interior)[0]
        pos[:, idx] += rng.uniform(-jitter * h, jitter * h, size=(dim, idx.size))
    if P > 1:
        # affine placement of non-vertex nodes from the element's (jittered) vertices
        vid = node_id[:, : dim + 1]                        # [n_e, dim+1]
        vx = pos[:, vid]                                   # [dim, n_e, dim+1]
        xn = np.einsum("pk,cek->cep", alpha.astype(np.float64) / P, vx)  # [dim, n_e, n_p]
        nonv = np.arange(dim + 1, alpha.shape[0])
        pos[:, node_id[:, nonv].reshape(-1)] = xn[:, :, nonv].reshape(dim, -1)
    return {
        "dim": dim,
        "order": order,
        "N": N,
        "h": h,
        "coords": np.ascontiguousarray(pos),
        "conn": conn,
        "vertex_mask": vertex_mask,
        "n_nodes": n_nodes,
        "n_elem": conn.shape[1],
        "n_p": alpha.shape[0],
    }


def boundary_mask(mesh) -> np.ndarray:
    """Nodes on the boundary of the unit square/cube (lattice extremes)."""
    dim = mesh["dim"]
    L = mesh["order"] * mesh["N"] + 1
    ids = np.arange(mesh["n_nodes"])
    out = np.zeros(mesh["n_nodes"], dtype=bool)
    for k in range(dim):
        c = (ids // (L ** k)) % L
        out |= (c == 0) | (c == L - 1)
    return out


def nnz_closed_form(dim: int, order: int, N: int) -> int:
    """Number of structural nonzeros of the P-order matrices on these meshes.

    Obtained by enumeration on small N and fitting (polynomials in N); used as
    a generator/pattern self-check.
    """
    if dim == 2:
        return {1: 7 * N * N + 6 * N + 1, 2: 46 * N * N + 16 * N + 1, 3: 153 * N * N + 30 * N + 1}[order]
    return {1: 15 * N ** 3 + 21 * N * N + 9 * N + 1,
            2: 230 * N ** 3 + 138 * N * N + 24 * N + 1,
            3: 1311 * N ** 3 + 459 * N * N + 45 * N + 1}[order]
