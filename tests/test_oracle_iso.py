"""Pins of the oracle's isoparametric (curved) elements: the element map uses the P-order
basis and every node's position, with B, |det B| and A per quadrature node.

Fixed by the mathematics: with nodes at their affine positions the map is affine and the
matrices equal the affine ones; on a curved mesh of the same domain the entries of M (m = 1)
sum to |Omega| (det B_q is a polynomial the rule integrates exactly); C annihilates constants;
and for c = 1 a linear field u gives (C u)_i = 0 at interior nodes (the integrand
grad phi_i . grad u |det B| reduces to the polynomial J_i^T adj(B) g, integrated exactly).
"""
import numpy as np
import pytest

import oracle
from workloads import boundary_mask, rule, structured_mesh

SHAPES = [(2, 2, 3), (2, 3, 2), (3, 2, 2), (3, 3, 1)]
CONST1 = ("const", 1.0)


def _curved(mesh, eps):
    """Every node moved by eps * prod_k sin(pi x_k) (zero on the boundary of the unit box)."""
    X = mesh["coords"].copy()
    bump = np.prod(np.sin(np.pi * X), axis=0)
    out = dict(mesh)
    out["coords"] = np.ascontiguousarray(X + eps * bump * np.array([1.0, -0.7, 0.5][:X.shape[0]])[:, None])
    return out


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_affine_positions_give_the_affine_matrices(dim, order, N):
    mesh = structured_mesh(dim, order, N, 0.2, seed=[101, dim, order])
    r = rule(dim, 2 * order)
    u = np.random.default_rng([102, dim]).uniform(-1, 1, size=mesh["coords"].shape[1])
    law_m, law_c = ("poly2", 1.0, 0.2, 0.0), ("exp", 0.0, 0.5)
    _, _, M1, C1 = oracle.assemble(mesh, r, r, law_m, law_c, u, u)
    _, _, M2, C2 = oracle.assemble_iso(mesh, r, r, law_m, law_c, u, u)
    assert np.abs(M1 - M2).max() <= 1e-13 * np.abs(M1).max()
    assert np.abs(C1 - C2).max() <= 1e-12 * np.abs(C1).max()


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_curved_mesh_area_constants_and_linear_fields(dim, order, N):
    mesh = _curved(structured_mesh(dim, order, N, 0.0), 0.08 / N)
    r = rule(dim, 2 * order)
    rp, ci, M, C = oracle.assemble_iso(mesh, r, r, CONST1, CONST1)
    _, _, Ma, _ = oracle.assemble(mesh, r, r, CONST1, CONST1)
    assert abs(M.sum() - 1.0) <= 1e-13
    assert np.abs(M - Ma).max() > 1e-6 * np.abs(M).max()      # the geometry is really curved
    n = mesh["coords"].shape[1]
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.abs(np.bincount(rows, weights=C, minlength=n)).max() <= 1e-13 * np.abs(C).max()
    g = np.array([0.3, -1.2, 0.7][:dim])
    u = g @ mesh["coords"]
    Cu = np.bincount(rows, weights=C * u[ci], minlength=n)
    interior = ~boundary_mask(mesh)
    assert np.abs(Cu[interior]).max() <= 1e-12 * np.abs(C).max()
