"""Input generators: quadrature exactness, mesh counts, the paper's size table."""
import math
import os

import numpy as np
import pytest

from workloads import boundary_mask, nnz_closed_form, rule, simplex_moment, structured_mesh
from workloads.quadrature import _monomials, available


@pytest.mark.parametrize("dim", [2, 3])
def test_quadrature_moments_exact(dim):
    """Each rule integrates every monomial up to its degree exactly (Section 3, step 4)."""
    for deg in available(dim):
        P, W = rule(dim, deg)
        assert abs(W.sum() - 1.0 / math.factorial(dim)) < 1e-16
        for a in _monomials(dim, deg):
            s = float(np.sum(W * np.prod(P ** np.array(a), axis=1)))
            assert abs(s - float(simplex_moment(a))) < 1e-16, (dim, deg, a)
        # points inside the simplex
        assert np.all(P > 0) and np.all(P.sum(1) < 1)


def test_quadrature_degree_is_sharp():
    """A degree-k rule is generally not exact at degree k+1 (guards against a wrong label)."""
    for dim in (2, 3):
        for deg in available(dim):
            P, W = rule(dim, deg)
            errs = [abs(float(np.sum(W * np.prod(P ** np.array(a), axis=1))) - float(simplex_moment(a)))
                    for a in _monomials(dim, deg + 1) if sum(a) == deg + 1]
            assert max(errs) > 1e-12, (dim, deg)


@pytest.mark.parametrize("dim,order,N", [(2, 1, 7), (2, 2, 5), (2, 3, 4), (3, 1, 3), (3, 2, 3), (3, 3, 2)])
def test_mesh_counts_and_measure(dim, order, N):
    m = structured_mesh(dim, order, N, jitter=0.2, seed=5)
    assert m["n_nodes"] == (order * N + 1) ** dim
    assert m["n_elem"] == (2 * N * N if dim == 2 else 6 * N ** 3)
    X, c = m["coords"], m["conn"]
    B = np.stack([X[:, c[k]] - X[:, c[0]] for k in range(1, dim + 1)], axis=1)
    det = np.linalg.det(np.moveaxis(B, 2, 0))
    assert abs(np.abs(det).sum() / math.factorial(dim) - 1.0) < 1e-13
    # every node is referenced, every element has distinct nodes
    assert np.unique(c).size == m["n_nodes"]
    s = np.sort(c, axis=0)
    assert np.all(s[1:] != s[:-1])
    # non-vertex nodes sit at their affine positions
    from workloads.mesh import local_alpha
    al = local_alpha(dim, order).astype(float) / order
    xn = np.einsum("pk,ckE->cpE", al, np.stack([X[:, c[k]] for k in range(dim + 1)], axis=1))
    assert np.allclose(xn, X[:, c], atol=1e-14)


def test_nnz_closed_forms_by_enumeration():
    for dim, order, N in [(2, 1, 6), (2, 2, 5), (2, 3, 4), (3, 1, 4), (3, 2, 3), (3, 3, 2)]:
        m = structured_mesh(dim, order, N)
        c = m["conn"].astype(np.int64)
        n = m["n_nodes"]
        I = np.repeat(c, c.shape[0], axis=0).reshape(-1)
        J = np.tile(c, (c.shape[0], 1)).reshape(-1)
        assert np.unique(I * n + J).size == nnz_closed_form(dim, order, N)


def test_paper_dof_table_consistency():
    """Pins the P2 node-count convention against the paper's printed sizes.

    For a triangulation of a square, Euler gives n_P2 = V + E = 4V - V_b - 3,
    so every row of the paper's table implies an integer number of boundary
    vertices V_b close to the perimeter/h = 4/h. Our generator satisfies the
    same identity exactly with V_b = 4N.
    """
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_mesh_sizes.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for h, n1, n2 in rows:
        h, n1, n2 = float(h), int(n1), int(n2)
        vb = 4 * n1 - 3 - n2
        assert vb > 0
        assert abs(vb - 4.0 / h) / (4.0 / h) < 0.01
    for N in (3, 8, 17):
        m1 = structured_mesh(2, 1, N)
        m2 = structured_mesh(2, 2, N)
        vb = int(boundary_mask(m1).sum())
        assert vb == 4 * N
        assert m2["n_nodes"] == 4 * m1["n_nodes"] - vb - 3


def test_jitter_is_seeded_and_keeps_boundary():
    a = structured_mesh(2, 2, 6, 0.25, seed=3)
    b = structured_mesh(2, 2, 6, 0.25, seed=3)
    assert np.array_equal(a["coords"], b["coords"])
    bm = boundary_mask(a)
    ref = structured_mesh(2, 2, 6, 0.0)
    assert np.allclose(a["coords"][:, bm], ref["coords"][:, bm], rtol=0, atol=1e-15)
