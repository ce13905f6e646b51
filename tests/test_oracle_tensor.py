"""Pins of the oracle's mass tensor-vector product (Section 5, the mass tensor
M_ijk = int m'(u_h) phi_i phi_j phi_k contracted with v in its second mode).

The oracle forms each element's full third-order tensor and contracts it; the
pins check it against the definition of the tensor as a derivative of the mass
matrix (an independent code path: the oracle's mass-matrix assembly), against
the partition of unity, and against its symmetry.
"""
import numpy as np
import pytest

import oracle
from workloads import rule, structured_mesh
from workloads.fields import gaussian_random_field

SHAPES = [(2, 1, 5), (2, 2, 3), (2, 3, 2), (3, 1, 2), (3, 2, 2), (3, 3, 1)]


def _fields(mesh, seed):
    rng = np.random.default_rng(seed)
    u = gaussian_random_field(mesh["coords"], 8, rng, length=0.4)
    v = gaussian_random_field(mesh["coords"], 8, rng, length=0.3)
    return u, v


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_derivative_of_the_mass_matrix(dim, order, N):
    """M_ijk = dM_ij/du_k: for m(u) = a0 + a1 u + a2 u^2 the mass matrix is quadratic in
    the nodal vector, so the central difference (M(u + t v) - M(u - t v)) / 2t equals
    the directional derivative, i.e. the tensor contracted with v, up to rounding."""
    mesh = structured_mesh(dim, order, N, 0.2, seed=[31, dim, order])
    u, v = _fields(mesh, [32, dim, order])
    r = rule(dim, 2 * order)   # any rule: both sides use the same quadrature
    a0, a1, a2 = 1.0, 0.3, 0.2
    law_m = ("poly2", a0, a1, a2)
    law_dm = ("poly2", a1, 2 * a2, 0.0)
    rp, ci, T = oracle.mass_tensor_product(mesh, r, law_dm, u, v)
    t = 0.5
    _, _, Mp, _ = oracle.assemble(mesh, r, r, law_m, ("const", 1.0), u + t * v, None)
    _, _, Mm, _ = oracle.assemble(mesh, r, r, law_m, ("const", 1.0), u - t * v, None)
    fd = (Mp - Mm) / (2 * t)
    assert _rel(T, fd) <= 1e-12


@pytest.mark.parametrize("dim,order,N", [(2, 2, 3), (3, 2, 2)])
def test_derivative_nonpolynomial_law(dim, order, N):
    """m = exp(u): the central difference converges to the tensor product at O(t^2)."""
    mesh = structured_mesh(dim, order, N, 0.2, seed=[33, dim, order])
    u, v = _fields(mesh, [34, dim, order])
    r = rule(dim, 2 * order)
    rp, ci, T = oracle.mass_tensor_product(mesh, r, ("exp", 0.0, 1.0), u, v)
    errs = []
    for t in (1e-2, 5e-3):
        _, _, Mp, _ = oracle.assemble(mesh, r, r, ("exp", 0.0, 1.0), ("const", 1.0), u + t * v, None)
        _, _, Mm, _ = oracle.assemble(mesh, r, r, ("exp", 0.0, 1.0), ("const", 1.0), u - t * v, None)
        errs.append(_rel(T, (Mp - Mm) / (2 * t)))
    assert errs[0] < 1e-4 and 3.0 < errs[0] / errs[1] < 5.0   # second order


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_unit_vector_gives_the_mass_matrix_of_m_prime(dim, order, N):
    """sum_j phi_j = 1, so contracting with the all-ones vector gives the mass matrix of m'."""
    mesh = structured_mesh(dim, order, N, 0.2, seed=[35, dim, order])
    u, _ = _fields(mesh, [36, dim, order])
    r = rule(dim, 2 * order)
    law_dm = ("exp", 0.1, 0.5)
    rp, ci, T = oracle.mass_tensor_product(mesh, r, law_dm, u, np.ones_like(u))
    _, _, M, _ = oracle.assemble(mesh, r, r, law_dm, ("const", 1.0), u, None)
    assert _rel(T, M) <= 1e-13


def test_symmetric_and_linear_in_v():
    mesh = structured_mesh(3, 2, 2, 0.2, seed=37)
    u, v = _fields(mesh, 38)
    w = np.random.default_rng(39).uniform(-1, 1, size=u.size)
    r = rule(3, 4)
    law = ("poly2", 0.5, 0.2, 0.1)
    rp, ci, T1 = oracle.mass_tensor_product(mesh, r, law, u, v)
    _, _, T2 = oracle.mass_tensor_product(mesh, r, law, u, w)
    _, _, T3 = oracle.mass_tensor_product(mesh, r, law, u, 2 * v - 3 * w)
    assert _rel(T3, 2 * T1 - 3 * T2) <= 1e-13
    n = u.size
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = T1[rp[i]:rp[i + 1]]
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
