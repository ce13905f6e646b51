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


# ---- conductivity tensor C_ijk = int c'(u_h) grad phi_i . grad phi_j phi_k, second mode ----

def _dense(rp, ci, vals, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = vals[rp[i]:rp[i + 1]]
    return A


@pytest.mark.parametrize("dim,order,N", [(2, 1, 3), (2, 2, 2), (2, 3, 1), (3, 1, 1), (3, 2, 1)])
def test_cond_tensor_is_the_jacobian_of_C_u_times_u(dim, order, N):
    """d/du_k (C(u) u)_i = sum_j C_ijk u_j + C_ik(u): with c quadratic, C(u) u is cubic in u,
    so the Richardson-extrapolated central difference of the oracle's own conductivity
    assembly is exact up to rounding."""
    mesh = structured_mesh(dim, order, N, 0.2, seed=[51, dim, order])
    u, _ = _fields(mesh, [52, dim, order])
    n = u.size
    r = rule(dim, 2 * order)
    a0, a1, a2 = 1.0, 0.4, 0.3
    law_c, law_dc = ("poly2", a0, a1, a2), ("poly2", a1, 2 * a2, 0.0)
    rp, ci, T = oracle.cond_tensor_product(mesh, r, law_dc, u, u)
    _, _, _, C0 = oracle.assemble(mesh, r, r, ("const", 1.0), law_c, None, u)

    def g(x):
        _, _, _, Cx = oracle.assemble(mesh, r, r, ("const", 1.0), law_c, None, x)
        return _dense(rp, ci, Cx, n) @ x

    J = np.zeros((n, n))
    t = 1e-2
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        d1 = (g(u + t * e) - g(u - t * e)) / (2 * t)
        d2 = (g(u + t / 2 * e) - g(u - t / 2 * e)) / t
        J[:, k] = (4 * d2 - d1) / 3
    want = J - _dense(rp, ci, C0, n)
    got = _dense(rp, ci, T, n)
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    assert np.abs(got - got.T).max() > 1e-6 * np.abs(got).max()      # not symmetric in general


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_cond_tensor_column_sums_vanish_and_constants(dim, order, N):
    """sum_i grad phi_i = 0, so every column of C o_2 v sums to zero; a constant v has no gradient."""
    mesh = structured_mesh(dim, order, N, 0.2, seed=[53, dim, order])
    u, v = _fields(mesh, [54, dim, order])
    r = rule(dim, 2 * order)
    law = ("exp", 0.0, 0.7)
    rp, ci, T = oracle.cond_tensor_product(mesh, r, law, u, v)
    n = u.size
    A = _dense(rp, ci, T, n)
    assert np.abs(A.sum(axis=0)).max() <= 1e-12 * np.abs(A).max()
    _, _, T1 = oracle.cond_tensor_product(mesh, r, law, u, np.full(n, 2.5))
    assert np.abs(T1).max() <= 1e-12 * np.abs(T).max()
    w = np.random.default_rng(55).uniform(-1, 1, size=n)
    _, _, T2 = oracle.cond_tensor_product(mesh, r, law, u, w)
    _, _, T3 = oracle.cond_tensor_product(mesh, r, law, u, v - 2 * w)
    assert _rel(T3, T - 2 * T2) <= 1e-13
