"""Pins of the oracle's volume load vector F_i = int f phi_i (Section 2).

For a nodal f with the identity law, f_h = sum_j f_j phi_j, so F = M f with the mass
matrix of the same rule (the oracle's mass assembly: an independent code path); a
constant f integrates the basis: sum_i F_i = f |Omega|; values per (q, e) reproduce the
nodal case when they are the interpolated values.
"""
import numpy as np
import pytest

import oracle
from workloads import rule, structured_mesh
from workloads.fields import gaussian_random_field

SHAPES = [(2, 1, 5), (2, 2, 3), (2, 3, 2), (3, 1, 2), (3, 2, 2), (3, 3, 1)]


def _dense(rp, ci, v, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return A


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_nodal_load_is_mass_times_values(dim, order, N):
    mesh = structured_mesh(dim, order, N, 0.2, seed=[61, dim, order])
    f = gaussian_random_field(mesh["coords"], 8, np.random.default_rng([62, dim]), length=0.3)
    r = rule(dim, 2 * order)
    F = oracle.load_vector(mesh, r, ("identity",), f)
    rp, ci, M, _ = oracle.assemble(mesh, r, r, ("const", 1.0), ("const", 1.0))
    Mf = _dense(rp, ci, M, f.size) @ f
    assert np.abs(F - Mf).max() <= 1e-13 * np.abs(Mf).max()


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_constant_load_integrates_the_basis(dim, order, N):
    mesh = structured_mesh(dim, order, N, 0.2, seed=[63, dim, order])
    F = oracle.load_vector(mesh, rule(dim, 2 * order), ("const", 2.5))
    assert abs(F.sum() - 2.5) <= 1e-13        # the unit square / cube


def test_qpoint_values_equal_interpolated_nodal():
    mesh = structured_mesh(3, 2, 2, 0.2, seed=64)
    f = gaussian_random_field(mesh["coords"], 8, np.random.default_rng(65), length=0.3)
    r = rule(3, 4)
    law = ("exp", 0.0, 0.5)
    F1 = oracle.load_vector(mesh, r, law, f)
    ne = mesh["conn"].shape[1]
    S = oracle.qpoint_coeff(mesh, np.arange(ne), r, ("identity",), f)   # [ne, nq]: u_h at the nodes
    F2 = oracle.load_vector(mesh, r, law, qpoint=np.ascontiguousarray(S.T))
    assert np.abs(F1 - F2).max() <= 1e-14 * np.abs(F1).max()
