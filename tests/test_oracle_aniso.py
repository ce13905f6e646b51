"""Pins of the oracle's anisotropic conductivity (Section 7: A_qe = B_e^{-1} c_q B_e^{-T},
here c_q = c(u_h) K with a constant symmetric K).

Change of variables: on the mesh Y = S^{-1} X, the isotropic conductivity matrix equals
|det S|^{-1} times the anisotropic one on X with K = S S^T (grad_y = S^T grad_x,
dy = |det S|^{-1} dx), for any invertible S; K = s I scales the isotropic matrix by s.
"""
import numpy as np
import pytest

import oracle
from workloads import rule, structured_mesh

SHAPES = [(2, 1, 4), (2, 2, 3), (2, 3, 2), (3, 1, 2), (3, 2, 2), (3, 3, 1)]


def _upper(K):
    d = K.shape[0]
    return np.array([K[a, b] for a in range(d) for b in range(a, d)])


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_anisotropic_equals_isotropic_on_mapped_mesh(dim, order, N):
    mesh = structured_mesh(dim, order, N, 0.2, seed=[81, dim, order])
    rng = np.random.default_rng([82, dim])
    S = np.eye(dim) + 0.4 * rng.uniform(-1, 1, size=(dim, dim))
    K = S @ S.T
    r = rule(dim, 2 * order)
    u = rng.uniform(-1, 1, size=mesh["coords"].shape[1])
    law = ("poly2", 1.0, 0.2, 0.3)
    _, _, _, Ca = oracle.assemble(mesh, r, r, ("const", 1.0), law, None, u, tensor_c=_upper(K))
    mapped = dict(mesh)
    mapped["coords"] = np.ascontiguousarray(np.linalg.solve(S, mesh["coords"]))
    _, _, _, Ci = oracle.assemble(mapped, r, r, ("const", 1.0), law, None, u)
    assert np.abs(Ca - abs(np.linalg.det(S)) * Ci).max() <= 1e-12 * np.abs(Ca).max()


def test_scaled_identity_and_tensor_product_consistency():
    mesh = structured_mesh(3, 2, 2, 0.2, seed=83)
    r = rule(3, 4)
    u = np.random.default_rng(84).uniform(-1, 1, size=mesh["coords"].shape[1])
    law = ("exp", 0.0, 0.5)
    _, _, _, C1 = oracle.assemble(mesh, r, r, ("const", 1.0), law, None, u)
    _, _, _, C3 = oracle.assemble(mesh, r, r, ("const", 1.0), law, None, u, tensor_c=[3.0, 0, 0, 3.0, 0, 3.0])
    assert np.abs(C3 - 3 * C1).max() <= 1e-13 * np.abs(C3).max()
    # the conductivity tensor product honours K the same way: K = 2 I doubles it
    v = np.random.default_rng(85).uniform(-1, 1, size=u.size)
    _, _, T1 = oracle.cond_tensor_product(mesh, r, law, u, v)
    _, _, T2 = oracle.cond_tensor_product(mesh, r, law, u, v, tensor=[2.0, 0, 0, 2.0, 0, 2.0])
    assert np.abs(T2 - 2 * T1).max() <= 1e-13 * np.abs(T2).max()
