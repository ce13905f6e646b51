"""Pins of the oracle's conductivity tensor that varies per quadrature node (Section 7:
c_q a symmetric d x d tensor, A_qe = B^{-1} c_q B^{-T}), affine and isoparametric.

The contribution of node q to C_e is linear in c_q, so a tensor field
K_qe = alpha_qe K1 + beta_qe K2 must give the sum of two assemblies that are already
pinned on their own: per-(q, e) scalar values alpha (or beta) times the constant tensor
K1 (or K2). A wrong q or e index, a transposed triangle or a metric taken once per
element instead of per node breaks the equality, since alpha and beta vary per node."""
import numpy as np
import pytest

import oracle
from helpers import row_scaled_error
from workloads import rule, structured_mesh

SHAPES = [(2, 1, 5), (2, 2, 4), (2, 3, 3), (3, 1, 3), (3, 2, 2), (3, 3, 2)]


def _spd(dim, seed):
    S = np.eye(dim) + 0.5 * np.random.default_rng(seed).uniform(-1, 1, size=(dim, dim))
    K = S @ S.T
    return np.array([K[a, b] for a in range(dim) for b in range(a, dim)])


def _curved(mesh, eps):
    X = mesh["coords"].copy()
    bump = np.prod(np.sin(np.pi * X), axis=0)
    out = dict(mesh)
    out["coords"] = np.ascontiguousarray(X + eps * bump * np.array([1.0, -0.7, 0.5][:X.shape[0]])[:, None])
    return out


def _field(dim, nq, ne, seed):
    rng = np.random.default_rng(seed)
    K1, K2 = _spd(dim, [seed, 1]), _spd(dim, [seed, 2])
    al = rng.uniform(0.5, 2.0, size=(nq, ne))
    be = rng.uniform(0.5, 2.0, size=(nq, ne))
    Kq = al[:, None, :] * K1[None, :, None] + be[:, None, :] * K2[None, :, None]
    return K1, K2, al, be, np.ascontiguousarray(Kq)


@pytest.mark.parametrize("iso", [False, True])
@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_per_node_tensor_is_linear_in_the_tensor(dim, order, N, iso):
    mesh = structured_mesh(dim, order, N, 0.2, seed=[131, dim, order])
    if iso:
        mesh = _curved(mesh, 0.05 / N)
    fn = oracle.assemble_iso if iso else oracle.assemble
    r = rule(dim, 2 * order)
    ne = mesh["conn"].shape[1]
    K1, K2, al, be, Kq = _field(dim, r[1].size, ne, 132 + dim + order)
    law_m = ("poly2", 1.0, 0.2, 0.0)
    u = np.random.default_rng(133).uniform(-1, 1, size=mesh["coords"].shape[1])
    rp, _, M, C = fn(mesh, r, r, law_m, ("const", 1.0), u, None, tensor_q=Kq)
    _, _, M0, C1 = fn(mesh, r, r, law_m, ("identity",), u, None, qpoint_c=al, tensor_c=K1)
    _, _, _, C2 = fn(mesh, r, r, law_m, ("identity",), u, None, qpoint_c=be, tensor_c=K2)
    assert np.array_equal(M, M0)                                   # the mass matrix does not see it
    assert row_scaled_error(C, C1 + C2, rp) <= 1e-13
    # a constant field reproduces the constant-tensor path
    Kc = np.ascontiguousarray(np.broadcast_to(K1[None, :, None], Kq.shape))
    _, _, _, Cc = fn(mesh, r, r, law_m, ("const", 1.0), u, None, tensor_q=Kc)
    _, _, _, Ck = fn(mesh, r, r, law_m, ("const", 1.0), u, None, tensor_c=K1)
    assert row_scaled_error(Cc, Ck, rp) <= 1e-14


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_per_node_tensor_iso_on_affine_mesh_equals_affine(dim, order, N):
    mesh = structured_mesh(dim, order, N, 0.2, seed=[134, dim, order])
    r = rule(dim, 2 * order)
    Kq = _field(dim, r[1].size, mesh["conn"].shape[1], 135)[-1]
    law_c = ("exp", 0.0, 0.5)
    u = np.random.default_rng(136).uniform(-1, 1, size=mesh["coords"].shape[1])
    rp, _, _, C1 = oracle.assemble(mesh, r, r, ("const", 1.0), law_c, None, u, tensor_q=Kq)
    _, _, _, C2 = oracle.assemble_iso(mesh, r, r, ("const", 1.0), law_c, None, u, tensor_q=Kq)
    assert row_scaled_error(C1, C2, rp) <= 1e-12
