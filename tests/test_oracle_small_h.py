"""Pins of the oracle's contraction forms on one small element far from the origin.

Two sums of the oracle are written with differences to vertex 0 instead of absolute
values; the reference gradients sum to zero, so both forms are equal in exact
arithmetic:
- the conductivity tensor product (Section 5) contracts the local tensor with
  v_j - v_0;
- the isoparametric geometry (Section 7; Section 3 builds B_e from a_k - a_0)
  sums B_q from x_i - x_0.

On an element of size about 3e-3 at (1000, 2000[, 3000]), with v a large constant
plus a small linear variation, the oracle is compared with exact rational values
(tests/exact_fem.py: barycentric polynomials with Fraction coefficients, no
quadrature). Every input is a dyadic rational, so the float64 inputs are exact and
the element is exactly straight-sided. The same quadrature sums evaluated in the
plain form (absolute coordinates, sum_j v_j grad phi_j; written out below in float64
with the oracle's basis values) lose about log10(|x| / h) or log10(|v| / (h |grad v|))
digits; the oracle's forms do not.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_fem import _add, _deriv, _det, _inv, _mul, _scale, element_matrices_exact, integrate, \
    lagrange_basis, linear_field_poly, poly_law
from workloads import rule
from workloads.mesh import local_alpha

# (dim, order, rule degree): the rule integrates every integrand below exactly
CASES = [(2, 3, 6), (3, 2, 4)]
ORIGIN = {2: (1000, 2000), 3: (1000, 2000, 3000)}


def _element(dim, order):
    """Vertices and node positions (Fractions) of a straight-sided element of size ~3e-3:
    vertex offsets are multiples of order/1024, so every node is a dyadic rational."""
    o = [Fraction(c) for c in ORIGIN[dim]]
    step = Fraction(order, 1024)
    if dim == 2:
        offs = [(0, 0), (1, 0), (Fraction(1, 2), 1)]
    else:
        offs = [(0, 0, 0), (1, 0, 0), (Fraction(1, 2), 1, 0), (Fraction(1, 2), Fraction(1, 2), 1)]
    verts = [[o[r] + step * Fraction(off[r]) for r in range(dim)] for off in offs]
    alpha = local_alpha(dim, order)
    nodes = [[sum(Fraction(int(a[k]), order) * verts[k][r] for k in range(dim + 1)) for r in range(dim)]
             for a in alpha]
    return verts, alpha, nodes


def _mesh(dim, order, nodes):
    X = np.array([[float(c) for c in x] for x in nodes])
    assert all(Fraction(float(c)) == c for x in nodes for c in x)  # exact in float64
    n = X.shape[0]
    return {"dim": dim, "order": order, "coords": np.ascontiguousarray(X.T),
            "conn": np.arange(n, dtype=np.int32).reshape(n, 1), "n_nodes": n, "n_elem": 1, "n_p": n}


def _linear_nodal(nodes, x0, c, g):
    """Nodal values of c + g . (x - x0) (exact Fractions)."""
    return [c + sum(g[r] * (x[r] - x0[r]) for r in range(len(g))) for x in nodes]


def _dense(rp, ci, vals, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = vals[rp[i]:rp[i + 1]]
    return A


def _rowerr(got, ref):
    return float(np.max(np.abs(got - ref) / np.abs(ref).max(axis=1, keepdims=True)))


def _tensor_exact(verts, alpha, order, u_vert, a, g):
    """T_ik = int c'(u) phi_k grad phi_i . g over the element, c'(u) = a0 + a1 u, u linear
    with vertex values u_vert, v linear with gradient g (exact rationals)."""
    d = len(verts) - 1
    B = [[verts[c + 1][r] - verts[0][r] for c in range(d)] for r in range(d)]
    vol = abs(_det(B)) / (2 if d == 2 else 6)
    Binv = _inv(B)
    grads = [[-sum(Binv[k][r] for k in range(d)) for r in range(d)]] + [list(Binv[k]) for k in range(d)]
    gl = [sum(grads[k][r] * g[r] for r in range(d)) for k in range(d + 1)]  # grad lambda_k . g
    phis = lagrange_basis(alpha, order, d)
    cdash = poly_law(linear_field_poly(u_vert, d), a[0], a[1], 0, d)
    n = len(phis)
    T = np.zeros((n, n))
    for i in range(n):
        gi = {}
        for k in range(d + 1):
            gi = _add(gi, _scale(_deriv(phis[i], k), gl[k]))
        cg = _mul(cdash, gi)
        for kk in range(n):
            T[i, kk] = float(integrate(_mul(cg, phis[kk]), vol, d))
    return T


@pytest.mark.parametrize("dim,order,deg", CASES)
def test_cond_tensor_product_small_element(dim, order, deg):
    verts, alpha, nodes = _element(dim, order)
    mesh = _mesh(dim, order, nodes)
    x0 = verts[0]
    gu = [Fraction(2), Fraction(1)] + ([Fraction(-1)] if dim == 3 else [])
    gv = [Fraction(1), Fraction(1, 2)] + ([Fraction(3, 4)] if dim == 3 else [])
    u = _linear_nodal(nodes, x0, Fraction(1, 4), gu)
    v = _linear_nodal(nodes, x0, Fraction(1000), gv)        # |v| / (h |grad v|) ~ 3e5
    uf = np.array([float(t) for t in u])
    vf = np.array([float(t) for t in v])
    assert all(Fraction(float(t)) == t for t in u + v)
    a = (Fraction(1), Fraction(1, 2))                        # c'(u) = 1 + u/2
    u_vert = [u[k] for k in range(dim + 1)]
    Tx = _tensor_exact(verts, alpha, order, u_vert, a, gv)
    r = rule(dim, deg)
    rp, ci, Tv = oracle.cond_tensor_product(mesh, r, ("poly2", 1.0, 0.5, 0.0), uf, vf)
    n = len(nodes)
    To = _dense(rp, ci, Tv, n)
    err_oracle = _rowerr(To, Tx)

    # the same quadrature sum with the plain contraction sum_j v_j grad phi_j
    pts, w = r
    phi, dphi = oracle.basis(dim, order, pts)
    X = mesh["coords"]
    B = X[:, 1:dim + 1] - X[:, [0]]
    Binv = np.linalg.inv(B)
    adet = abs(np.linalg.det(B))
    Tp = np.zeros((n, n))
    for q in range(w.size):
        G = dphi[q] @ Binv                                  # physical gradients [n, d]
        uh = phi[q] @ uf
        gvh = vf @ G                                        # sum_j v_j grad phi_j
        Tp += w[q] * (1.0 + 0.5 * uh) * adet * np.outer(G @ gvh, phi[q])
    err_plain = _rowerr(Tp, Tx)
    print(f"d={dim} P={order}: oracle (v_j - v_0) {err_oracle:.2e}, plain sum_j v_j grad phi_j {err_plain:.2e}")
    assert err_oracle <= 1e-13
    assert err_plain >= 100 * err_oracle and err_plain >= 1e-12


@pytest.mark.parametrize("dim,order,deg", CASES)
def test_isoparametric_small_element(dim, order, deg):
    verts, alpha, nodes = _element(dim, order)
    mesh = _mesh(dim, order, nodes)
    one = lambda d: {tuple([0] * (d + 1)): Fraction(1)}
    Mx, Cx = element_matrices_exact(verts, alpha, order, one, one)
    Mx = np.array([[float(t) for t in row] for row in Mx])
    Cx = np.array([[float(t) for t in row] for row in Cx])
    r = rule(dim, deg)
    rp, ci, Mv, Cv = oracle.assemble_iso(mesh, r, r, ("const", 1.0), ("const", 1.0))
    n = len(nodes)
    em, ec = _rowerr(_dense(rp, ci, Mv, n), Mx), _rowerr(_dense(rp, ci, Cv, n), Cx)

    # the same quadrature sums with B_q = sum_i x_i grad phi_i(xhat_q)^T from absolute coordinates
    pts, w = r
    phi, dphi = oracle.basis(dim, order, pts)
    X = mesh["coords"]
    Mp = np.zeros((n, n))
    Cp = np.zeros((n, n))
    for q in range(w.size):
        Bq = X @ dphi[q]
        adet = abs(np.linalg.det(Bq))
        G = dphi[q] @ np.linalg.inv(Bq)
        Mp += w[q] * adet * np.outer(phi[q], phi[q])
        Cp += w[q] * adet * (G @ G.T)
    pm, pc = _rowerr(Mp, Mx), _rowerr(Cp, Cx)
    print(f"d={dim} P={order}: oracle (x_i - x_0) mass {em:.2e} cond {ec:.2e}; absolute coordinates "
          f"mass {pm:.2e} cond {pc:.2e}")
    assert em <= 1e-13 and ec <= 1e-13
    assert max(pm, pc) >= 100 * max(em, ec) and max(pm, pc) >= 1e-12
