"""Exact rational element integrals on simplices (test helper, pins the oracle).

Everything is kept as polynomials in barycentric coordinates lambda_0..lambda_d
with Fraction coefficients and integrated with the closed form
    int_T lambda^alpha dx = d! alpha! |T| / (|alpha| + d)!,
so element mass and conductivity matrices with polynomial coefficients are
exact rationals. The Lagrange basis uses the barycentric product formula
phi_i = prod_k prod_{j < alpha_ik} (P lambda_k - j) / (j + 1), which is
independent of the Vandermonde construction used by the oracle.
"""
from __future__ import annotations

import math
from fractions import Fraction

Poly = dict  # exponent tuple (len d+1) -> Fraction


def _add(p, q, s=1):
    out = dict(p)
    for k, v in q.items():
        out[k] = out.get(k, 0) + s * v
    return {k: v for k, v in out.items() if v != 0}


def _mul(p, q):
    out = {}
    for k1, v1 in p.items():
        for k2, v2 in q.items():
            k = tuple(a + b for a, b in zip(k1, k2))
            out[k] = out.get(k, 0) + v1 * v2
    return {k: v for k, v in out.items() if v != 0}


def _scale(p, s):
    return {k: v * s for k, v in p.items() if v * s != 0}


def _lam(k, d):
    e = [0] * (d + 1)
    e[k] = 1
    return {tuple(e): Fraction(1)}


def _const(c, d):
    return {tuple([0] * (d + 1)): Fraction(c)}


def _deriv(p, k):
    out = {}
    for e, v in p.items():
        if e[k] > 0:
            e2 = list(e)
            e2[k] -= 1
            out[tuple(e2)] = out.get(tuple(e2), 0) + v * e[k]
    return out


def lagrange_basis(alpha, P, d):
    """Barycentric-form Lagrange polynomials for multi-indices alpha [n_p][d+1]."""
    out = []
    for a in alpha:
        p = _const(1, d)
        for k in range(d + 1):
            for j in range(int(a[k])):
                f = _add(_scale(_lam(k, d), Fraction(P)), _const(-j, d))
                p = _mul(p, _scale(f, Fraction(1, j + 1)))
        out.append(p)
    return out


def integrate(p, vol, d):
    s = Fraction(0)
    for e, v in p.items():
        num = math.factorial(d)
        for a in e:
            num *= math.factorial(a)
        s += v * Fraction(num, math.factorial(sum(e) + d))
    return s * vol


def _inv(M):
    n = len(M)
    A = [[Fraction(x) for x in row] + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        pv = A[c][c]
        A[c] = [x / pv for x in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [row[n:] for row in A]


def _det(M):
    n = len(M)
    A = [[Fraction(x) for x in row] for row in M]
    det = Fraction(1)
    for c in range(n):
        piv = next((r for r in range(c, n) if A[r][c] != 0), None)
        if piv is None:
            return Fraction(0)
        if piv != c:
            A[c], A[piv] = A[piv], A[c]
            det = -det
        det *= A[c][c]
        for r in range(c + 1, n):
            f = A[r][c] / A[c][c]
            A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return det


def element_matrices_exact(verts, alpha, P, coeff_m, coeff_c):
    """Exact M_e, C_e for a simplex with rational vertices verts[d+1][d].

    coeff_m / coeff_c: polynomial coefficients given by their values at the
    vertices after mapping through a polynomial law: a callable taking the
    barycentric-polynomial of the linear field and returning the polynomial
    of the coefficient (e.g. lambda u: 1 + u*u).
    """
    d = len(verts) - 1
    verts = [[Fraction(x) for x in v] for v in verts]
    # x = x0 + sum_k lambda_k (x_k - x0): grad lambda_k (k>=1) = rows of B^{-T}
    B = [[verts[c + 1][r] - verts[0][r] for c in range(d)] for r in range(d)]
    det = _det(B)
    vol = abs(det) / math.factorial(d)
    Binv = _inv(B)  # row k of Binv = grad lambda_{k+1}
    grads = [[-sum(Binv[k][r] for k in range(d)) for r in range(d)]] + [list(Binv[k]) for k in range(d)]
    G = [[sum(grads[a][r] * grads[b][r] for r in range(d)) for b in range(d + 1)] for a in range(d + 1)]
    phis = lagrange_basis(alpha, P, d)
    dphis = [[_deriv(p, k) for k in range(d + 1)] for p in phis]
    n = len(phis)
    cm = coeff_m(d)
    cc = coeff_c(d)
    M = [[integrate(_mul(cm, _mul(phis[i], phis[j])), vol, d) for j in range(n)] for i in range(n)]
    Cm = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(i, n):
            acc = {}
            for a in range(d + 1):
                for b in range(d + 1):
                    if G[a][b] != 0:
                        acc = _add(acc, _scale(_mul(dphis[i][a], dphis[j][b]), G[a][b]))
            v = integrate(_mul(cc, acc), vol, d)
            Cm[i][j] = v
            Cm[j][i] = v
    return M, Cm


def linear_field_poly(vals_at_vertices, d):
    """Barycentric polynomial of a linear field from its vertex values."""
    p = {}
    for k in range(d + 1):
        p = _add(p, _scale(_lam(k, d), Fraction(vals_at_vertices[k])))
    return p


def poly_law(u, a0, a1, a2, d):
    return _add(_add(_const(a0, d), _scale(u, Fraction(a1))), _scale(_mul(u, u), Fraction(a2)))
