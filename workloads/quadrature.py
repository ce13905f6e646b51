"""Symmetric quadrature rules on the reference simplex (input data).

The method takes the quadrature weights and nodes as inputs (Algorithm 1 and
Algorithm 2, "Input"), possibly one rule per matrix. The paper points to
Laursen and Gellert for the values but prints none, so the rules here are
defined by their symmetric orbit structure plus a starting guess, and every
parameter is polished by Gauss-Newton on the moment equations in 40-digit
arithmetic. A rule is correct iff it integrates every monomial up to its
degree exactly on the reference simplex (Section 3, step 4); the moment test
in the test suite is the pin.

Reference simplex: vertex 0 at the origin and vertex k at e_k, so weights sum
to |T| = 1/d! (the change of variables of Section 3 carries |det B_e|).
Points are returned in reference Cartesian coordinates x = (l_1, ..., l_d)
where l_k are barycentric coordinates and l_0 = 1 - sum(x).
"""
from __future__ import annotations

import functools
import itertools
import math

import mpmath
import numpy as np

# Orbit types, as barycentric tuples of length d+1 built from parameters.
def _orbit_points(kind, params, d):
    if d == 2:
        if kind == "S3":
            base = (mpmath.mpf(1) / 3,) * 3
        elif kind == "S21":
            a, = params
            base = (a, a, 1 - 2 * a)
        elif kind == "S111":
            a, b = params
            base = (a, b, 1 - a - b)
        else:
            raise ValueError(kind)
    else:
        if kind == "S4":
            base = (mpmath.mpf(1) / 4,) * 4
        elif kind == "S31":
            a, = params
            base = (a, a, a, 1 - 3 * a)
        elif kind == "S22":
            a, = params
            base = (a, a, mpmath.mpf(1) / 2 - a, mpmath.mpf(1) / 2 - a)
        elif kind == "S211":
            a, b = params
            base = (a, a, b, 1 - 2 * a - b)
        else:
            raise ValueError(kind)
    # distinct permutations in a fixed (lexicographic index) order
    seen = []
    keys = set()
    for perm in itertools.permutations(range(d + 1)):
        pt = tuple(base[p] for p in perm)
        key = tuple(mpmath.nstr(v, 25) for v in pt)
        if key not in keys:
            keys.add(key)
            seen.append(pt)
    return seen


# (dim, degree) -> list of (orbit kind, [initial params], initial weight per point)
# Weights are per point, for a simplex of measure 1/d!.
_SPECS = {
    (2, 1): [("S3", [], 0.5)],
    (2, 2): [("S21", [1 / 6], 1 / 6)],
    (2, 4): [("S21", [0.445948490915965], 0.223381589678011 / 2),
             ("S21", [0.091576213509771], 0.109951743655322 / 2)],
    (2, 6): [("S21", [0.249286745170910], 0.116786275726379 / 2),
             ("S21", [0.063089014491502], 0.050844906370207 / 2),
             ("S111", [0.053145049844817, 0.310352451033784], 0.082851075618374 / 2)],
    (3, 1): [("S4", [], 1 / 6)],
    (3, 2): [("S31", [0.1381966011250105], 1 / 24)],
    (3, 4): [("S4", [], -74 / 5625),
             ("S31", [1 / 14], 343 / 45000),
             ("S22", [0.399403576166799], 56 / 2250)],
    (3, 6): [("S31", [0.214602871259151684], 0.00665379170969464506),
             ("S31", [0.0406739585346113397], 0.00167953517588677620),
             ("S31", [0.322337890142275646], 0.00922619692394239843),
             ("S211", [0.0636610018750175299, 0.269672331458315867], 0.00803571428571428248)],
}


def _monomials(d, degree):
    out = []
    for total in range(degree + 1):
        for alpha in itertools.product(range(total + 1), repeat=d):
            if sum(alpha) == total:
                out.append(alpha)
    return out


def simplex_moment(alpha):
    """Exact integral of x^alpha over the reference d-simplex: alpha! / (|alpha|+d)!."""
    d = len(alpha)
    num = 1
    for a in alpha:
        num *= math.factorial(a)
    return mpmath.mpf(num) / math.factorial(sum(alpha) + d)


def _assemble(spec, unknowns, d):
    pts, wts = [], []
    pos = 0
    for kind, p0, _ in spec:
        npar = len(p0)
        params = unknowns[pos:pos + npar]
        w = unknowns[pos + npar]
        pos += npar + 1
        for bary in _orbit_points(kind, params, d):
            pts.append(bary[1:])
            wts.append(w)
    return pts, wts


@functools.lru_cache(maxsize=None)
def _solve(d, degree):
    spec = _SPECS[(d, degree)]
    mpmath.mp.dps = 40
    x = []
    for _, p0, w0 in spec:
        x.extend(mpmath.mpf(v) for v in p0)
        x.append(mpmath.mpf(w0))
    monos = _monomials(d, degree)
    target = [simplex_moment(a) for a in monos]

    def residual(xv):
        pts, wts = _assemble(spec, xv, d)
        r = []
        for a, t in zip(monos, target):
            s = mpmath.mpf(0)
            for p, w in zip(pts, wts):
                term = w
                for k in range(d):
                    term *= p[k] ** a[k]
                s += term
            r.append(s - t)
        return r

    for _ in range(60):
        r = residual(x)
        if max(abs(v) for v in r) < mpmath.mpf(10) ** -36:
            break
        n = len(x)
        jac = mpmath.matrix(len(r), n)
        h = mpmath.mpf(10) ** -20
        for j in range(n):
            xp = list(x)
            xp[j] += h
            rp = residual(xp)
            for i in range(len(r)):
                jac[i, j] = (rp[i] - r[i]) / h
        # least-squares Gauss-Newton step via normal equations
        jt = jac.T
        step = mpmath.lu_solve(jt * jac, jt * mpmath.matrix(r))
        x = [x[j] - step[j] for j in range(n)]
    r = residual(x)
    if max(abs(v) for v in r) > mpmath.mpf(10) ** -30:
        raise RuntimeError(f"quadrature rule d={d} degree={degree} did not converge")
    pts, wts = _assemble(spec, x, d)
    P = np.array([[float(v) for v in p] for p in pts], dtype=np.float64).reshape(len(pts), d)
    W = np.array([float(w) for w in wts], dtype=np.float64)
    mpmath.mp.dps = 15
    return P, W


def rule(dim: int, degree: int):
    """Return (points [n_q, dim], weights [n_q]) of the rule of the given exact degree."""
    key = (dim, degree)
    if key not in _SPECS:
        # fall back to the next available higher degree
        cands = sorted(dg for (dd, dg) in _SPECS if dd == dim and dg >= degree)
        if not cands:
            raise ValueError(f"no rule of degree {degree} in {dim}D")
        key = (dim, cands[0])
    P, W = _solve(*key)
    return P.copy(), W.copy()


def rule_degree(dim: int, degree: int) -> int:
    """Actual exact degree of the rule returned by rule(dim, degree)."""
    cands = sorted(dg for (dd, dg) in _SPECS if dd == dim and dg >= degree)
    return cands[0]


def available(dim: int):
    return sorted(dg for (dd, dg) in _SPECS if dd == dim)


# Rules of sizes other than the built-in ones (inputs that the library pads to
# a compiled rule size): two classical closed-form rules and a conical product.

def radon7():
    """Radon's 7-node rule of degree 5 on the triangle: the centroid and two
    S21 orbits with a = (6 -+ sqrt 15) / 21 (weights 9/80 and (155 -+ sqrt 15) / 2400,
    summing to the area 1/2)."""
    s = math.sqrt(15.0)
    pts, wts = [(1.0 / 3.0, 1.0 / 3.0)], [9.0 / 80.0]
    for a, w in (((6.0 - s) / 21.0, (155.0 - s) / 2400.0), ((6.0 + s) / 21.0, (155.0 + s) / 2400.0)):
        for p in ((a, a), (1.0 - 2.0 * a, a), (a, 1.0 - 2.0 * a)):
            pts.append(p)
            wts.append(w)
    return np.array(pts), np.array(wts)


def keast5():
    """The 5-node rule of degree 3 on the tetrahedron: the centroid with weight
    -2/15 and the S31 orbit with l = (1/2, 1/6, 1/6, 1/6), weight 3/40 each (a
    negative weight; the total is the volume 1/6)."""
    pts, wts = [(0.25, 0.25, 0.25)], [-2.0 / 15.0]
    for k in range(4):
        l = [1.0 / 6.0] * 4
        l[k] = 0.5
        pts.append(tuple(l[1:]))
        wts.append(3.0 / 40.0)
    return np.array(pts), np.array(wts)


def conical(dim: int, n: int):
    """Conical product rule with n Gauss-Legendre nodes per axis (n^dim nodes):
    the square or cube mapped onto the simplex by collapsing one side at a time,
    x = u, y = v (1 - u) (, z = t (1 - u)(1 - v)), with the Jacobian (1 - u) (1 - u)^2 (1 - v)
    in the weights; exact up to degree 2n - 2 in 2D and 2n - 3 in 3D."""
    g, gw = np.polynomial.legendre.leggauss(n)
    g, gw = (g + 1.0) / 2.0, gw / 2.0
    pts, wts = [], []
    for idx in itertools.product(range(n), repeat=dim):
        u = [g[i] for i in idx]
        w = float(np.prod([gw[i] for i in idx]))
        if dim == 2:
            pts.append((u[0], u[1] * (1.0 - u[0])))
            wts.append(w * (1.0 - u[0]))
        else:
            pts.append((u[0], u[1] * (1.0 - u[0]), u[2] * (1.0 - u[0]) * (1.0 - u[1])))
            wts.append(w * (1.0 - u[0]) ** 2 * (1.0 - u[1]))
    return np.array(pts), np.array(wts)
