"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses a closed form,
an exact rational computation, a brute-force construction in physical
coordinates, or an invariant of the exact matrices.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_fem import element_matrices_exact, linear_field_poly, poly_law
from workloads import boundary_mask, nnz_closed_form, rule, structured_mesh
from workloads.mesh import local_alpha

CONST1 = ("const", 1.0)


def _csr_dense(rp, ci, v, n):
    A = np.zeros((n, n))
    for r in range(n):
        A[r, ci[rp[r]:rp[r + 1]]] = v[rp[r]:rp[r + 1]]
    return A


def _one_element_mesh(verts, order):
    """A single simplex with its P-order nodes at affine positions."""
    verts = np.asarray(verts, dtype=np.float64)
    d = verts.shape[1]
    al = local_alpha(d, order).astype(np.float64) / order
    X = al @ verts  # [n_p, d]
    n = X.shape[0]
    return {"dim": d, "order": order, "coords": np.ascontiguousarray(X.T),
            "conn": np.arange(n, dtype=np.int32).reshape(n, 1), "n_nodes": n, "n_elem": 1, "n_p": n}


def _vol(verts):
    verts = np.asarray(verts, float)
    d = verts.shape[1]
    return abs(np.linalg.det((verts[1:] - verts[0]).T)) / math.factorial(d)


# ---------------------------------------------------------------- basis
@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_basis_invariants(dim, order):
    rng = np.random.default_rng(0)
    x = rng.dirichlet(np.ones(dim + 1), size=17)[:, 1:]
    phi, dphi = oracle.basis(dim, order, x)
    assert np.abs(phi.sum(1) - 1).max() < 1e-13          # partition of unity
    assert np.abs(dphi.sum(1)).max() < 1e-12             # sum of gradients vanishes
    # Lagrange property at the local nodes (which are the mesh format's nodes)
    xn = local_alpha(dim, order)[:, 1:] / order
    assert np.allclose(oracle.local_nodes(dim, order), xn, atol=0)
    phin, _ = oracle.basis(dim, order, xn)
    assert np.abs(phin - np.eye(xn.shape[0])).max() < 1e-12


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_basis_reproduces_polynomials(dim, order):
    """Interpolating a degree-P polynomial through the nodes reproduces it and its gradient."""
    rng = np.random.default_rng(1)
    x = rng.dirichlet(np.ones(dim + 1), size=9)[:, 1:]
    xn = local_alpha(dim, order)[:, 1:] / order
    coef = rng.normal(size=(dim + 1,))
    f = lambda y: (coef[0] + y @ coef[1:]) ** order
    g = lambda y: order * (coef[0] + y @ coef[1:])[:, None] ** (order - 1) * coef[1:][None, :]
    phi, dphi = oracle.basis(dim, order, x)
    assert np.abs(phi @ f(xn) - f(x)).max() < 1e-12
    assert np.abs(np.einsum("qnd,n->qd", dphi, f(xn)) - g(x)).max() < 1e-11


# ---------------------------------------------------------------- P1 closed forms
def test_p1_mass_closed_form():
    """P1 mass: |T|/((d+1)(d+2)) (1 + delta_ij) for a degree-2 rule."""
    rng = np.random.default_rng(2)
    for d in (2, 3):
        for _ in range(5):
            verts = rng.normal(size=(d + 1, d))
            m = _one_element_mesh(verts, 1)
            Me, Ce = oracle.element_matrices(m, [0], rule(d, 2), rule(d, 2), CONST1, CONST1)
            ref = _vol(verts) / ((d + 1) * (d + 2)) * (1 + np.eye(d + 1))
            assert np.abs(Me[0] - ref).max() <= 1e-14 * np.abs(ref).max()


def test_p1_stiffness_cotangent_2d():
    """2D P1 conductivity: off-diagonal entry (i,j) equals -cot(theta_k)/2."""
    rng = np.random.default_rng(3)
    for _ in range(8):
        verts = rng.normal(size=(3, 2))
        m = _one_element_mesh(verts, 1)
        _, Ce = oracle.element_matrices(m, [0], rule(2, 1), rule(2, 1), CONST1, CONST1)
        ref = np.zeros((3, 3))
        for i, j in [(0, 1), (1, 2), (0, 2)]:
            k = 3 - i - j
            u, v = verts[i] - verts[k], verts[j] - verts[k]
            cot = (u @ v) / abs(u[0] * v[1] - u[1] * v[0])
            ref[i, j] = ref[j, i] = -0.5 * cot
        for i in range(3):
            ref[i, i] = -ref[i].sum()
        assert np.abs(Ce[0] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_p1_stiffness_face_normals_3d():
    """3D P1 conductivity: C_ij = A_i A_j n_i.n_j / (9|T|) with face areas/normals."""
    rng = np.random.default_rng(4)
    for _ in range(8):
        verts = rng.normal(size=(4, 3))
        vol = _vol(verts)
        an = []
        for i in range(4):
            f = [k for k in range(4) if k != i]
            nrm = 0.5 * np.cross(verts[f[1]] - verts[f[0]], verts[f[2]] - verts[f[0]])
            if nrm @ (verts[i] - verts[f[0]]) > 0:   # make it outward (away from vertex i)
                nrm = -nrm
            an.append(nrm)
        an = np.array(an)
        ref = an @ an.T / (9 * vol)
        m = _one_element_mesh(verts, 1)
        _, Ce = oracle.element_matrices(m, [0], rule(3, 1), rule(3, 1), CONST1, CONST1)
        assert np.abs(Ce[0] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_p1_unit_right_triangles():
    """The two triangles of an unjittered cell have the textbook local matrices."""
    h = 1.0 / 64
    T1 = [(0, 0), (h, 0), (h, h)]
    T2 = [(0, 0), (h, h), (0, h)]
    ref1 = np.array([[0.5, -0.5, 0], [-0.5, 1, -0.5], [0, -0.5, 0.5]])
    ref2 = np.array([[0.5, 0, -0.5], [0, 0.5, -0.5], [-0.5, -0.5, 1]])
    for T, ref in [(T1, ref1), (T2, ref2)]:
        Me, Ce = oracle.element_matrices(_one_element_mesh(T, 1), [0], rule(2, 2), rule(2, 2), CONST1, CONST1)
        assert np.abs(Ce[0] - ref).max() < 1e-14
        assert np.abs(Me[0] - h * h / 24 * (1 + np.eye(3))).max() < 1e-19


# ---------------------------------------------------------------- global closed forms on the 64x64 mesh
def test_p1_64_interior_stencils():
    """Interior rows of the 64x64 P1 matrices: 5-point Laplacian (exact zeros on the diagonal
    neighbours) and mass h^2/2 on the diagonal, h^2/12 on the 6 neighbours."""
    N = 64
    h = 1.0 / N
    m = structured_mesh(2, 1, N)
    rp, ci, M, Cv = oracle.assemble(m, rule(2, 2), rule(2, 2), CONST1, CONST1)
    assert rp[-1] == nnz_closed_form(2, 1, N)
    L = N + 1
    bnd = boundary_mask(m)
    for r in np.nonzero(~bnd)[0][::37]:
        cols = ci[rp[r]:rp[r + 1]]
        mv = M[rp[r]:rp[r + 1]]
        cv = Cv[rp[r]:rp[r + 1]]
        expect_c = {r: 4.0, r - 1: -1.0, r + 1: -1.0, r - L: -1.0, r + L: -1.0, r - L - 1: 0.0, r + L + 1: 0.0}
        assert sorted(expect_c) == list(cols)
        for c, v, w in zip(cols, cv, mv):
            assert abs(v - expect_c[c]) < 1e-15
            assert abs(w - (h * h / 2 if c == r else h * h / 12)) <= 2e-16 * h * h
        assert np.all(cv[[list(cols).index(r - L - 1), list(cols).index(r + L + 1)]] == 0.0)


# ---------------------------------------------------------------- invariants on jittered meshes
CASES = [(2, 1, 6, 2), (2, 2, 4, 4), (2, 3, 3, 6), (3, 1, 3, 2), (3, 2, 2, 4), (3, 3, 2, 6)]


@pytest.mark.parametrize("dim,order,N,deg", CASES)
def test_mass_total_and_row_sums(dim, order, N, deg):
    m = structured_mesh(dim, order, N, 0.2, seed=11)
    rng = np.random.default_rng(5)
    u = rng.normal(size=m["n_nodes"])
    r = rule(dim, deg)
    rp, ci, M, Cv = oracle.assemble(m, r, r, CONST1, ("poly2", 1.0, 0.3, 0.5), None, u)
    assert abs(M.sum() - 1.0) < 1e-13                    # 1^T M 1 = |Omega|
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    rs = np.bincount(rows, weights=Cv)
    rmax = np.maximum.reduceat(np.abs(Cv), rp[:-1])
    assert np.all(np.abs(rs) <= 1e-13 * rmax)            # C 1 = 0 for any coefficient


@pytest.mark.parametrize("dim,order,N,deg", CASES)
def test_stiffness_kills_linear_fields_at_interior_nodes(dim, order, N, deg):
    m = structured_mesh(dim, order, N, 0.2, seed=12)
    r = rule(dim, deg)
    rp, ci, M, Cv = oracle.assemble(m, r, r, CONST1, ("const", 2.5))
    n = m["n_nodes"]
    A = _csr_dense(rp, ci, Cv, n)
    ell = 0.3 + m["coords"].T @ np.arange(1, dim + 1)
    res = A @ ell
    inner = ~boundary_mask(m)
    assert np.abs(res[inner]).max() < 1e-12 * np.abs(A).max()
    assert np.abs(res[~inner]).max() > 1e-6              # not trivially zero


@pytest.mark.parametrize("dim,order,N,deg", CASES)
def test_symmetry(dim, order, N, deg):
    m = structured_mesh(dim, order, N, 0.2, seed=13)
    u = np.sin(3 * m["coords"][0]) + m["coords"][1]
    r = rule(dim, deg)
    rp, ci, M, Cv = oracle.assemble(m, r, r, ("poly2", 1.0, 0.1, 0.0), ("exp", 0.0, 1.0), u, u)
    n = m["n_nodes"]
    for V in (M, Cv):
        A = _csr_dense(rp, ci, V, n)
        assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()


def _phys_qpoints(m, pts):
    X, c = m["coords"], m["conn"]
    d = m["dim"]
    a0 = X[:, c[0]]                                          # [d, ne]
    B = np.stack([X[:, c[k]] - a0 for k in range(1, d + 1)], axis=1)   # [d, d, ne]
    xq = a0[:, None, :] + np.einsum("rce,qc->rqe", B, pts)             # [d, nq, ne]
    det = np.abs(np.linalg.det(np.moveaxis(B, 2, 0)))
    return xq, det


@pytest.mark.parametrize("dim,order,N,deg", CASES)
def test_basis_free_quadrature_identities(dim, order, N, deg):
    """p^T M q and p^T C q for polynomials p, q of degree <= P equal the quadrature of
    m p q and c grad p . grad q at physical quadrature points; the coefficient is a law
    applied to a degree-P polynomial field (reproduced exactly by u_h)."""
    m = structured_mesh(dim, order, N, 0.2, seed=14)
    X = m["coords"]
    rng = np.random.default_rng(6)
    a, b, g = rng.normal(size=(3, dim + 1))
    lin = lambda Y, cf: cf[0] + np.tensordot(cf[1:], Y, axes=(0, 0))
    p = lambda Y: lin(Y, a) ** order
    q = lambda Y: lin(Y, b) ** max(order - 1, 1) * lin(Y, g) if order > 1 else lin(Y, b)
    f = lambda Y: 0.4 * lin(Y, g) ** order                     # field of degree P

    def grad(fun, Y, eps=1e-6):
        out = []
        for k in range(dim):
            Yp = Y.copy(); Yp[k] += eps
            Ym = Y.copy(); Ym[k] -= eps
            out.append((fun(Yp) - fun(Ym)) / (2 * eps))
        return np.array(out)

    lawm = ("poly2", 1.0, 0.2, 0.1)
    lawc = ("exp", 0.1, 0.5)
    r = rule(dim, deg)
    rp, ci, M, Cv = oracle.assemble(m, r, r, lawm, lawc, f(X), f(X))
    n = m["n_nodes"]
    Am, Ac = _csr_dense(rp, ci, M, n), _csr_dense(rp, ci, Cv, n)
    xq, det = _phys_qpoints(m, r[0])
    fq = f(xq)
    mq = 1.0 + 0.2 * fq + 0.1 * fq * fq
    cq = np.exp(0.1 + 0.5 * fq)
    w = r[1][:, None]
    refM = np.sum(w * mq * p(xq) * q(xq) * det[None, :])
    refC = np.sum(w * cq * np.sum(grad(p, xq) * grad(q, xq), axis=0) * det[None, :])
    assert abs(p(X) @ Am @ q(X) - refM) <= 1e-12 * abs(refM)
    assert abs(p(X) @ Ac @ q(X) - refC) <= 1e-8 * abs(refC)   # central differences in the reference


# ---------------------------------------------------------------- exact rationals and brute force
@pytest.mark.parametrize("dim,order,law_deg", [(2, 1, 2), (2, 2, 2), (2, 3, 0), (3, 1, 2), (3, 2, 2), (3, 3, 0)])
def test_exact_rational_element_matrices(dim, order, law_deg):
    """Polynomial coefficients with a rule of sufficient degree give exact rationals."""
    rng = np.random.default_rng(7)
    verts = [[Fraction(int(v), 8) for v in rng.integers(-8, 9, size=dim)] for _ in range(dim + 1)]
    while _vol(np.array(verts, float)) < 0.05:
        verts = [[Fraction(int(v), 8) for v in rng.integers(-8, 9, size=dim)] for _ in range(dim + 1)]
    uv = [Fraction(int(v), 4) for v in rng.integers(-4, 5, size=dim + 1)]
    a = (Fraction(1), Fraction(1, 2), Fraction(1, 4)) if law_deg == 2 else (Fraction(3, 2), 0, 0)
    cm = lambda d: poly_law(linear_field_poly(uv, d), a[0], a[1], a[2], d)
    cc = lambda d: poly_law(linear_field_poly(uv, d), a[0], a[2], a[1], d)
    alpha = local_alpha(dim, order)
    Mx, Cx = element_matrices_exact(verts, alpha, order, cm, cc)
    deg = min(6, 2 * order + law_deg)
    mesh = _one_element_mesh(np.array(verts, float), order)
    # nodal field: the linear field at every local node
    al = alpha.astype(float) / order
    u_nodes = al @ np.array(uv, float)
    lm = ("poly2", float(a[0]), float(a[1]), float(a[2]))
    lc = ("poly2", float(a[0]), float(a[2]), float(a[1]))
    Me, Ce = oracle.element_matrices(mesh, [0], rule(dim, deg), rule(dim, deg), lm, lc, u_nodes, u_nodes)
    Mx = np.array([[float(v) for v in row] for row in Mx])
    Cx = np.array([[float(v) for v in row] for row in Cx])
    assert np.abs(Me[0] - Mx).max() <= 1e-14 * np.abs(Mx).max()
    assert np.abs(Ce[0] - Cx).max() <= 1e-13 * np.abs(Cx).max()


def _physical_brute_force(verts, order, pts, w, mfun, cfun):
    """Element matrices with the Lagrange basis built in physical coordinates (no map)."""
    verts = np.asarray(verts, float)
    d = verts.shape[1]
    al = local_alpha(d, order).astype(float) / order
    Xn = al @ verts
    expo = [e for t in range(order + 1) for e in itertools.product(range(t + 1), repeat=d) if sum(e) == t]
    V = np.array([[np.prod(x ** np.array(e)) for e in expo] for x in Xn])
    Cf = np.linalg.solve(V, np.eye(len(expo)))
    B = (verts[1:] - verts[0]).T
    det = abs(np.linalg.det(B))
    n = Xn.shape[0]
    M = np.zeros((n, n))
    Cm = np.zeros((n, n))
    for xh, wq in zip(pts, w):
        x = verts[0] + B @ xh
        mono = np.array([np.prod(x ** np.array(e)) for e in expo])
        dmono = np.zeros((len(expo), d))
        for k, e in enumerate(expo):
            for a in range(d):
                if e[a]:
                    e2 = list(e); e2[a] -= 1
                    dmono[k, a] = e[a] * np.prod(x ** np.array(e2))
        phi = Cf.T @ mono
        dphi = Cf.T @ dmono
        M += wq * mfun(x) * np.outer(phi, phi) * det
        Cm += wq * cfun(x) * (dphi @ dphi.T) * det
    return M, Cm


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_brute_force_physical_basis(dim, order):
    """Small meshes: element matrices from a basis built in physical coordinates."""
    m = structured_mesh(dim, order, 1, 0.0)
    rng = np.random.default_rng(8)
    m["coords"] = m["coords"] + 0.05 * rng.normal(size=m["coords"].shape)
    # keep straight-sided elements: recompute non-vertex nodes of element 0 only, test element 0
    al = local_alpha(dim, order).astype(float) / order
    c0 = m["conn"][:, 0]
    verts = m["coords"][:, c0[:dim + 1]].T
    m["coords"][:, c0] = (al @ verts).T
    r = rule(dim, 4 if dim == 3 else 6)
    # coefficient: a law of a degree-P polynomial field f(x) = (0.5 + x . g)^P
    gvec = np.arange(1, dim + 1) * 0.3
    f = lambda x: (0.5 + x @ gvec) ** order
    Me, Ce = oracle.element_matrices(m, [0], r, r, ("poly2", 1.0, 0.5, 0.0), ("exp", 0.0, 1.0),
                                     f(m["coords"].T), f(m["coords"].T))
    Mb, Cb = _physical_brute_force(verts, order, r[0], r[1], lambda x: 1.0 + 0.5 * f(x), lambda x: np.exp(f(x)))
    assert np.abs(Me[0] - Mb).max() <= 1e-12 * np.abs(Mb).max()
    assert np.abs(Ce[0] - Cb).max() <= 1e-10 * np.abs(Cb).max()


# ---------------------------------------------------------------- invariances
def test_translation_scaling_relabelling():
    for dim, order in [(2, 2), (3, 1)]:
        m = structured_mesh(dim, order, 2, 0.2, seed=15)
        r = rule(dim, 4)
        base = oracle.assemble(m, r, r, CONST1, CONST1)
        m2 = dict(m)
        m2["coords"] = m["coords"] + 3.7
        t = oracle.assemble(m2, r, r, CONST1, CONST1)
        assert np.abs(t[2] - base[2]).max() < 1e-13 * np.abs(base[2]).max()
        assert np.abs(t[3] - base[3]).max() < 1e-11 * np.abs(base[3]).max()
        s = 2.5
        m3 = dict(m)
        m3["coords"] = m["coords"] * s
        sc = oracle.assemble(m3, r, r, CONST1, CONST1)
        assert np.abs(sc[2] - s ** dim * base[2]).max() < 1e-13 * s ** dim * np.abs(base[2]).max()
        assert np.abs(sc[3] - s ** (dim - 2) * base[3]).max() < 1e-12 * np.abs(base[3]).max() * s ** (dim - 2)
        # relabel nodes by a permutation sigma: new id = sigma[old id]
        n = m["n_nodes"]
        sigma = np.random.default_rng(9).permutation(n)
        m4 = dict(m)
        m4["conn"] = sigma[m["conn"]].astype(np.int32)
        X4 = np.empty_like(m["coords"])
        X4[:, sigma] = m["coords"]
        m4["coords"] = X4
        rl = oracle.assemble(m4, r, r, CONST1, CONST1)
        A = _csr_dense(*base[:2], base[3], n)
        B = _csr_dense(*rl[:2], rl[3], n)
        assert np.abs(B[np.ix_(sigma, sigma)] - A).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("dim,order,N", [(2, 1, 5), (2, 2, 4), (2, 3, 3), (3, 1, 3), (3, 2, 2), (3, 3, 2)])
def test_pattern_closed_form(dim, order, N):
    m = structured_mesh(dim, order, N)
    rp, ci = oracle.pattern(m)
    assert rp[-1] == nnz_closed_form(dim, order, N)
    assert np.all(np.diff(rp) > 0)
    for r in range(rp.size - 1):
        seg = ci[rp[r]:rp[r + 1]]
        assert np.all(np.diff(seg) > 0) and r in seg


def test_rows_match_full_assembly():
    m = structured_mesh(3, 2, 2, 0.2, seed=16)
    r = rule(3, 4)
    u = np.cos(m["coords"].sum(0))
    rp, ci, M, Cv = oracle.assemble(m, r, r, CONST1, ("poly2", 1, 0, 0.5), None, u)
    rows = np.array([0, 7, 100, m["n_nodes"] - 1])
    sp, sc, sM, sC = oracle.assemble_rows(m, rows, r, r, CONST1, ("poly2", 1, 0, 0.5), None, u)
    for k, rr in enumerate(rows):
        assert np.array_equal(sc[sp[k]:sp[k + 1]], ci[rp[rr]:rp[rr + 1]])
        assert np.array_equal(sM[sp[k]:sp[k + 1]], M[rp[rr]:rp[rr + 1]])
        assert np.array_equal(sC[sp[k]:sp[k + 1]], Cv[rp[rr]:rp[rr + 1]])


def test_degenerate_element_rejected():
    m = _one_element_mesh([[0, 0], [1, 0], [2, 0]], 1)
    with pytest.raises(ValueError):
        oracle.assemble(m, rule(2, 2), rule(2, 2), CONST1, CONST1)


# ---------------------------------------------------------------- planted mistakes are caught
def _quick_pins():
    """A compact subset of the pins above; returns the list of failures."""
    fails = []
    try:
        test_p1_mass_closed_form()
    except AssertionError:
        fails.append("p1 mass")
    try:
        test_p1_stiffness_face_normals_3d()
    except AssertionError:
        fails.append("p1 stiffness 3d")
    try:
        test_basis_free_quadrature_identities(2, 2, 3, 4)
    except AssertionError:
        fails.append("basis-free")
    try:
        test_mass_total_and_row_sums(3, 2, 2, 4)
    except AssertionError:
        fails.append("totals")
    return fails


def test_pins_pass_on_the_oracle():
    assert _quick_pins() == []


@pytest.mark.parametrize("fault", [1, 2, 3, 4, 5, 6])
def test_planted_mistakes_fail_a_pin(fault):
    """Dropped |det B|, transposed inverse product, a gradient sign, a shifted weight index,
    a dropped coefficient, phi_i^2 instead of phi_i phi_j: each must break some pin."""
    with oracle.planted_fault(fault):
        assert _quick_pins() != []
