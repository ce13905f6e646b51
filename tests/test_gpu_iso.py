"""Isoparametric (curved) elements (Section 7) on the GPU: the per-node geometry path
against the oracle on curved meshes of every shape, with nodal, per-quadrature-node and
anisotropic coefficients, the lower-degree stiffness rule, the affine special case,
symmetry, and the degenerate-map report."""
import numpy as np
import pytest

import oracle
from helpers import row_scaled_error, transpose_slots
from workloads import rule, structured_mesh
from workloads.fields import gaussian_random_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(2, 1, 23), (2, 2, 13), (2, 3, 9), (3, 1, 7), (3, 2, 5), (3, 3, 3)]


def _curved(mesh, eps):
    """Every node moved by eps * prod_k sin(pi x_k) (zero on the boundary of the unit box)."""
    X = mesh["coords"].copy()
    bump = np.prod(np.sin(np.pi * X), axis=0)
    out = dict(mesh)
    out["coords"] = np.ascontiguousarray(X + eps * bump * np.array([1.0, -0.7, 0.5][:X.shape[0]])[:, None])
    return out


def _K(dim, seed):
    S = np.eye(dim) + 0.4 * np.random.default_rng(seed).uniform(-1, 1, size=(dim, dim))
    K = S @ S.T
    return np.array([K[a, b] for a in range(dim) for b in range(a, dim)])


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_iso_nodal_fields_against_oracle(dim, order, N):
    import paper_2204_03893_amd as qxa
    print("case iso nodal", dim, order, N, flush=True)
    mesh = _curved(structured_mesh(dim, order, N, 0.1, seed=[111, dim, order]), 0.1 / N)
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([112, dim]), length=0.3)
    r = rule(dim, 2 * order)
    law_m, law_c = ("poly2", 1.0, 0.1, 0.2), ("exp", 0.0, 1.0)
    K = _K(dim, [113, dim]) if order != 1 else None
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    M, Cv = qxa.assemble_iso(plan, law_m, law_c, uf, uf, tensor=K)
    M2, C2 = qxa.assemble_iso(plan, law_m, law_c, uf, uf, tensor=K)   # second call: no allocation, same bits
    qxa.sync(plan)
    rpo, cio, Mo, Co = oracle.assemble_iso(mesh, r, r, law_m, law_c, u, u, tensor_c=K)
    Mg, Cg = M.cpu().numpy(), Cv.cpu().numpy()
    assert row_scaled_error(Mg, Mo, rpo) <= 1e-12
    assert row_scaled_error(Cg, Co, rpo) <= 1e-12
    assert torch.equal(M, M2) and torch.equal(Cv, C2)
    tr = transpose_slots(rpo, cio)
    assert np.array_equal(Mg, Mg[tr]) and np.array_equal(Cg, Cg[tr])


@pytest.mark.parametrize("dim,order", [(2, 2), (3, 2), (2, 3)])
def test_iso_qpoint_field_and_lower_degree_rule(dim, order):
    import paper_2204_03893_amd as qxa
    print("case iso qpoint", dim, order, flush=True)
    mesh = _curved(structured_mesh(dim, order, 4, 0.1, seed=[114, dim, order]), 0.03)
    rm, rc = rule(dim, 2 * order), rule(dim, 2 * order - 2)
    ne = mesh["conn"].shape[1]
    s = np.random.default_rng(115).uniform(0.5, 2.0, size=(len(rm[1]), ne))
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rm, rc)
    M, Cv = qxa.assemble_iso(plan, ("poly2", 0.0, 1.0, 0.0), ("const", 1.7), torch.tensor(s, device="cuda"), None,
                             qpoint=True)
    qxa.sync(plan)
    rpo, _, Mo, Co = oracle.assemble_iso(mesh, rm, rc, ("poly2", 0.0, 1.0, 0.0), ("const", 1.7), qpoint_m=s)
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= 1e-12
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= 1e-12


def test_iso_affine_mesh_matches_the_fused_assembly():
    import paper_2204_03893_amd as qxa
    dim, order = 3, 2
    mesh = structured_mesh(dim, order, 4, 0.2, seed=116)
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng(117), length=0.3)
    r = rule(dim, 2 * order)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    law_m, law_c = ("poly2", 1.0, 0.3, 0.0), ("exp", 0.0, 0.5)
    Mi, Ci = qxa.assemble_iso(plan, law_m, law_c, uf, uf)
    Mf, Cf = qxa.assemble(plan, law_m, law_c, uf, uf)
    qxa.sync(plan)
    rp = np.asarray(oracle.pattern(mesh)[0])
    assert row_scaled_error(Mi.cpu().numpy(), Mf.cpu().numpy(), rp) <= 1e-12
    assert row_scaled_error(Ci.cpu().numpy(), Cf.cpu().numpy(), rp) <= 1e-12
    Mo, _ = qxa.assemble_iso(plan, law_m, law_c, uf, uf, want_c=False)   # one output only
    _, Co = qxa.assemble_iso(plan, law_m, law_c, uf, uf, want_m=False)
    qxa.sync(plan)
    assert torch.equal(Mo, Mi) and torch.equal(Co, Ci)


def test_iso_nonfinite_coefficient_is_reported():
    import paper_2204_03893_amd as qxa
    dim, order = 2, 2
    mesh = _curved(structured_mesh(dim, order, 3, 0.0), 0.02)
    u = np.ones(mesh["coords"].shape[1])
    u[mesh["conn"][3, 4]] = np.nan
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rule(dim, 2 * order))
    qxa.assemble_iso(plan, ("const", 1.0), ("poly2", 1.0, 1.0, 0.0), None, torch.tensor(u, device="cuda"))
    with pytest.raises(qxa.QxaError) as ei:
        qxa.sync(plan)
    assert ei.value.code == -4                       # QXA_E_NONFINITE
    qxa.assemble_iso(plan, ("const", 1.0), ("const", 1.0))   # the report is cleared by qxa_sync
    qxa.sync(plan)


def _Kq(dim, nq, ne, seed):
    rng = np.random.default_rng(seed)
    ng = dim * (dim + 1) // 2
    S = np.eye(dim)[None, None] + 0.3 * rng.uniform(-1, 1, size=(nq, ne, dim, dim))
    K = np.einsum("qeab,qecb->qeac", S, S)                       # SPD per (q, e)
    iu = np.triu_indices(dim)
    return np.ascontiguousarray(K[:, :, iu[0], iu[1]].transpose(0, 2, 1)).reshape(nq, ng, ne)


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_iso_per_node_tensor_against_oracle(dim, order, N):
    import paper_2204_03893_amd as qxa
    print("case iso per-node tensor", dim, order, N, flush=True)
    base = structured_mesh(dim, order, N, 0.1, seed=[121, dim, order])
    r = rule(dim, 2 * order)
    ne = base["conn"].shape[1]
    Kq = _Kq(dim, r[1].size, ne, [122, dim, order])
    u = gaussian_random_field(base["coords"], 16, np.random.default_rng([123, dim]), length=0.3)
    law_c = ("exp", 0.0, 0.5)
    Kd = torch.tensor(Kq, device="cuda")
    uf = torch.tensor(u, device="cuda")
    for curved in (False, True):
        mesh = _curved(base, 0.1 / N) if curved else base
        m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
        plan = qxa.Plan(m, r)
        M, Cv = qxa.assemble_iso(plan, ("const", 1.0), law_c, None, uf, tensor_q=Kd)
        qxa.sync(plan)
        fn = oracle.assemble_iso if curved else oracle.assemble    # straight sides: the affine oracle
        rpo, cio, Mo, Co = fn(mesh, r, r, ("const", 1.0), law_c, None, u, tensor_q=Kq)
        assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= 1e-12
        Cg = Cv.cpu().numpy()
        assert row_scaled_error(Cg, Co, rpo) <= 1e-12
        tr = transpose_slots(rpo, cio)
        assert np.array_equal(Cg, Cg[tr])


def test_per_node_tensor_errors():
    import paper_2204_03893_amd as qxa
    dim, order = 2, 2
    mesh = structured_mesh(dim, order, 3, 0.0)
    r = rule(dim, 2 * order)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    Kd = torch.tensor(_Kq(dim, r[1].size, mesh["conn"].shape[1], 124), device="cuda")
    with pytest.raises(qxa.QxaError) as ei:                       # the fused path does not take it
        cc, k = qxa.make_coeff(("const", 1.0), tensor_q=Kd)
        qxa.check(qxa.lib().qxa_assemble(plan.handle, None, qxa.C.byref(cc), 0, None, None, None))
    assert ei.value.code == -6
    with pytest.raises(qxa.QxaError) as ei:                       # constant and per-node tensor together
        qxa.assemble_iso(plan, ("const", 1.0), ("const", 1.0), tensor=np.array([1.0, 0.0, 1.0]), tensor_q=Kd)
    assert ei.value.code == -1
    with pytest.raises(qxa.QxaError) as ei:                       # not on the mass coefficient
        cm, k = qxa.make_coeff(("const", 1.0), tensor_q=Kd)
        M = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
        qxa.check(qxa.lib().qxa_assemble_iso(plan.handle, qxa.C.byref(cm), None, M.data_ptr(), None, None))
    assert ei.value.code == -1
    Kn = Kd.clone()
    Kn[0, 0, 2] = float("nan")
    qxa.assemble_iso(plan, ("const", 1.0), ("const", 1.0), tensor_q=Kn)
    with pytest.raises(qxa.QxaError) as ei:                       # a non-finite entry is reported
        qxa.sync(plan)
    assert ei.value.code == -4


@pytest.mark.parametrize("dim,order,N,one_pass", [(2, 2, 13, True), (3, 2, 5, True), (2, 3, 9, True),
                                                  (3, 3, 3, False), (3, 1, 7, False), (2, 1, 23, False)])
def test_iso_path_choice(dim, order, N, one_pass):
    """One pass (the matrix-core kernel forming X per quadrature node) where the shape's
    kernel stages Q^T in LDS, one rule serves both matrices and the reference gradients fit
    beside the plan's carry entries (2D P2, 2D P3, 3D P2); two passes otherwise (3D P3: Q^T
    read from global memory; P1: the vector-ALU kernel; different mass and stiffness rules,
    test_iso_qpoint_field_and_lower_degree_rule). Either way the result meets the oracle at
    1e-12."""
    import paper_2204_03893_amd as qxa
    print("case iso path", dim, order, N, flush=True)
    mesh = _curved(structured_mesh(dim, order, N, 0.15, seed=[120, dim, order]), 0.02)
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng(121), length=0.3)
    r = rule(dim, 2 * order)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    law_m, law_c = ("poly2", 1.0, 0.3, 0.0), ("exp", 0.0, 0.5)
    plan.set_timing(True)
    M, Cv = qxa.assemble_iso(plan, law_m, law_c, uf, uf)
    qxa.sync(plan)
    rep = plan.timing_report()
    plan.set_timing(False)
    assert ("fused_iso" in rep) == one_pass and ("iso_rows" in rep) == (not one_pass), rep
    rpo, _, Mo, Co = oracle.assemble_iso(mesh, r, r, law_m, law_c, u, u)
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= 1e-12
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= 1e-12


@pytest.mark.parametrize("dim,order,N", [(2, 2, 11), (3, 2, 4), (2, 3, 7)])
def test_iso_one_pass_qpoint_and_second_field(dim, order, N):
    """The one-pass isoparametric kernel with a per-(q, e) mass coefficient, then with
    different nodal fields for the mass and the conductivity (the second one read through
    the element's connectivity), against the oracle at 1e-12."""
    import paper_2204_03893_amd as qxa
    print("case iso one pass qpoint / second field", dim, order, N, flush=True)
    mesh = _curved(structured_mesh(dim, order, N, 0.1, seed=[140, dim, order]), 0.03)
    r = rule(dim, 2 * order)
    ne = mesh["conn"].shape[1]
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    s = np.random.default_rng(141).uniform(0.5, 2.0, size=(len(r[1]), ne))
    plan.set_timing(True)
    M, Cv = qxa.assemble_iso(plan, ("poly2", 0.0, 1.0, 0.0), ("const", 1.7), torch.tensor(s, device="cuda"), None,
                             qpoint=True)
    qxa.sync(plan)
    rep = plan.timing_report()
    plan.set_timing(False)
    assert "fused_iso" in rep, rep
    rpo, _, Mo, Co = oracle.assemble_iso(mesh, r, r, ("poly2", 0.0, 1.0, 0.0), ("const", 1.7), qpoint_m=s)
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= 1e-12
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= 1e-12
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng(142), length=0.3)
    v = gaussian_random_field(mesh["coords"], 16, np.random.default_rng(143), length=0.2)
    law_m, law_c = ("poly2", 1.0, 0.3, 0.0), ("exp", 0.0, 0.5)
    M2, C2 = qxa.assemble_iso(plan, law_m, law_c, torch.tensor(u, device="cuda"), torch.tensor(v, device="cuda"))
    qxa.sync(plan)
    rpo, _, Mo2, Co2 = oracle.assemble_iso(mesh, r, r, law_m, law_c, u, v)
    assert row_scaled_error(M2.cpu().numpy(), Mo2, rpo) <= 1e-12
    assert row_scaled_error(C2.cpu().numpy(), Co2, rpo) <= 1e-12
