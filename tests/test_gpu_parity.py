"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Bar: CSR pattern bit-exact; FP64 values within 1e-12 row-scaled relative
error; bitwise run-to-run determinism; bitwise symmetry. Reduced-precision
forms are reported against the oracle with their own stated bound.
"""
import sys

import numpy as np
import pytest

import oracle
from helpers import FORM_BOUNDS, row_scaled_error, transpose_slots
from workloads import WORKLOADS, make_inputs, rule, scaled, structured_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _qxa():
    import paper_2204_03893_amd as qxa
    return qxa


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(w, precision="fp64", reps=1, stream_id=0):
    qxa = _qxa()
    mesh, r, u = make_inputs(w, stream_id)
    m = qxa.Mesh(w.dim, w.order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    outs = []
    for _ in range(reps):
        M, Cv = qxa.assemble(plan, w.mass_law, w.stiff_law, uf, uf, precision=precision)
        qxa.sync(plan)
        outs.append((M.cpu().numpy(), Cv.cpu().numpy()))
    rp, ci = plan.pattern()
    return mesh, r, u, plan, rp.cpu().numpy(), ci.cpu().numpy(), outs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_3d_p3_run_chains_against_oracle(precision):
    """3D P3 on a mesh with enough tiles for the run layout (one chain of 4-tile runs per
    workgroup, carries between a run's tiles): against the oracle, run-to-run bitwise,
    bitwise symmetric."""
    qxa = _qxa()
    from workloads.fields import gaussian_random_field
    dim, order, N = 3, 3, 14
    _say("case 3D P3 runs", N, precision)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[9, dim, order])
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([10, dim, order]), length=0.3)
    r = rule(dim, 2 * order)
    law_m, law_c = ("poly2", 1.0, 0.1, 0.0), ("exp", 0.0, 1.0)
    plan = qxa.Plan(qxa.Mesh(dim, order, mesh["coords"], mesh["conn"]), r)
    assert plan.n_chains == 256 and plan.n_carry_reads > 0
    uf = torch.tensor(u, device="cuda")
    M, Cv = qxa.assemble(plan, law_m, law_c, uf, uf, precision=precision)
    M2, C2 = qxa.assemble(plan, law_m, law_c, uf, uf, precision=precision)
    qxa.sync(plan)
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, law_m, law_c, u, u)
    tol = 1e-12 if precision == "fp64" else FORM_BOUNDS["fp32"]
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= tol
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= tol
    assert torch.equal(M.view(torch.int64), M2.view(torch.int64))
    assert torch.equal(Cv.view(torch.int64), C2.view(torch.int64))
    t = transpose_slots(rpo, cio)
    Mh, Ch = M.cpu().numpy(), Cv.cpu().numpy()
    assert np.array_equal(Mh, Mh[t]) and np.array_equal(Ch, Ch[t])


SMALL = [("p1_2d_64", None), ("p2_3d_32", 6), ("p3_2d_1024", 24), ("p1_3d_96_heat", 10)]


# every (dim, order) shape of the fused kernels, degree-2P rule for both
# matrices, variable coefficients; meshes spanning several tiles plus a ragged tail
SHAPES = [(2, 1, 23), (2, 2, 13), (2, 3, 9), (3, 1, 7), (3, 2, 5), (3, 3, 3)]


@pytest.mark.parametrize("dim,order,N", SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_all_shapes_against_oracle(dim, order, N, precision):
    qxa = _qxa()
    from workloads.fields import gaussian_random_field
    _say("case", dim, order, N, precision)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[7, dim, order])
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([8, dim, order]), length=0.3)
    r = rule(dim, 2 * order)
    law_m, law_c = ("poly2", 1.0, 0.1, 0.0), ("exp", 0.0, 1.0)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    M, Cv = qxa.assemble(plan, law_m, law_c, uf, uf, precision=precision)
    M2, C2 = qxa.assemble(plan, law_m, law_c, uf, uf, precision=precision)
    qxa.sync(plan)
    rp, ci = plan.pattern()
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, law_m, law_c, u, u)
    assert np.array_equal(rp.cpu().numpy(), rpo) and np.array_equal(ci.cpu().numpy(), cio)
    tol = 1e-12 if precision == "fp64" else FORM_BOUNDS["fp32"]
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= tol
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= tol
    assert torch.equal(M.view(torch.int64), M2.view(torch.int64))   # run-to-run bitwise
    assert torch.equal(Cv.view(torch.int64), C2.view(torch.int64))
    t = transpose_slots(rpo, cio)
    Mh, Ch = M.cpu().numpy(), Cv.cpu().numpy()
    assert np.array_equal(Mh, Mh[t]) and np.array_equal(Ch, Ch[t])  # bitwise symmetric
    assert plan.n_tiles > 1


@pytest.mark.parametrize("name,N", SMALL)
def test_fp64_parity_against_oracle(name, N):
    w = WORKLOADS[name] if N is None else scaled(name, N)
    _say("case", w.name)
    mesh, r, u, plan, rp, ci, outs = _run(w, reps=3)
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, w.mass_law, w.stiff_law, u, u)
    assert np.array_equal(rp, rpo) and np.array_equal(ci, cio)
    M, Cv = outs[0]
    assert row_scaled_error(M, Mo, rpo) <= 1e-12
    assert row_scaled_error(Cv, Co, rpo) <= 1e-12
    for M2, C2 in outs[1:]:                      # bitwise deterministic
        assert np.array_equal(M2.view(np.uint64), M.view(np.uint64))
        assert np.array_equal(C2.view(np.uint64), Cv.view(np.uint64))
    t = transpose_slots(rp, ci)                  # bitwise symmetric
    assert np.array_equal(M[t], M) and np.array_equal(Cv[t], Cv)


def test_fp64_parity_full_p2_3d_32():
    """The benchmark workload at full size, every value compared."""
    w = WORKLOADS["p2_3d_32"]
    _say("case", w.name, "full")
    mesh, r, u, plan, rp, ci, outs = _run(w)
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, w.mass_law, w.stiff_law, u, u)
    assert np.array_equal(rp, rpo) and np.array_equal(ci, cio)
    assert row_scaled_error(outs[0][0], Mo, rpo) <= 1e-12
    assert row_scaled_error(outs[0][1], Co, rpo) <= 1e-12


@pytest.mark.parametrize("name,N", [("p2_3d_32", 6), ("p1_3d_96_heat", 8)])
def test_fp32_contraction_error(name, N):
    w = scaled(name, N)
    _say("case", w.name, "fp32")
    mesh, r, u, plan, rp, ci, outs = _run(w, precision="fp32", reps=2)
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, w.mass_law, w.stiff_law, u, u)
    em = row_scaled_error(outs[0][0], Mo, rpo)
    ec = row_scaled_error(outs[0][1], Co, rpo)
    _say("fp32 row-scaled error", em, ec)
    assert em <= 1e-6 and ec <= 1e-6
    assert np.array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("dim,order,deg", [(2, 1, 2), (2, 2, 4), (2, 3, 6), (3, 1, 2), (3, 2, 4), (3, 3, 6)])
def test_element_matrices_formation(dim, order, deg):
    """Formation only (element matrices of Algorithm 2, no global assembly) against the oracle's local matrices, all orders."""
    qxa = _qxa()
    _say("case formation", dim, order)
    mesh = structured_mesh(dim, order, 3 if dim == 2 else 2, 0.2, seed=4)
    r = rule(dim, deg)
    u = np.sin(3 * mesh["coords"][0]) + 0.5 * mesh["coords"][1]
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    lm, lc = ("poly2", 1.0, 0.1, 0.0), ("exp", 0.0, 1.0)
    Vm, Vc = qxa.element_matrices(plan, lm, lc, uf, uf)
    qxa.sync(plan)
    ne = mesh["conn"].shape[1]
    Me, Ce = oracle.element_matrices(mesh, np.arange(ne), r, r, lm, lc, u, u)
    n = Me.shape[1]
    Vm = Vm.cpu().numpy().reshape(n, n, ne).transpose(2, 0, 1)
    Vc = Vc.cpu().numpy().reshape(n, n, ne).transpose(2, 0, 1)
    assert np.abs(Vm - Me).max() <= 1e-12 * np.abs(Me).max()
    assert np.abs(Vc - Ce).max() <= 1e-12 * np.abs(Ce).max()


def test_qpoint_coefficients_and_separate_rules():
    """Coefficient values given per (q, e), and different rules for M and C (paper policy)."""
    qxa = _qxa()
    mesh = structured_mesh(3, 2, 3, 0.2, seed=9)
    rm, rc = rule(3, 4), rule(3, 2)
    ne = mesh["conn"].shape[1]
    rng = np.random.default_rng(1)
    sm = rng.uniform(0.5, 2.0, size=(rm[1].size, ne))
    sc = rng.uniform(0.5, 2.0, size=(rc[1].size, ne))
    m = qxa.Mesh(3, 2, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rm, rc)
    M, Cv = qxa.assemble(plan, ("identity",), ("identity",), torch.tensor(sm, device="cuda"),
                         torch.tensor(sc, device="cuda"), qpoint=True)
    qxa.sync(plan)
    rpo, cio, Mo, Co = oracle.assemble(mesh, rm, rc, ("identity",), ("identity",), qpoint_m=sm, qpoint_c=sc)
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= 1e-12
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= 1e-12


def test_error_paths():
    qxa = _qxa()
    mesh = structured_mesh(2, 1, 4)
    # out-of-range node index
    c = mesh["conn"].copy()
    c[2, 3] = -1
    with pytest.raises(qxa.QxaError) as ei:
        qxa.Mesh(2, 1, mesh["coords"], c)
    assert ei.value.code == -2
    # degenerate element
    X = mesh["coords"].copy()
    v = mesh["conn"][:, 0]
    X[:, v[2]] = 2 * X[:, v[1]] - X[:, v[0]]
    with pytest.raises(qxa.QxaError) as ei:
        qxa.Mesh(2, 1, X, mesh["conn"])
    assert ei.value.code == -3
    # a rule larger than every compiled size (25 nodes in 2D; smaller ones are padded)
    from workloads.quadrature import conical
    m = qxa.Mesh(2, 1, mesh["coords"], mesh["conn"])
    with pytest.raises(qxa.QxaError) as ei:
        qxa.Plan(m, conical(2, 5))
    assert ei.value.code == -6
    # non-finite coefficient detected on the device, reported at sync
    plan = qxa.Plan(m, rule(2, 2))
    u = torch.zeros(mesh["n_nodes"], dtype=torch.float64, device="cuda")
    u[7] = float("nan")
    qxa.assemble(plan, ("const", 1.0), ("poly2", 1.0, 0.0, 1.0), None, u)
    with pytest.raises(qxa.QxaError) as ei:
        qxa.sync(plan)
    assert ei.value.code == -4
    qxa.assemble(plan, ("const", 1.0), ("const", 1.0))
    qxa.sync(plan)                                # flag was cleared


def test_empty_and_single_element_meshes():
    qxa = _qxa()
    X = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    m = qxa.Mesh(2, 1, X, np.zeros((3, 0), dtype=np.int32))
    plan = qxa.Plan(m, rule(2, 2))
    assert plan.nnz == 0
    qxa.assemble(plan, ("const", 1.0), ("const", 1.0))
    qxa.sync(plan)
    m1 = qxa.Mesh(2, 1, X, np.array([[0], [1], [2]], dtype=np.int32))
    p1 = qxa.Plan(m1, rule(2, 2))
    M, Cv = qxa.assemble(p1, ("const", 1.0), ("const", 1.0))
    qxa.sync(p1)
    assert abs(M.sum().item() - 0.5) < 1e-15
    assert np.allclose(Cv.cpu().numpy(), [1, -0.5, -0.5, -0.5, 0.5, 0, -0.5, 0, 0.5], atol=1e-15)




@pytest.mark.parametrize("name,N", [("p2_3d_32", 6), ("p3_2d_1024", 24)])
@pytest.mark.parametrize("form", ["fp32", "f16x2", "bf16x2", "bf16x3"])
def test_reduced_precision_forms(name, N, form):
    w = scaled(name, N)
    _say("case", w.name, form)
    mesh, r, u, plan, rp, ci, outs = _run(w, precision=form, reps=2)
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, w.mass_law, w.stiff_law, u, u)
    assert np.array_equal(rp, rpo) and np.array_equal(ci, cio)
    em = row_scaled_error(outs[0][0], Mo, rpo)
    ec = row_scaled_error(outs[0][1], Co, rpo)
    _say(f"{form} row-scaled error: mass {em:.3e} conductivity {ec:.3e}")
    assert em <= FORM_BOUNDS[form] and ec <= FORM_BOUNDS[form]
    assert np.array_equal(outs[0][0].view(np.uint64), outs[1][0].view(np.uint64))
    assert np.array_equal(outs[0][1].view(np.uint64), outs[1][1].view(np.uint64))


def test_split_forms_rejected_on_vector_alu_path():
    qxa = _qxa()
    w = scaled("p1_3d_96_heat", 3)
    mesh, r, u = make_inputs(w)
    plan = qxa.Plan(qxa.Mesh(w.dim, w.order, mesh["coords"], mesh["conn"]), r)
    uf = torch.tensor(u, device="cuda")
    with pytest.raises(qxa.QxaError) as ei:
        qxa.assemble(plan, w.mass_law, w.stiff_law, uf, uf, precision="bf16x2")
    assert ei.value.code == -6


# shapes whose coefficient paths the cases above leave out: per-(q, e) values with a
# lower-degree conductivity rule, two different nodal fields, one matrix only
EXTRA_SHAPES = [(2, 3, 7), (3, 2, 4), (3, 3, 3)]


@pytest.mark.parametrize("dim,order,N", EXTRA_SHAPES)
def test_qpoint_values_with_lower_degree_stiffness_rule(dim, order, N):
    qxa = _qxa()
    _say("case qpoint", dim, order, N)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[11, dim, order])
    rm, rc = rule(dim, 2 * order), rule(dim, 2 * order - 2)
    ne = mesh["conn"].shape[1]
    rng = np.random.default_rng([12, dim, order])
    sm = rng.uniform(0.5, 2.0, size=(rm[1].size, ne))
    sc = rng.uniform(-0.5, 0.5, size=(rc[1].size, ne))
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rm, rc)
    law_c = ("exp", 0.0, 1.0)
    M, Cv = qxa.assemble(plan, ("identity",), law_c, torch.tensor(sm, device="cuda"),
                         torch.tensor(sc, device="cuda"), qpoint=True)
    qxa.sync(plan)
    rpo, cio, Mo, Co = oracle.assemble(mesh, rm, rc, ("identity",), law_c, qpoint_m=sm, qpoint_c=sc)
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= 1e-12
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= 1e-12


@pytest.mark.parametrize("dim,order,N", EXTRA_SHAPES)
def test_two_nodal_fields_and_single_matrix(dim, order, N):
    qxa = _qxa()
    from workloads.fields import gaussian_random_field
    _say("case two fields", dim, order, N)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[13, dim, order])
    um = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([14, dim]), length=0.3)
    uc = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([15, dim]), length=0.2)
    r = rule(dim, 2 * order)
    law_m, law_c = ("poly2", 1.0, 0.2, 0.1), ("exp", 0.0, 1.0)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    fm, fc = torch.tensor(um, device="cuda"), torch.tensor(uc, device="cuda")
    M, Cv = qxa.assemble(plan, law_m, law_c, fm, fc)
    M1, _ = qxa.assemble(plan, law_m, law_c, fm, fc, want_c=False)
    _, C1 = qxa.assemble(plan, law_m, law_c, fm, fc, want_m=False)
    qxa.sync(plan)
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, law_m, law_c, um, uc)
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= 1e-12
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= 1e-12
    assert torch.equal(M.view(torch.int64), M1.view(torch.int64))
    assert torch.equal(Cv.view(torch.int64), C1.view(torch.int64))


@pytest.mark.parametrize("dim,order,N", [(2, 2, 9), (2, 3, 7), (3, 2, 4), (3, 3, 3)])
def test_plain_store_path_equals_buffer_store_path(dim, order, N, monkeypatch):
    """The consumers' plain-store path (arrays past 2^31 bytes) on a small mesh, forced
    through QXA_FLAT_STORES: the same bits as the buffer-store path."""
    qxa = _qxa()
    from workloads.fields import gaussian_random_field
    _say("case flat stores", dim, order, N)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[16, dim, order])
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([17, dim]), length=0.3)
    r = rule(dim, 2 * order)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    law_m, law_c = ("poly2", 1.0, 0.1, 0.0), ("exp", 0.0, 1.0)
    M, Cv = qxa.assemble(plan, law_m, law_c, uf, uf)
    qxa.sync(plan)
    monkeypatch.setenv("QXA_FLAT_STORES", "1")
    M2, C2 = qxa.assemble(plan, law_m, law_c, uf, uf)
    qxa.sync(plan)
    monkeypatch.delenv("QXA_FLAT_STORES")
    assert torch.equal(M.view(torch.int64), M2.view(torch.int64))
    assert torch.equal(Cv.view(torch.int64), C2.view(torch.int64))
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, law_m, law_c, u, u)
    assert row_scaled_error(M2.cpu().numpy(), Mo, rpo) <= 1e-12
