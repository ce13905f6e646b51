"""Mass tensor contracted with a nodal vector (Section 5, Newton Jacobian) on the
GPU: qxa_coeff_product evaluates m'(u_h) v_h at the quadrature nodes, the fused
assembly forms the mass matrix of that coefficient; compared with the oracle,
which forms each element's full third-order tensor and contracts it."""
import numpy as np
import pytest

import oracle
from helpers import row_scaled_error
from workloads import rule, structured_mesh
from workloads.fields import gaussian_random_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(2, 1, 23), (2, 2, 13), (2, 3, 9), (3, 1, 7), (3, 2, 5), (3, 3, 3)]


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_mass_tensor_product_against_oracle(dim, order, N):
    import paper_2204_03893_amd as qxa
    print("case", dim, order, N, flush=True)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[41, dim, order])
    rng = np.random.default_rng([42, dim, order])
    u = gaussian_random_field(mesh["coords"], 16, rng, length=0.3)
    v = gaussian_random_field(mesh["coords"], 16, rng, length=0.2)
    r = rule(dim, 2 * order)
    law_dm = ("poly2", 0.3, 0.4, 0.0)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf, vf = torch.tensor(u, device="cuda"), torch.tensor(v, device="cuda")
    T, S = qxa.mass_tensor_product(plan, law_dm, uf, vf)
    T2, _ = qxa.mass_tensor_product(plan, law_dm, uf, vf)
    qxa.sync(plan)
    rpo, cio, To = oracle.mass_tensor_product(mesh, r, law_dm, u, v)
    assert row_scaled_error(T.cpu().numpy(), To, rpo) <= 1e-12
    assert torch.equal(T.view(torch.int64), T2.view(torch.int64))
    # the per-node coefficient itself, against the oracle's coefficient evaluation
    sel = np.arange(0, mesh["conn"].shape[1], 7)
    su = oracle.qpoint_coeff(mesh, sel, r, law_dm, u)
    sv = oracle.qpoint_coeff(mesh, sel, r, ("identity",), v)
    Sg = S.cpu().numpy()[:, sel].T
    assert np.abs(Sg - su * sv).max() <= 1e-13 * max(1.0, np.abs(su * sv).max())


def test_coeff_product_errors():
    import paper_2204_03893_amd as qxa
    mesh = structured_mesh(2, 2, 3, 0.0)
    m = qxa.Mesh(2, 2, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rule(2, 4))
    u = torch.zeros(mesh["n_nodes"], dtype=torch.float64, device="cuda")
    with pytest.raises(qxa.QxaError) as ei:
        qxa.coeff_product(plan, ("const", 1.0), None, u)     # the first factor must be nodal
    assert ei.value.code == -1
    with pytest.raises(KeyError):
        qxa.coeff_product(plan, ("identity",), u, u, rule="load")
    v = u.clone()
    v[3] = float("nan")
    qxa.coeff_product(plan, ("identity",), u + 1.0, v)
    with pytest.raises(qxa.QxaError) as ei:
        qxa.sync(plan)
    assert ei.value.code == -4


@pytest.mark.parametrize("dim,order,N", SHAPES)
def test_cond_tensor_product_against_oracle(dim, order, N):
    import paper_2204_03893_amd as qxa
    print("case cond", dim, order, N, flush=True)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[43, dim, order])
    rng = np.random.default_rng([44, dim, order])
    u = gaussian_random_field(mesh["coords"], 16, rng, length=0.3)
    v = gaussian_random_field(mesh["coords"], 16, rng, length=0.2)
    r = rule(dim, 2 * order)
    law_dc = ("exp", 0.0, 0.5)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf, vf = torch.tensor(u, device="cuda"), torch.tensor(v, device="cuda")
    T = qxa.cond_tensor_product(plan, law_dc, uf, vf)
    T2 = qxa.cond_tensor_product(plan, law_dc, uf, vf)
    qxa.sync(plan)
    rp, ci = plan.pattern()
    rpo, cio, To = oracle.cond_tensor_product(mesh, r, law_dc, u, v)
    assert np.array_equal(rp.cpu().numpy(), rpo) and np.array_equal(ci.cpu().numpy(), cio)
    assert row_scaled_error(T.cpu().numpy(), To, rpo) <= 1e-12
    assert torch.equal(T.view(torch.int64), T2.view(torch.int64))


def test_cond_tensor_product_errors():
    import paper_2204_03893_amd as qxa
    mesh = structured_mesh(2, 2, 3, 0.0)
    m = qxa.Mesh(2, 2, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rule(2, 4))
    u = torch.zeros(mesh["n_nodes"], dtype=torch.float64, device="cuda")
    with pytest.raises(qxa.QxaError) as ei:
        qxa.cond_tensor_product(plan, ("const", 1.0), None, u)
    assert ei.value.code == -1
    bad = u.clone()
    bad[5] = float("inf")
    qxa.cond_tensor_product(plan, ("identity",), bad, u + 1.0)
    with pytest.raises(qxa.QxaError) as ei:
        qxa.sync(plan)
    assert ei.value.code == -4
