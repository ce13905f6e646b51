"""The next items at the size of the 2D P3 workload (1024^2 cells, 2,097,152 elements,
9,443,329 nodes), every value compared with the oracle: the mass and conductivity tensor
products, the load vector and the isoparametric assembly (curved by a bump that vanishes
on the boundary)."""
import numpy as np
import pytest

import oracle
from helpers import row_scaled_error, workload_inputs
from workloads import WORKLOADS
from workloads.fields import gaussian_random_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    import paper_2204_03893_amd as qxa
    w = WORKLOADS["p3_2d_1024"]
    print("case next-items full size", w.name, flush=True)
    mesh, r, u = workload_inputs("p3_2d_1024")
    v = gaussian_random_field(mesh["coords"], 16, np.random.default_rng(2204), length=0.2)
    m = qxa.Mesh(w.dim, w.order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    return qxa, w, mesh, r, u, v, plan


def test_tensor_products_full_size_p3(setup):
    qxa, w, mesh, r, u, v, plan = setup
    print("case tensor products, 2D P3 full size", flush=True)
    uf, vf = torch.tensor(u, device="cuda"), torch.tensor(v, device="cuda")
    law = ("poly2", 0.0, 1.0, 0.0)
    Tc = qxa.cond_tensor_product(plan, law, uf, vf)
    Tm, _ = qxa.mass_tensor_product(plan, law, uf, vf)
    qxa.sync(plan)
    rpo, _, Tco = oracle.cond_tensor_product(mesh, r, law, u, v)
    err = row_scaled_error(Tc.cpu().numpy(), Tco, rpo)
    print("conductivity tensor product: row-scaled error", err, flush=True)
    assert err <= 1e-12
    del Tco
    _, _, Tmo = oracle.mass_tensor_product(mesh, r, law, u, v)
    assert row_scaled_error(Tm.cpu().numpy(), Tmo, rpo) <= 1e-12


def test_load_vector_full_size_p3(setup):
    qxa, w, mesh, r, u, v, plan = setup
    print("case load vector, 2D P3 full size", flush=True)
    F = qxa.load_vector(plan, ("exp", 0.0, 1.0), torch.tensor(u, device="cuda"))
    qxa.sync(plan)
    Fo = oracle.load_vector(mesh, r, ("exp", 0.0, 1.0), u)
    assert np.abs(F.cpu().numpy() - Fo).max() <= 1e-12 * np.abs(Fo).max()


def test_isoparametric_full_size_p3(setup):
    qxa, w, mesh, r, u, v, _ = setup
    print("case isoparametric, 2D P3 full size", flush=True)
    X = mesh["coords"]
    bump = np.prod(np.sin(np.pi * X), axis=0)
    curved = dict(mesh)
    curved["coords"] = np.ascontiguousarray(X + (0.1 / w.N) * bump * np.array([1.0, -0.7])[:, None])
    m = qxa.Mesh(w.dim, w.order, curved["coords"], curved["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    M, Cv = qxa.assemble_iso(plan, w.mass_law, w.stiff_law, uf, uf)
    qxa.sync(plan)
    rpo, _, Mo, Co = oracle.assemble_iso(curved, r, r, w.mass_law, w.stiff_law, u, u)
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= 1e-12
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= 1e-12
