"""Degenerate cases of the next items on the GPU: a mesh without elements, a single element
(straight and with a curved edge), and a node that belongs to no element."""
import numpy as np
import pytest

import oracle
from helpers import row_scaled_error
from workloads import rule

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# P2 triangle: vertices, then edge nodes (0,1), (1,2), (2,0)
X6 = np.array([[0.0, 1.0, 0.0, 0.5, 0.5, 0.0],
               [0.0, 0.0, 1.0, 0.0, 0.5, 0.5]])
C6 = np.arange(6, dtype=np.int32).reshape(6, 1)


def test_next_items_on_a_mesh_without_elements():
    import paper_2204_03893_amd as qxa
    print("case next items, no elements", flush=True)
    m = qxa.Mesh(2, 2, X6, np.zeros((6, 0), dtype=np.int32))
    plan = qxa.Plan(m, rule(2, 4))
    assert plan.nnz == 0
    u = torch.ones(6, dtype=torch.float64, device="cuda")
    T, _ = qxa.mass_tensor_product(plan, ("poly2", 0.0, 1.0, 0.0), u, u)
    Tc = qxa.cond_tensor_product(plan, ("poly2", 0.0, 1.0, 0.0), u, u)
    F = qxa.load_vector(plan, ("const", 2.0))
    M, Cv = qxa.assemble_iso(plan, ("const", 1.0), ("const", 1.0))
    qxa.sync(plan)
    assert T.numel() == 0 and Tc.numel() == 0 and M.numel() == 0 and Cv.numel() == 0
    assert torch.equal(F, torch.zeros(6, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("bend", [0.0, 0.12])
def test_next_items_on_a_single_element(bend):
    import paper_2204_03893_amd as qxa
    print("case next items, one element, bend", bend, flush=True)
    X = X6.copy()
    X[:, 4] += bend * np.array([1.0, 1.0])           # curve the hypotenuse
    mesh = {"dim": 2, "order": 2, "coords": X, "conn": C6}
    r = rule(2, 4)
    m = qxa.Mesh(2, 2, X, C6)
    plan = qxa.Plan(m, r)
    u = np.array([0.1, -0.3, 0.7, 0.2, 0.5, -0.4])
    v = np.array([1.0, 0.5, -0.2, 0.3, -0.6, 0.8])
    uf, vf = torch.tensor(u, device="cuda"), torch.tensor(v, device="cuda")
    law = ("poly2", 0.2, 1.0, 0.3)
    M, Cv = qxa.assemble_iso(plan, ("const", 1.0), ("exp", 0.0, 1.0), None, uf)
    F = qxa.load_vector(plan, ("exp", 0.0, 1.0), uf)
    qxa.sync(plan)
    rp, _, Mo, Co = oracle.assemble_iso(mesh, r, r, ("const", 1.0), ("exp", 0.0, 1.0), None, u)
    assert row_scaled_error(M.cpu().numpy(), Mo, rp) <= 1e-13
    assert row_scaled_error(Cv.cpu().numpy(), Co, rp) <= 1e-13
    if bend == 0.0:
        assert abs(M.sum().item() - 0.5) <= 1e-15
        T, _ = qxa.mass_tensor_product(plan, law, uf, vf)
        Tc = qxa.cond_tensor_product(plan, law, uf, vf)
        qxa.sync(plan)
        _, _, To = oracle.mass_tensor_product(mesh, r, law, u, v)
        _, _, Tco = oracle.cond_tensor_product(mesh, r, law, u, v)
        assert row_scaled_error(T.cpu().numpy(), To, rp) <= 1e-13
        assert row_scaled_error(Tc.cpu().numpy(), Tco, rp) <= 1e-13
        Fo = oracle.load_vector(mesh, r, ("exp", 0.0, 1.0), u)
        assert np.abs(F.cpu().numpy() - Fo).max() <= 1e-14 * np.abs(Fo).max()
    else:
        assert abs(M.sum().item() - 0.5) > 1e-4                 # the curved edge changes the area


def test_node_outside_every_element():
    import paper_2204_03893_amd as qxa
    print("case next items, orphan node", flush=True)
    X = np.array([[0.0, 1.0, 0.0, 2.0], [0.0, 0.0, 1.0, 2.0]])
    conn = np.array([[0], [1], [2]], dtype=np.int32)
    mesh = {"dim": 2, "order": 1, "coords": X, "conn": conn}
    r = rule(2, 2)
    m = qxa.Mesh(2, 1, X, conn)
    plan = qxa.Plan(m, r)
    u = torch.tensor([0.5, 1.0, -1.0, 3.0], dtype=torch.float64, device="cuda")
    F = qxa.load_vector(plan, ("poly2", 1.0, 1.0, 0.0), u)
    M, Cv = qxa.assemble_iso(plan, ("const", 1.0), ("const", 1.0))
    qxa.sync(plan)
    Fo = oracle.load_vector(mesh, r, ("poly2", 1.0, 1.0, 0.0), u.cpu().numpy())
    assert F[3].item() == 0.0 and Fo[3] == 0.0
    assert np.abs(F.cpu().numpy() - Fo).max() <= 1e-15
    rp, _, Mo, Co = oracle.assemble_iso(mesh, r, r, ("const", 1.0), ("const", 1.0))
    assert rp[4] == rp[3]                                         # the orphan's row is empty
    assert np.abs(M.cpu().numpy() - Mo).max() <= 1e-14 * np.abs(Mo).max()   # (an empty row: no row scaling)
    assert np.abs(Cv.cpu().numpy() - Co).max() <= 1e-14 * np.abs(Co).max()
