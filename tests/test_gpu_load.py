"""Volume load vector and reaction matrix on the GPU against the oracle."""
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
def test_load_vector_against_oracle(dim, order, N):
    import paper_2204_03893_amd as qxa
    print("case load", dim, order, N, flush=True)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[71, dim, order])
    f = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([72, dim]), length=0.3)
    r = rule(dim, 2 * order)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    ff = torch.tensor(f, device="cuda")
    for law in [("exp", 0.0, 1.0), ("const", 3.0)]:
        F = qxa.load_vector(plan, law, ff if law[0] != "const" else None)
        F2 = qxa.load_vector(plan, law, ff if law[0] != "const" else None)
        qxa.sync(plan)
        Fo = oracle.load_vector(mesh, r, law, f if law[0] != "const" else None)
        Fh = F.cpu().numpy()
        assert np.abs(Fh - Fo).max() <= 1e-12 * np.abs(Fo).max()
        assert torch.equal(F.view(torch.int64), F2.view(torch.int64))
    # per-(q, e) values
    ne = mesh["conn"].shape[1]
    S = np.random.default_rng([73, dim]).uniform(0.5, 2.0, size=(r[1].size, ne))
    F = qxa.load_vector(plan, ("identity",), torch.tensor(S, device="cuda"), qpoint=True)
    qxa.sync(plan)
    Fo = oracle.load_vector(mesh, r, ("identity",), qpoint=S)
    assert np.abs(F.cpu().numpy() - Fo).max() <= 1e-12 * np.abs(Fo).max()


@pytest.mark.parametrize("dim,order,N", [(2, 2, 9), (3, 3, 2)])
def test_reaction_matrix_is_the_mass_path(dim, order, N):
    import paper_2204_03893_amd as qxa
    mesh = structured_mesh(dim, order, N, 0.2, seed=[74, dim, order])
    a = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([75, dim]), length=0.3)
    r = rule(dim, 2 * order)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    law = ("poly2", 0.5, 0.0, 1.0)
    A = qxa.reaction_matrix(plan, law, torch.tensor(a, device="cuda"))
    qxa.sync(plan)
    rpo, cio, Ao, _ = oracle.assemble(mesh, r, r, law, ("const", 1.0), a, None)
    assert row_scaled_error(A.cpu().numpy(), Ao, rpo) <= 1e-12
