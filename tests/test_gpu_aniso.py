"""Anisotropic conductivity c(u_h) K with a constant symmetric K (Section 7) on the GPU:
the fused assembly (every shape, FP64 and FP32), the serving path and the conductivity
tensor product, against the oracle."""
import numpy as np
import pytest

import oracle
from helpers import row_scaled_error
from workloads import rule, structured_mesh
from workloads.fields import gaussian_random_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(2, 1, 23), (2, 2, 13), (2, 3, 9), (3, 1, 7), (3, 2, 5), (3, 3, 3)]


def _K(dim, seed):
    S = np.eye(dim) + 0.4 * np.random.default_rng(seed).uniform(-1, 1, size=(dim, dim))
    K = S @ S.T
    return np.array([K[a, b] for a in range(dim) for b in range(a, dim)])


@pytest.mark.parametrize("dim,order,N", SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_anisotropic_assembly_against_oracle(dim, order, N, precision):
    import paper_2204_03893_amd as qxa
    print("case aniso", dim, order, N, precision, flush=True)
    mesh = structured_mesh(dim, order, N, 0.2, seed=[91, dim, order])
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng([92, dim]), length=0.3)
    r = rule(dim, 2 * order)
    K = _K(dim, [93, dim])
    law_m, law_c = ("poly2", 1.0, 0.1, 0.0), ("exp", 0.0, 1.0)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    uf = torch.tensor(u, device="cuda")
    M, Cv = qxa.assemble(plan, law_m, law_c, uf, uf, precision=precision, tensor=K)
    qxa.sync(plan)
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, law_m, law_c, u, u, tensor_c=K)
    tol = 1e-12 if precision == "fp64" else 5e-6
    assert row_scaled_error(M.cpu().numpy(), Mo, rpo) <= tol
    assert row_scaled_error(Cv.cpu().numpy(), Co, rpo) <= tol


def test_anisotropic_serving_and_tensor_product():
    import paper_2204_03893_amd as qxa
    dim, order = 3, 2
    mesh = structured_mesh(dim, order, 3, 0.2, seed=94)
    u = gaussian_random_field(mesh["coords"], 16, np.random.default_rng(95), length=0.3)
    r = rule(dim, 2 * order)
    K = _K(dim, 96)
    law_c = ("poly2", 1.0, 0.0, 0.5)
    m = qxa.Mesh(dim, order, mesh["coords"], mesh["conn"])
    uf = torch.tensor(u, device="cuda")
    srv = qxa.Server()
    t = srv.submit(m, r, r, ("const", 1.0), law_c, None, uf, tensor=K.copy())
    c = srv.wait(1)[0]
    assert c["status"] == 0, c["message"]
    Ms, Cs = srv.result(t)
    torch.cuda.synchronize()
    rpo, cio, Mo, Co = oracle.assemble(mesh, r, r, ("const", 1.0), law_c, None, u, tensor_c=K)
    assert row_scaled_error(Cs.cpu().numpy(), Co, rpo) <= 1e-12
    srv.release(t)
    srv.close()
    plan = qxa.Plan(m, r)
    v = torch.tensor(np.random.default_rng(97).uniform(-1, 1, size=u.size), device="cuda")
    T = qxa.cond_tensor_product(plan, ("poly2", 0.0, 1.0, 0.0), uf, v, tensor=K)
    qxa.sync(plan)
    _, _, To = oracle.cond_tensor_product(mesh, r, ("poly2", 0.0, 1.0, 0.0), u, v.cpu().numpy(), tensor=K)
    assert row_scaled_error(T.cpu().numpy(), To, rpo) <= 1e-12
    with pytest.raises(qxa.QxaError) as ei:        # a tensor on the mass coefficient is rejected
        cm, k = qxa.make_coeff(("const", 1.0), tensor=K)
        qxa.check(qxa.lib().qxa_assemble(plan.handle, qxa.C.byref(cm), None, 0, None, None, None))
    assert ei.value.code == -1
