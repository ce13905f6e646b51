"""The allocation-free formation entry point (qxa_element_matrices_noalloc) against
qxa_element_matrices, called through the C-ABI: bitwise-equal element matrices on two
calls in a row (a larger mesh, then a smaller one, so the second call reuses scratch
holding the first call's values), in FP64 and FP32, and the size limit refused with an
error before anything is launched."""
import numpy as np
import pytest

from workloads import WORKLOADS, make_inputs, scaled

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(name, N):
    import paper_2204_03893_amd as qxa
    w = scaled(name, N)
    mesh, rule, u = make_inputs(w)
    m = qxa.Mesh(w.dim, w.order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rule)
    return qxa, w, m, plan, torch.tensor(u, device="cuda")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_allocating_entry_point(precision):
    cases = [("p2_3d_32", 8), ("p3_2d_1024", 6)]   # 3,072 elements, then 72
    for name, N in cases:
        qxa, w, m, plan, uf = _case(name, N)
        print("case noalloc", name, N, precision, flush=True)
        Vm0, Vc0 = qxa.element_matrices(plan, w.mass_law, w.stiff_law, uf, uf, precision=precision)
        Vm1, Vc1 = qxa.element_matrices_noalloc(plan, w.mass_law, w.stiff_law, uf, uf, precision=precision)
        qxa.sync(plan)
        assert torch.equal(Vm0.view(torch.int64), Vm1.view(torch.int64))
        assert torch.equal(Vc0.view(torch.int64), Vc1.view(torch.int64))
        assert torch.isfinite(Vm1).all() and torch.isfinite(Vc1).all()
        del plan, m


def test_noalloc_refuses_meshes_beyond_the_scratch():
    # 3D P2 on 24^3 cells: 82,944 elements, 2 * 55 * 82,944 doubles > 8,388,608
    qxa, w, m, plan, uf = _case("p2_3d_32", 24)
    n2 = plan.n_p ** 2
    Vm = torch.full((n2, plan.n_elem), 7.0, dtype=torch.float64, device="cuda")
    Vc = torch.full_like(Vm, 7.0)
    with pytest.raises(qxa.QxaError) as ei:
        qxa.element_matrices_noalloc(plan, w.mass_law, w.stiff_law, uf, uf, Vm=Vm, Vc=Vc)
    assert ei.value.code == -6 and "exceeds the scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((Vm == 7.0).all()) and bool((Vc == 7.0).all())   # nothing was launched
