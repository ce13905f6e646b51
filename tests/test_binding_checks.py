"""The binding rejects device arguments of the wrong dtype, device, layout or length with
ValueError before anything reaches the library (CPU only: every case raises before a
kernel could be launched, and the stub plan below has no library handle at all)."""
from types import SimpleNamespace

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2204_03893_amd as qxa  # noqa: E402


def _stub_plan(dim=2, order=2, n_nodes=25, n_elem=32, nnz=200, nqm=6, nqc=6):
    mesh = SimpleNamespace(dim=dim, order=order, device=0, handle=None)
    return SimpleNamespace(mesh=mesh, n_nodes=n_nodes, n_elem=n_elem, nnz=nnz, n_q_mass=nqm, n_q_stiff=nqc,
                           n_p=qxa._n_local(dim, order), handle=None)


def test_dev_arg_checks_each_property():
    f64 = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        qxa._dev_arg(torch.zeros(10, dtype=torch.float32), "x", 10, 0)
    with pytest.raises(ValueError, match="expected cuda:0"):
        qxa._dev_arg(f64, "x", 10, 0)                       # a CPU tensor
    with pytest.raises(ValueError, match="torch tensor"):
        qxa._dev_arg(np.zeros(10), "x", 10, 0)
    assert qxa._dev_arg(None, "x", 10, 0) is None


def test_coefficient_fields_are_checked_against_the_plan():
    plan = _stub_plan()
    sz = qxa._sizes(plan, "mass")
    # a nodal field on the host, or of the wrong dtype, or a non-constant law without a field
    with pytest.raises(ValueError, match="mass field"):
        qxa.make_coeff(("exp", 0.0, 1.0), torch.zeros(plan.n_nodes, dtype=torch.float64), sizes=sz, name="mass")
    with pytest.raises(ValueError, match="dtype"):
        qxa.make_coeff(("exp", 0.0, 1.0), torch.zeros(plan.n_nodes, dtype=torch.float32), sizes=sz)
    with pytest.raises(ValueError):
        qxa.make_coeff(("exp", 0.0, 1.0), None, sizes=sz)
    # a constant tensor with the wrong number of upper-triangle entries
    with pytest.raises(ValueError, match="upper-triangle"):
        qxa.make_coeff(("const", 1.0), tensor=[1.0, 0.0], sizes=sz)


@pytest.mark.parametrize("call", ["assemble", "assemble_iso", "cond_tensor_product", "load_vector", "coeff_product"])
def test_entry_points_reject_host_tensors(call):
    plan = _stub_plan()
    u = torch.zeros(plan.n_nodes, dtype=torch.float64)      # host memory: never a device pointer
    law = ("poly2", 1.0, 0.0, 1.0)
    with pytest.raises(ValueError):
        if call == "assemble":
            qxa.assemble(plan, law, law, u, u)
        elif call == "assemble_iso":
            qxa.assemble_iso(plan, law, law, u, u)
        elif call == "cond_tensor_product":
            qxa.cond_tensor_product(plan, law, u, u)
        elif call == "load_vector":
            qxa.load_vector(plan, law, u)
        else:
            qxa.coeff_product(plan, law, u, u)


def test_output_arrays_are_checked():
    plan = _stub_plan()
    with pytest.raises(ValueError, match="M: dtype"):
        qxa.assemble(plan, ("const", 1.0), ("const", 1.0), M=torch.zeros(plan.nnz, dtype=torch.float32))
    with pytest.raises(ValueError, match="Cv: on cpu"):
        qxa.assemble(plan, ("const", 1.0), ("const", 1.0), Cv=torch.zeros(plan.nnz, dtype=torch.float64))
    with pytest.raises(ValueError, match="F: on cpu"):
        qxa.load_vector(plan, ("const", 1.0), F=torch.zeros(plan.n_nodes, dtype=torch.float64))


def test_mesh_connectivity_rows_match_the_order():
    X = np.zeros((2, 6))
    conn = np.zeros((3, 1), dtype=np.int32)                  # 3 rows: P1, not the P2 that is claimed
    with pytest.raises(ValueError, match="nodes"):
        qxa.Mesh(2, 2, X, conn)
    with pytest.raises(ValueError, match="coords"):
        qxa.Mesh(3, 1, X, np.zeros((4, 1), dtype=np.int32))  # 2 coordinate rows for a 3D mesh
