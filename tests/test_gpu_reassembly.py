"""Reassembly through a captured HIP graph (only the coefficient field changes).

Every replay must equal a direct assembly of the same field bitwise, and the
first and last steps must match the CPU oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from helpers import row_scaled_error
from workloads import heat_increment, make_inputs, scaled

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name,N,precision", [("p1_3d_96_heat", 10, "fp64"), ("p2_3d_32", 5, "fp64"),
                                               ("p1_3d_96_heat", 8, "fp32")])
def test_graph_replay_matches_direct_assembly(name, N, precision):
    import paper_2204_03893_amd as qxa
    w = scaled(name, N)
    print("case", w.name, precision, flush=True)
    mesh, r, u0 = make_inputs(w)
    m = qxa.Mesh(w.dim, w.order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, r)
    u = torch.tensor(u0, device="cuda")
    g = qxa.ReassemblyGraph(plan, w.mass_law, w.stiff_law, u, u, precision=precision)
    u_host = u0.copy()
    steps = 5
    for s in range(steps):
        if s > 0:
            d = heat_increment(w, mesh, s)
            u += torch.tensor(d, device="cuda")       # in-place update of the captured field
            u_host = u_host + d
        Mg, Cg = g.launch()
        qxa.sync(plan)
        Mg, Cg = Mg.clone(), Cg.clone()
        Md, Cd = qxa.assemble(plan, w.mass_law, w.stiff_law, u, u, precision=precision)
        qxa.sync(plan)
        torch.cuda.synchronize()
        assert torch.equal(Mg.view(torch.int64), Md.view(torch.int64))
        assert torch.equal(Cg.view(torch.int64), Cd.view(torch.int64))
        if s in (0, steps - 1):
            uh = u.cpu().numpy()
            rp, ci, Mo, Co = oracle.assemble(mesh, r, r, w.mass_law, w.stiff_law, uh, uh)
            tol = 1e-12 if precision == "fp64" else 1e-6
            assert row_scaled_error(Mg.cpu().numpy(), Mo, rp) <= tol
            assert row_scaled_error(Cg.cpu().numpy(), Co, rp) <= tol
    g.close()
