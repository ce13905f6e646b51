"""Quadrature rules of any size at the boundary (Algorithm 2 takes the nodes and
weights as inputs, possibly one rule per matrix; Section 4). The library pads a
rule with zero-weight copies of its node 0 up to the compiled rule size of least
work that holds it. Host-only checks: the rules themselves against exact
moments, and the plan build (reference tables, pattern, tile plan, executed with
exact integer sums) accepting them with the padded sizes it reports."""
import itertools
import math

import numpy as np
import pytest

import paper_2204_03893_amd as qxa
from workloads import structured_mesh
from workloads.quadrature import conical, keast5, radon7


def _moment_error(P, W, deg):
    d = P.shape[1]
    err = 0.0
    for a in itertools.product(range(deg + 1), repeat=d):
        if sum(a) > deg:
            continue
        exact = math.prod(math.factorial(x) for x in a) / math.factorial(sum(a) + d)
        err = max(err, abs(float(np.sum(W * np.prod(P ** np.array(a), axis=1))) - exact))
    return err


@pytest.mark.parametrize("name,P_W,deg", [("radon7", radon7(), 5), ("keast5", keast5(), 3),
                                          ("conical 2D 4", conical(2, 4), 6), ("conical 3D 3", conical(3, 3), 3)])
def test_extra_rules_integrate_monomials_exactly(name, P_W, deg):
    """Every monomial up to the rule's degree on the reference simplex
    (int x^alpha = alpha! / (|alpha| + d)!), and one degree above is not exact."""
    P, W = P_W
    assert _moment_error(P, W, deg) <= 1e-15
    assert _moment_error(P, W, deg + 1) > 1e-6


# (dim, order, mass rule, stiffness rule, kernel sizes the least-work padding picks)
CASES = [
    (2, 1, "radon7", "radon7", (16, 16)),   # P1 compiles 3 nodes and the padded 16
    (2, 2, "radon7", "radon7", (16, 16)),
    (2, 3, "radon7", "radon7", (12, 12)),   # fits the tuned 12-node kernel
    (2, 3, "radon7", "centroid", (12, 6)),
    (2, 2, "conical4", "centroid", (16, 16)),
    (3, 1, "keast5", "keast5", (32, 32)),
    (3, 2, "keast5", "keast5", (11, 11)),
    (3, 3, "keast5", "keast5", (24, 11)),
    (3, 2, "keast5", "centroid", (11, 4)),
    (3, 3, "conical27", "conical27", (32, 32)),
    (3, 2, "conical27", "keast5", (32, 32)),  # too large for Q^T on chip: the vector-ALU variant
]


def _rule(name, dim):
    if name == "radon7":
        return radon7()
    if name == "keast5":
        return keast5()
    if name == "conical4":
        return conical(2, 4)
    if name == "conical27":
        return conical(3, 3)
    assert name == "centroid"
    return np.full((1, dim), 1.0 / (dim + 1)), np.array([1.0 / math.factorial(dim)])


@pytest.mark.parametrize("dim,order,rm,rc,sizes", CASES)
def test_plan_accepts_rules_of_any_size(dim, order, rm, rc, sizes):
    m = structured_mesh(dim, order, 6 if dim == 2 else 3, 0.2, seed=5)
    Rm, Rc = _rule(rm, dim), _rule(rc, dim)
    s = qxa.plan_check_host(dim, order, m["coords"], m["conn"], rule_m=Rm, rule_c=Rc)
    assert (s["n_q_mass"], s["n_q_stiff"]) == (len(Rm[1]), len(Rc[1]))
    assert (s["n_q_mass_kernel"], s["n_q_stiff_kernel"]) == sizes
    assert s["n_tiles"] >= 1


@pytest.mark.parametrize("dim,n", [(2, 5), (3, 4)])
def test_rules_beyond_the_compiled_sizes_are_refused(dim, n):
    """25 nodes in 2D (more than 16) and 64 in 3D (more than 32): QXA_E_UNSUPPORTED."""
    m = structured_mesh(dim, 1, 3, 0.0)
    with pytest.raises(qxa.QxaError) as ei:
        qxa.plan_check_host(dim, 1, m["coords"], m["conn"], rule_m=conical(dim, n))
    assert ei.value.code == -6
    assert "at most" in str(ei.value)


def test_rule_weights_must_sum_to_the_volume():
    m = structured_mesh(2, 1, 3, 0.0)
    P, W = radon7()
    with pytest.raises(qxa.QxaError) as ei:
        qxa.plan_check_host(2, 1, m["coords"], m["conn"], rule_m=(P, 2 * W))
    assert ei.value.code == -1
