"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle
import paper_2204_03893_amd as qxa
from workloads import structured_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*\b(qxa_[a-z0-9_]+)\s*\(", txt, re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    names = _declared_symbols()
    assert {"qxa_mesh_create", "qxa_plan_create", "qxa_assemble", "qxa_sync"} <= names
    L = ctypes.CDLL(qxa.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert missing == []


@pytest.mark.parametrize("dim,order,N", [(2, 1, 9), (2, 2, 5), (2, 3, 4), (3, 1, 4), (3, 2, 3), (3, 3, 2)])
def test_host_pattern_matches_oracle(dim, order, N):
    m = structured_mesh(dim, order, N, 0.1, seed=2)
    rp, ci = qxa.pattern_host(dim, order, m["n_nodes"], m["conn"])
    rpo, cio = oracle.pattern(m)
    assert np.array_equal(rp, rpo)
    assert np.array_equal(ci, cio)


def test_host_pattern_relabelled_mesh():
    m = structured_mesh(3, 2, 2)
    sigma = np.random.default_rng(3).permutation(m["n_nodes"])
    m["conn"] = sigma[m["conn"]].astype(np.int32)
    rp, ci = qxa.pattern_host(3, 2, m["n_nodes"], m["conn"])
    rpo, cio = oracle.pattern(m)
    assert np.array_equal(rp, rpo) and np.array_equal(ci, cio)


def test_host_pattern_rejects_bad_index():
    m = structured_mesh(2, 1, 3)
    c = m["conn"].copy()
    c[1, 5] = m["n_nodes"]
    with pytest.raises(qxa.QxaError) as ei:
        qxa.pattern_host(2, 1, m["n_nodes"], c)
    assert ei.value.code == -2


def test_host_pattern_empty_mesh():
    rp, ci = qxa.pattern_host(2, 1, 5, np.zeros((3, 0), dtype=np.int32))
    assert ci.size == 0 and np.all(rp == 0)


@pytest.mark.parametrize("dim,order,N", [(2, 1, 64), (2, 1, 7), (2, 2, 9), (2, 3, 5), (3, 1, 5), (3, 2, 3),
                                         (3, 3, 2), (3, 2, 32)])
def test_tile_plan_selfcheck(dim, order, N):
    """Fused-kernel plan executed on the host with exact integer sums: every CSR slot gets
    exactly its element entries, every index is in bounds, every slot written once."""
    m = structured_mesh(dim, order, N, 0.2, seed=3)
    s = qxa.plan_check_host(dim, order, m["coords"], m["conn"])
    assert s["n_tiles"] >= 1 and s["n_units"] >= s["n_pair_units"] and s["n_outputs"] >= 2 * s["n_pair_units"]
    # every output is a pair half or ends one single unit
    assert s["n_outputs"] == 2 * s["n_pair_units"] + s["n_units"] - s["n_pair_units"] - s["n_ext_units"] \
        - s["n_empty_units"]


@pytest.mark.parametrize("dim,order,N", [(2, 1, 40), (2, 2, 20), (2, 3, 24), (3, 1, 12), (3, 2, 8), (3, 3, 4)])
@pytest.mark.parametrize("chains,cap", [(1, 4096), (3, 4096), (4, 64), (5, 3), (2, 0)])
def test_tile_plan_carries(dim, order, N, chains, cap):
    """Chains of tiles with LDS carry entries (plenty, few, one tile's worth, none): the
    plan executes exactly on the host, slots touched by several tiles of a chain are
    carried instead of being summed from partials, and a smaller carry budget only moves
    slots back to partials."""
    m = structured_mesh(dim, order, N, 0.2, seed=7)
    s = qxa.plan_check_host(dim, order, m["coords"], m["conn"], chains=chains, carry_cap=cap)
    nt, npart, ncr = s["n_tiles"], s["n_partials"], s["n_carry_reads"]
    s1 = qxa.plan_check_host(dim, order, m["coords"], m["conn"], chains=nt, carry_cap=cap)
    npart1, ncr1 = s1["n_partials"], s1["n_carry_reads"]
    assert ncr1 == 0                       # one tile per chain: nothing to carry
    if cap == 0:
        assert ncr == 0 and npart == npart1
    elif nt > chains:
        assert ncr > 0 and npart < npart1  # carries replace partials


@pytest.mark.parametrize("dim,order,N,chains,cap", [(3, 1, 12, 0, -1), (3, 2, 8, 0, -1), (3, 2, 8, 3, 4096),
                                                    (2, 3, 24, 2, 4096), (2, 1, 40, 0, -1)])
def test_tile_plan_extended_outputs(dim, order, N, chains, cap):
    """Outputs of more than six entries (a vertex diagonal summed over the elements of a
    tile that hold the vertex, plus a carried sum) run over several units of one thread;
    the plan still executes exactly. Kuhn meshes in 3D put up to 24 tetrahedra around a
    vertex, so such outputs must occur there."""
    m = structured_mesh(dim, order, N, 0.2, seed=11)
    s = qxa.plan_check_host(dim, order, m["coords"], m["conn"], chains=chains, carry_cap=cap)
    if dim == 3:
        assert s["n_ext_units"] > 0


def test_tile_plan_of_a_mesh_without_elements():
    m = structured_mesh(2, 2, 2, 0.0)
    for kw in ({}, {"chains": 4, "carry_cap": 8}):
        s = qxa.plan_check_host(2, 2, m["coords"], np.zeros((6, 0), dtype=np.int32), **kw)
        assert s["n_tiles"] == s["n_units"] == s["n_partials"] == s["nnz"] == 0


def test_tile_plan_selfcheck_relabelled_and_shuffled():
    m = structured_mesh(3, 2, 4, 0.2, seed=4)
    rng = np.random.default_rng(5)
    sigma = rng.permutation(m["n_nodes"])
    conn = sigma[m["conn"]].astype(np.int32)[:, rng.permutation(m["conn"].shape[1])]
    X = np.empty_like(m["coords"])
    X[:, sigma] = m["coords"]
    qxa.plan_check_host(3, 2, X, conn)
    qxa.plan_check_host(3, 2, X, conn, chains=2, carry_cap=16)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("degree", [1, 2, 3, 4, 5, 6])
def test_builtin_rules(dim, degree):
    """qxa_quad_builtin: the same doubles as the input module's rules, and every monomial
    moment of its degree on the reference simplex (int x^alpha = alpha! / (|alpha| + d)!)."""
    import itertools
    import math
    from workloads import rule
    from workloads.quadrature import rule_degree
    P, W = qxa.quad_builtin(dim, degree)
    Pr, Wr = rule(dim, degree)
    assert np.array_equal(P, Pr) and np.array_equal(W, Wr)
    deg = rule_degree(dim, degree)
    for alpha in itertools.product(range(deg + 1), repeat=dim):
        if sum(alpha) > deg:
            continue
        exact = math.prod(math.factorial(a) for a in alpha) / math.factorial(sum(alpha) + dim)
        got = float(np.sum(W * np.prod(P ** np.array(alpha), axis=1)))
        assert abs(got - exact) <= 1e-15


def test_builtin_rule_errors():
    with pytest.raises(qxa.QxaError) as ei:
        qxa.quad_builtin(2, 7)
    assert ei.value.code == -6
    with pytest.raises(qxa.QxaError) as ei:
        qxa.quad_builtin(4, 2)
    assert ei.value.code == -1


def test_builtin_rule_tables_are_generated():
    """csrc/rules_builtin.cpp is exactly what paper_2204_03893_amd/gen_rules.py writes."""
    from paper_2204_03893_amd import gen_rules
    path = os.path.join(os.path.dirname(qxa.__file__), "csrc", "rules_builtin.cpp")
    with open(path) as f:
        assert f.read() == gen_rules.render()


@pytest.mark.parametrize("dim,order,N,chains", [(2, 2, 12, 8), (2, 3, 10, 0), (3, 2, 4, 0), (3, 1, 6, 0)])
@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5, 6])
def test_plan_check_rejects_corrupted_plans(dim, order, N, chains, mutation):
    """The host plan check (which every qxa_plan_create runs before anything reaches the
    GPU) rejects a plan with one deliberate corruption: a doubly written slot, a dropped
    or exchanged entry, an out-of-range LDS index, a doubly written partial, a wrong
    fix-up mirror. The uncorrupted plan of the same mesh passes."""
    mesh = structured_mesh(dim, order, N, 0.2, seed=[131, dim, order])
    qxa.plan_check_host(dim, order, mesh["coords"], mesh["conn"], chains=chains)
    st, msg = qxa.plan_check_host_corrupted(dim, order, mesh["coords"], mesh["conn"], mutation, chains=chains)
    assert st == -1, (st, msg)  # QXA_E_INVALID
    assert msg.startswith("tile plan:"), msg


def test_tile_plan_runs_on_3d_p3():
    """3D P3 (896 carry entries, too few for long chains): one chain per workgroup made of
    4-tile runs, the workgroups of one XCD on neighbouring runs. The plan passes the host
    execution check, uses carries, and has fewer partials than one-tile chains; a mesh with
    too few tiles for a run per workgroup gets one-tile chains."""
    mesh = structured_mesh(3, 3, 14, 0.2, seed=[150, 3, 3])
    s = qxa.plan_check_host(3, 3, mesh["coords"], mesh["conn"])
    assert s["n_chains"] == 256 and s["carry_cap"] == 896 and s["n_carry_reads"] > 0, s
    one = qxa.plan_check_host(3, 3, mesh["coords"], mesh["conn"], chains=s["n_tiles"], carry_cap=0)
    assert s["n_partials"] < 0.9 * one["n_partials"], (s["n_partials"], one["n_partials"])
    small = structured_mesh(3, 3, 6, 0.2, seed=[151, 3, 3])
    t = qxa.plan_check_host(3, 3, small["coords"], small["conn"])
    assert t["n_chains"] == t["n_tiles"] and t["n_carry_reads"] == 0, t
