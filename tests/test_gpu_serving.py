"""Serving loop: continuous batching, resident plans, device-memory budget.

Every job's CSR values must be bitwise identical to the same job assembled
alone (qxa_assemble with its own plan); batched launches must actually occur;
a plan-cache hit must give the same bits as the miss; a tight budget must
queue jobs instead of failing them, and only a job that can never fit fails
(QXA_E_NOMEM).
"""
import numpy as np
import pytest

import oracle
from helpers import row_scaled_error
from workloads import rule, structured_mesh
from workloads.fields import gaussian_random_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(2, 1, 12), (2, 2, 6), (2, 3, 4), (3, 1, 4), (3, 2, 2), (3, 3, 2)]
LAW_M = ("poly2", 1.0, 0.1, 0.0)
LAW_C = ("exp", 0.0, 1.0)


def _mesh(dim, order, N, seed):
    return structured_mesh(dim, order, N, 0.2, seed=seed)


def _field(m, seed):
    return gaussian_random_field(m["coords"], 16, np.random.default_rng(seed), length=0.3)


def _alone(qxa, mesh_obj, r, u, precision="fp64"):
    plan = qxa.Plan(mesh_obj, r)
    M, Cv = qxa.assemble(plan, LAW_M, LAW_C, u, u, precision=precision)
    qxa.sync(plan)
    return plan, M, Cv


def test_mix_is_bitwise_equal_to_alone_and_batches():
    import paper_2204_03893_amd as qxa
    srv = qxa.Server(max_inflight=64, n_streams=4, batch_tile_limit=512)
    srv.pause(True)
    jobs = {}
    meshes = []
    for si, (dim, order, N) in enumerate(SHAPES):
        for mi in range(2):
            m = _mesh(dim, order, N, seed=100 + 10 * si + mi)
            mo = qxa.Mesh(dim, order, m["coords"], m["conn"])
            r = rule(dim, 2 * order)
            meshes.append((m, mo, r))
            for k in range(3):
                u = torch.tensor(_field(m, 1000 + 100 * si + 10 * mi + k), device="cuda")
                t = srv.submit(mo, r, r, LAW_M, LAW_C, u, u, precision="fp64", tag=len(jobs))
                jobs[t] = (m, mo, r, u)
    print("submitted", len(jobs), "jobs", flush=True)
    srv.pause(False)
    done = srv.wait(len(jobs))
    st = srv.stats()
    print("stats", st, flush=True)
    assert all(c["status"] == 0 for c in done), [c["message"] for c in done if c["status"]]
    assert st["max_batch"] > 1 and st["batched_launches"] >= 1
    assert st["plan_builds"] == len(meshes)
    checked_oracle = 0
    for c in done:
        m, mo, r, u = jobs[c["ticket"]]
        Ms, Cs = srv.result(c["ticket"])
        plan, Ma, Ca = _alone(qxa, mo, r, u)
        torch.cuda.synchronize()
        assert torch.equal(Ms.view(torch.int64), Ma.view(torch.int64)), c
        assert torch.equal(Cs.view(torch.int64), Ca.view(torch.int64)), c
        if c["batched"] > 1 and checked_oracle < 3:
            uh = u.cpu().numpy()
            rp, ci, Mo, Co = oracle.assemble(m, r, r, LAW_M, LAW_C, uh, uh)
            assert row_scaled_error(Ms.cpu().numpy(), Mo, rp) <= 1e-12
            assert row_scaled_error(Cs.cpu().numpy(), Co, rp) <= 1e-12
            checked_oracle += 1
        srv.release(c["ticket"])
        plan.close()
    assert checked_oracle >= 1
    assert srv.stats()["bytes_in_use"] <= st["budget_bytes"]
    srv.close()


def test_cache_hit_equals_miss_and_pattern():
    import paper_2204_03893_amd as qxa
    srv = qxa.Server()
    m = _mesh(3, 2, 3, seed=7)
    mo = qxa.Mesh(3, 2, m["coords"], m["conn"])
    r = rule(3, 4)
    u = torch.tensor(_field(m, 8), device="cuda")
    t1 = srv.submit(mo, r, r, LAW_M, LAW_C, u, u)
    c1 = srv.wait(1)[0]
    t2 = srv.submit(mo, r, r, LAW_M, LAW_C, u, u)
    c2 = srv.wait(1)[0]
    assert (c1["ticket"], c2["ticket"]) == (t1, t2)
    assert c1["status"] == 0 and c2["status"] == 0
    assert not c1["plan_cached"] and c2["plan_cached"]
    M1, C1 = srv.result(t1)
    M2, C2 = srv.result(t2)
    torch.cuda.synchronize()
    assert torch.equal(M1.view(torch.int64), M2.view(torch.int64))
    assert torch.equal(C1.view(torch.int64), C2.view(torch.int64))
    rp, ci = oracle.pattern(m)
    assert c1["nnz"] == ci.size
    st = srv.stats()
    assert st["plan_hits"] == 1 and st["plan_builds"] == 1
    srv.release(t1)
    srv.release(t2)
    srv.close()


def test_tight_budget_queues_and_never_exceeds():
    import paper_2204_03893_amd as qxa
    shapes = [(2, 2, 10), (3, 1, 6), (2, 1, 16)]
    meshes = []
    for k, (dim, order, N) in enumerate(shapes):
        m = _mesh(dim, order, N, seed=50 + k)
        meshes.append((m, qxa.Mesh(dim, order, m["coords"], m["conn"]), rule(dim, 2 * order)))
    # budget: the largest plan plus about two jobs' buffers
    sizes = []
    for m, mo, r in meshes:
        p = qxa.Plan(mo, r)
        sizes.append((p.device_bytes, 16 * p.nnz + 16 * p.n_partials))
        p.close()
    budget = max(a for a, _ in sizes) + 2 * max(b for _, b in sizes) + (64 << 10)
    print("budget", budget, sizes, flush=True)
    srv = qxa.Server(hbm_budget=budget, max_inflight=8)
    want = {}
    for rep in range(4):
        for m, mo, r in meshes:
            u = torch.tensor(_field(m, 300 + rep), device="cuda")
            t = srv.submit(mo, r, r, LAW_M, LAW_C, u, u)
            want[t] = (mo, r, u)
    got = 0
    import time
    t0 = time.perf_counter()
    while got < len(want):
        cs = srv.poll()
        for c in cs:
            assert c["status"] == 0, c["message"]
            mo, r, u = want[c["ticket"]]
            Ms, Cs = srv.result(c["ticket"])
            plan, Ma, Ca = _alone(qxa, mo, r, u)
            torch.cuda.synchronize()
            assert torch.equal(Ms.view(torch.int64), Ma.view(torch.int64))
            assert torch.equal(Cs.view(torch.int64), Ca.view(torch.int64))
            plan.close()
            srv.release(c["ticket"])
            got += 1
        if not cs:
            assert time.perf_counter() - t0 < 60, srv.stats()
            time.sleep(0.0005)
    st = srv.stats()
    print("stats", st, flush=True)
    assert st["peak_bytes"] <= budget
    assert st["completed"] == len(want)
    # a job whose buffers cannot fit even in an empty budget fails alone
    big = _mesh(2, 2, 40, seed=9)
    mb = qxa.Mesh(2, 2, big["coords"], big["conn"])
    u = torch.tensor(_field(big, 1), device="cuda")
    t = srv.submit(mb, rule(2, 4), rule(2, 4), LAW_M, LAW_C, u, u)
    m0, mo0, r0 = meshes[0]
    u0 = torch.tensor(_field(m0, 2), device="cuda")
    t_ok = srv.submit(mo0, r0, r0, LAW_M, LAW_C, u0, u0)
    cs = {c["ticket"]: c for c in srv.wait(2)}
    assert cs[t]["status"] == -5, cs[t]
    assert cs[t_ok]["status"] == 0
    srv.release(t)
    srv.release(t_ok)
    assert srv.stats()["peak_bytes"] <= budget
    srv.close()


def test_nonfinite_field_fails_only_its_job():
    import paper_2204_03893_amd as qxa
    srv = qxa.Server()
    srv.pause(True)
    m = _mesh(2, 2, 5, seed=3)
    mo = qxa.Mesh(2, 2, m["coords"], m["conn"])
    r = rule(2, 4)
    good = torch.tensor(_field(m, 4), device="cuda")
    bad = good.clone()
    bad[7] = float("nan")
    tg = srv.submit(mo, r, r, LAW_M, LAW_C, good, good)
    tb = srv.submit(mo, r, r, LAW_M, LAW_C, bad, bad)
    srv.pause(False)
    cs = {c["ticket"]: c for c in srv.wait(2)}
    assert cs[tb]["status"] == -4 and cs[tg]["status"] == 0
    assert cs[tg]["batched"] == 2
    plan, Ma, Ca = _alone(qxa, mo, r, good)
    Ms, Cs = srv.result(tg)
    torch.cuda.synchronize()
    assert torch.equal(Ms.view(torch.int64), Ma.view(torch.int64))
    srv.release(tg)
    srv.release(tb)
    plan.close()
    srv.close()


def test_release_right_after_result_keeps_the_copied_values():
    """result() queues the copy on the caller's stream; release() right after it, with
    no synchronisation, must not let the next job (which takes the freed buffer, first
    fit) overwrite the values before the copy has read them."""
    import paper_2204_03893_amd as qxa
    srv = qxa.Server(max_inflight=4, n_streams=2)
    m = _mesh(2, 2, 6, seed=7)
    mo = qxa.Mesh(2, 2, m["coords"], m["conn"])
    r = rule(2, 4)
    u1 = torch.tensor(_field(m, 71), device="cuda")
    u2 = torch.tensor(_field(m, 72), device="cuda")
    t1 = srv.submit(mo, r, r, LAW_M, LAW_C, u1, u1)
    c1 = srv.wait(1)[0]
    assert c1["status"] == 0
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        torch.cuda._sleep(50_000_000)     # holds back the copy queued behind it on `side`
    M1, C1 = srv.result(t1, stream=side)
    srv.release(t1)                       # no synchronisation of `side` before this
    t2 = srv.submit(mo, r, r, LAW_M, LAW_C, u2, u2)
    c2 = srv.wait(1)[0]
    assert c2["status"] == 0 and c2["ticket"] == t2
    side.synchronize()
    plan, Ma, Ca = _alone(qxa, mo, r, u1)
    torch.cuda.synchronize()
    assert torch.equal(M1.view(torch.int64), Ma.view(torch.int64))
    assert torch.equal(C1.view(torch.int64), Ca.view(torch.int64))
    srv.release(t2)
    plan.close()
    srv.close()


def test_jobs_submitted_mid_flight_match_alone_bitwise():
    """Jobs submitted while others are queued or running (no pause), some on meshes the
    server has not seen (their plans are built while other jobs run), in FP64 and FP32:
    each result is bitwise equal to the same job assembled alone. A new mesh's plans are
    freed by drop_mesh once its jobs are released (QXA_E_BUSY before)."""
    import time
    import paper_2204_03893_amd as qxa
    srv = qxa.Server(max_inflight=16, n_streams=4, batch_tile_limit=512)
    rng = np.random.default_rng(77)
    specs = []
    big = _mesh(3, 2, 9, seed=300)
    specs.append((big, qxa.Mesh(3, 2, big["coords"], big["conn"]), rule(3, 4)))
    for si, (dim, order, N) in enumerate(SHAPES):
        m = _mesh(dim, order, N + 1, seed=310 + si)
        specs.append((m, qxa.Mesh(dim, order, m["coords"], m["conn"]), rule(dim, 2 * order)))
    jobs, mid_flight, new_meshes = {}, 0, []

    def submit(m, mo, r, precision, seed):
        nonlocal mid_flight
        st = srv.stats()
        mid_flight += (st["in_flight"] + st["queued"]) > 0
        u = torch.tensor(_field(m, seed), device="cuda")
        t = srv.submit(mo, r, r, LAW_M, LAW_C, u, u, precision=precision, tag=len(jobs))
        jobs[t] = (mo, r, u, precision)

    submit(*specs[0], "fp64", 400)
    results = {}
    for wave in range(4):
        for k in range(len(specs)):
            m, mo, r = specs[int(rng.integers(1, len(specs)))]
            submit(m, mo, r, "fp64" if k % 2 == 0 else "fp32", 500 + 10 * wave + k)
        # a mesh the server has not seen, submitted while the others run
        dim, order, N = SHAPES[wave % len(SHAPES)]
        m = _mesh(dim, order, N + 2, seed=600 + wave)
        mo = qxa.Mesh(dim, order, m["coords"], m["conn"])
        new_meshes.append(mo)
        submit(m, mo, rule(dim, 2 * order), "fp64", 700 + wave)
        for c in srv.poll():
            results[c["ticket"]] = c
        time.sleep(0.002)
    while len(results) < len(jobs):
        for c in srv.wait(1, timeout_s=120):
            results[c["ticket"]] = c
    print("mid-flight submissions", mid_flight, "of", len(jobs), srv.stats(), flush=True)
    assert mid_flight >= len(jobs) // 2
    cold = [c for c in results.values() if not c["plan_cached"]]
    assert cold and all(c["plan_ms"] > 0.0 for c in cold)
    with pytest.raises(qxa.QxaError) as ei:       # its jobs are not released yet
        srv.drop_mesh(new_meshes[0])
    assert ei.value.code == -8
    plans = {}
    for t, c in results.items():
        assert c["status"] == 0, c
        mo, r, u, precision = jobs[t]
        M, Cv = srv.result(t)
        torch.cuda.synchronize()
        srv.release(t)
        key = id(mo)
        if key not in plans:
            plans[key] = qxa.Plan(mo, r)
        Ma, Ca = qxa.assemble(plans[key], LAW_M, LAW_C, u, u, precision=precision)
        qxa.sync(plans[key])
        assert torch.equal(M.view(torch.int64), Ma.view(torch.int64)), (t, precision)
        assert torch.equal(Cv.view(torch.int64), Ca.view(torch.int64)), (t, precision)
    for mo in new_meshes:
        srv.drop_mesh(mo)
    srv.close()


def test_run_plans_batched_match_alone_bitwise():
    """3D P3 plans with runs (one chain of 4-tile runs per workgroup) batched into one
    launch: 768 chains on 256 workgroups, each walking three chains one after another.
    Every job is bitwise equal to the same job assembled alone, and matches the oracle."""
    import paper_2204_03893_amd as qxa
    srv = qxa.Server(max_inflight=8, n_streams=1, batch_tile_limit=1 << 20, hbm_budget=8 << 30)
    srv.pause(True)
    m = _mesh(3, 3, 14, seed=160)
    mo = qxa.Mesh(3, 3, m["coords"], m["conn"])
    r = rule(3, 6)
    jobs = {}
    for k in range(3):
        u = torch.tensor(_field(m, 161 + k), device="cuda")
        jobs[srv.submit(mo, r, r, LAW_M, LAW_C, u, u, precision="fp64", tag=k)] = u
    print("submitted 3D P3 run-plan jobs", flush=True)
    srv.pause(False)
    done = srv.wait(len(jobs))
    assert all(c["status"] == 0 for c in done), [c["message"] for c in done if c["status"]]
    assert srv.stats()["max_batch"] > 1
    for i, c in enumerate(done):
        u = jobs[c["ticket"]]
        Ms, Cs = srv.result(c["ticket"])
        plan, Ma, Ca = _alone(qxa, mo, r, u)
        assert plan.n_chains == 256 and plan.n_carry_reads > 0
        torch.cuda.synchronize()
        assert torch.equal(Ms.view(torch.int64), Ma.view(torch.int64))
        assert torch.equal(Cs.view(torch.int64), Ca.view(torch.int64))
        if i == 0:
            uh = u.cpu().numpy()
            rp, ci, Mo, Co = oracle.assemble(m, r, r, LAW_M, LAW_C, uh, uh)
            assert row_scaled_error(Ms.cpu().numpy(), Mo, rp) <= 1e-12
            assert row_scaled_error(Cs.cpu().numpy(), Co, rp) <= 1e-12
        srv.release(c["ticket"])
        plan.close()
    srv.close()
