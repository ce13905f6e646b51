"""Benchmark: element-matrix entries assembled per second on one MI355X.

One step = one full assembly of the mass and conductivity matrices (geometry,
coefficients at quadrature nodes, Lambda, X, V = Q X, deterministic scatter
into CSR). Default workload: 2D P3 triangles on the 1024^2 square (2,097,152
elements, 9,443,329 nodes), jitter 0.25h, 12-point rule, conductivity
c(x) = exp(g(x)) with g a smooth Gaussian random field, mass m = 1, FP64.
Inputs are resident in HBM before timing; the plan (pattern, tile plan) is
built once and reported separately.

Prints one JSON line (rank 0). Extra objects: "roofline" for the dominant
kernel (its algorithmic bytes per launch / its HIP-event duration vs 8 TB/s,
with the whole path's floor bytes / time per assembly beside it) and
"cpu_baseline" (the CPU oracle on the host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(kernel, w, plan, mesh):
    """Algorithmic bytes of one launch of `kernel`; the kernels' shares add up to the
    path floor (floor_bytes).

    fused: the inputs once, the element-entry -> slot map at 4 B per element entry,
    and every CSR value the fused kernel writes (all slots but the shared ones).
    fixup: the CSR values of the shared slots (both triangles), which it writes.
    Partial sums are design overhead, not algorithmic bytes.
    """
    fb = floor_bytes(w, plan, mesh)
    if kernel == "fused":
        return fb - 16 * plan.n_fix_slots
    if kernel == "fixup":
        return 16 * plan.n_fix_slots
    raise KeyError(kernel)


def floor_bytes(w, plan, mesh):
    """Whole-path floor: inputs once, the element-entry -> slot map once (4 B per
    element entry), both CSR value arrays written once."""
    d, ne, nn, npl, nnz = w.dim, plan.n_elem, plan.n_nodes, plan.n_p, plan.nnz
    n_vert = int(mesh["vertex_mask"].sum())
    return 4 * npl * ne + 8 * d * n_vert + 8 * nn + 4 * ne * npl * npl + 16 * nnz


KERNEL_SOURCES = ("paper_2204_03893_amd/csrc/kernels_fused.hip", "paper_2204_03893_amd/csrc/kernels_common.hpp",
                  "paper_2204_03893_amd/csrc/kernels.hpp", "paper_2204_03893_amd/csrc/plan_format.hpp",
                  "paper_2204_03893_amd/csrc/tiles.cpp")


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch from the committed counter summary, if it was taken
    with the kernel sources as they are now (else None)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()[:16]
    path = os.path.join(ROOT, "profiles", f"fused_{workload}.md")
    if not os.path.exists(path):
        return None
    pat = re.compile(r"traffic (\S+) (\S+) (\S+): bytes=(\d+) sources=([0-9a-f]+)")
    for line in open(path):
        m = pat.search(line)
        if m and m.group(2) == workload and m.group(3) == precision and m.group(5) == digest and \
                kernel == "fused" and m.group(1).startswith("fused"):
            return int(m.group(4))
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, mesh, rule, u):
    """The oracle on the host: one full assembly of the same workload with all the threads
    this process may use (at most 16, the host share of one GPU) and one with a single thread.
    Formation (element matrices) and assembly (global CSR sums) are timed separately inside
    the oracle, as the paper times them (Section 6.1); the CSR pattern, built once per mesh
    like the GPU plan, is left out of both. value = entries / (formation + assembly)."""
    import oracle
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    threads = max(1, min(avail, 16))
    entries = 2 * mesh["conn"].shape[1] * mesh["conn"].shape[0] ** 2
    runs = {}
    for th in (threads, 1):
        t0 = time.perf_counter()
        oracle.assemble(mesh, rule, rule, w.mass_law, w.stiff_law, u, u, nthreads=th)
        wall = time.perf_counter() - t0
        f, a = oracle.last_timing()
        runs[th] = {"threads": th, "formation_s": f, "assembly_s": a, "call_wall_s": wall,
                    "entries_per_s": entries / (f + a), "formation_entries_per_s": entries / f}
    allr = runs[threads]
    return {"value": allr["entries_per_s"], "unit": "entries/s", "cores": threads, "kind": "oracle",
            "sample": f"one full assembly of the same workload ({w.name}) per thread count; formation and "
                      f"assembly timed inside the oracle, pattern build excluded",
            "nproc": os.cpu_count(), "affinity_cpus": avail, "cpu_model": cpu_model(),
            "formation_s": allr["formation_s"], "assembly_s": allr["assembly_s"],
            "single_thread": runs[1]}


def serving_pool(n_pool, max_elements, seed=2204):
    """Heterogeneous request meshes: (dim, order) uniform over {2,3} x {1,2,3}, element count
    log-uniform on [1e3, max_elements] (the first mesh at max_elements), interior vertices
    jittered by 0.2h; per mesh four smooth random fields (16 random Fourier features),
    conductivity exp(g) or 1 + g^2, mass 1, and the rule exact to degree 2P for both matrices."""
    import numpy as np
    from workloads import rule, structured_mesh
    from workloads.fields import gaussian_random_field
    rng = np.random.default_rng([seed, 5])
    out = []
    for k in range(n_pool):
        dim = int(rng.integers(2, 4))
        order = int(rng.integers(1, 4))
        ne = float(np.exp(rng.uniform(np.log(1e3), np.log(max_elements)))) if k else max_elements
        N = max(2, int(round((ne / 2) ** 0.5 if dim == 2 else (ne / 6) ** (1 / 3))))
        m = structured_mesh(dim, order, N, 0.2, seed=[seed, 6, k])
        fields = [gaussian_random_field(m["coords"], 16, np.random.default_rng([seed, 7, k, j]), length=0.1)
                  for j in range(4)]
        law = ("exp", 0.0, 1.0) if rng.uniform() < 0.5 else ("poly2", 1.0, 0.0, 1.0)
        out.append({"mesh": m, "dim": dim, "order": order, "rule": rule(dim, 2 * order), "fields": fields,
                    "law_c": law, "entries": 2 * m["conn"].shape[1] * m["conn"].shape[0] ** 2})
    return out


def serving(args):
    """Serving run: requests pick a pool geometry and one of its fields at random; a
    fraction new_mesh_fraction of them bring a new mesh (a fresh mesh object the server has
    no plan for, built on the server's builder thread while other jobs run, and dropped after
    the job), the others reuse a resident mesh (plans cached by a warm-up pass). Loads:
    saturation (all queued at once), then Poisson arrivals at 50% and 80% of the saturation
    rate. Latency = completion seen by the server - scheduled arrival; cold (new mesh) and
    warm requests are reported apart, with the plan-build share of the cold ones. Prints one
    JSON line."""
    import numpy as np
    import torch
    import paper_2204_03893_amd as qxa
    t0 = time.perf_counter()
    pool = serving_pool(args.pool, args.max_elements)
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda", 0)
    srv = qxa.Server(hbm_budget=int(args.budget_gib) << 30, max_inflight=64, n_streams=4, batch_tile_limit=512)
    for p in pool:
        m = p["mesh"]
        p["obj"] = qxa.Mesh(p["dim"], p["order"], m["coords"], m["conn"])
        p["dev_fields"] = [torch.tensor(f, device=dev) for f in p["fields"]]
    # warm-up: one job per resident mesh builds every plan (cold-miss cost, reported separately)
    t0 = time.perf_counter()
    for k, p in enumerate(pool):
        u = p["dev_fields"][0]
        srv.submit(p["obj"], p["rule"], p["rule"], ("const", 1.0), p["law_c"], u, u, precision=args.precision, tag=k)
    warm = srv.wait(len(pool), timeout_s=600)
    warm_s = time.perf_counter() - t0
    bad = [c for c in warm if c["status"] != 0]
    if bad:
        raise RuntimeError(f"serving warm-up failed: {bad[0]}")
    for c in warm:
        srv.release(c["ticket"])
    rng = np.random.default_rng([2204, 8])
    frac = args.new_mesh_fraction

    def pct(x, q):
        return float(np.percentile(x, q)) if len(x) else None

    def run(rate):
        n = args.requests
        picks = rng.integers(0, len(pool), size=n)
        fsel = rng.integers(0, 4, size=n)
        cold = rng.uniform(size=n) < frac
        gaps = rng.exponential(1.0 / rate, size=n) if rate else np.zeros(n)
        sched = np.cumsum(gaps)
        lat, plan_ms, is_cold, waits, entries, done = [], [], [], [], 0, 0
        paused = not rate
        if paused:
            srv.pause(True)
        t_start = time.perf_counter()
        submit_late, fresh = {}, {}
        i = 0
        while done < n:
            now = time.perf_counter() - t_start
            while i < n and sched[i] <= now:
                p = pool[picks[i]]
                u = p["dev_fields"][fsel[i]]
                mo = p["obj"]
                if cold[i]:  # the request brings its mesh: uploaded and checked now
                    m = p["mesh"]
                    mo = qxa.Mesh(p["dim"], p["order"], m["coords"], m["conn"])
                t = srv.submit(mo, p["rule"], p["rule"], ("const", 1.0), p["law_c"], u, u,
                               precision=args.precision, tag=i)
                if cold[i]:
                    fresh[t] = mo
                submit_late[t] = (time.perf_counter() - t_start - sched[i]) * 1e3
                i += 1
                now = time.perf_counter() - t_start
            if not rate and i == n and paused:
                srv.pause(False)
                paused = False
                t_start_sat = time.perf_counter()
            for c in srv.poll():
                if c["status"] != 0:
                    raise RuntimeError(f"serving request failed: {c}")
                lat.append(submit_late.pop(c["ticket"]) + c["total_ms"])
                plan_ms.append(c["plan_ms"])
                is_cold.append(c["ticket"] in fresh)
                waits.append(c["queue_ms"])
                entries += pool[picks[c["tag"]]]["entries"]
                srv.release(c["ticket"])
                if c["ticket"] in fresh:
                    mo = fresh.pop(c["ticket"])
                    srv.drop_mesh(mo)
                    mo.close()
                done += 1
            if i == n and done < n:
                time.sleep(0.0001)
        span = time.perf_counter() - (t_start_sat if not rate else t_start)
        lat, plan_ms, is_cold = np.array(lat), np.array(plan_ms), np.array(is_cold, dtype=bool)
        lc, lw = lat[is_cold], lat[~is_cold]
        return {"offered_jobs_per_s": rate, "jobs": n, "new_meshes": int(is_cold.sum()), "makespan_s": span,
                "jobs_per_s": n / span, "entries_per_s": entries / span,
                "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(lat.mean()),
                "cold": {"p50_ms": pct(lc, 50), "p99_ms": pct(lc, 99),
                         "mean_ms": float(lc.mean()) if lc.size else None,
                         "mean_plan_ms": float(plan_ms[is_cold].mean()) if lc.size else None,
                         "plan_share": float(plan_ms[is_cold].sum() / lc.sum()) if lc.size else None},
                "warm": {"p50_ms": pct(lw, 50), "p99_ms": pct(lw, 99),
                         "mean_ms": float(lw.mean()) if lw.size else None},
                "mean_queue_ms": float(np.mean(waits))}

    sat = run(0.0)
    loads = [run(f * sat["jobs_per_s"]) for f in (0.5, 0.8)]
    st = srv.stats()
    srv.close()
    sizes = [p["mesh"]["conn"].shape[1] for p in pool]
    out = {"metric": "serving element-matrix entries assembled/sec", "value": sat["entries_per_s"],
           "unit": "entries/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "dtype": "f64" if args.precision == "fp64" else args.precision, "vs_baseline": None,
           "config": {"workload": "serving mix", "pool_meshes": len(pool), "elements_min": min(sizes),
                      "elements_max": max(sizes), "requests_per_load": args.requests, "precision": args.precision,
                      "new_mesh_fraction": frac, "budget_gib": args.budget_gib},
           "saturation": sat, "loads": loads, "warmup_plan_builds_s": warm_s, "pool_generation_s": gen_s,
           "server": st}
    print(json.dumps(out))


def reassembly(args, n_steps=20):
    """Reassembly loop (only the coefficients change): the heat workload by default
    (p1_3d_96_heat, 5,308,416 elements). Each step updates the nodal field in place
    (u += 0.05 * smooth increment, a device add on the same stream) and replays the
    captured assembly graph; the same loop with direct assembly calls is timed beside it.
    Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2204_03893_amd as qxa
    from workloads import WORKLOADS, heat_increment, make_inputs
    name = args.workload if args.workload not in ("p2_3d_32", "p3_2d_1024") else "p1_3d_96_heat"
    w = WORKLOADS[name]
    mesh, rule, u0 = make_inputs(w)
    m = qxa.Mesh(w.dim, w.order, mesh["coords"], mesh["conn"])
    t0 = time.perf_counter()
    plan = qxa.Plan(m, rule)
    plan_s = time.perf_counter() - t0
    dev = torch.device("cuda", 0)
    u = torch.tensor(u0, device=dev)
    incs = [torch.tensor(heat_increment(w, mesh, s), device=dev) for s in range(1, n_steps + 1)]
    stream = torch.cuda.current_stream()
    g = qxa.ReassemblyGraph(plan, w.mass_law, w.stiff_law, u, u, precision=args.precision)
    M = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    Cv = torch.empty_like(M)

    def loop(use_graph):
        u.copy_(torch.tensor(u0, device=dev))
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for s in range(n_steps):
            u.add_(incs[s])
            if use_graph:
                g.launch(stream)
            else:
                qxa.assemble(plan, w.mass_law, w.stiff_law, u, u, precision=args.precision, M=M, Cv=Cv,
                             stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        qxa.sync(plan, stream)
        return ev0.elapsed_time(ev1) / n_steps

    loop(True)
    loop(False)  # warm-up
    ms_graph = loop(True)
    ms_direct = loop(False)
    same = bool(torch.equal(g.M.view(torch.int64), M.view(torch.int64)) and
                torch.equal(g.Cv.view(torch.int64), Cv.view(torch.int64)))
    entries = 2 * plan.n_elem * plan.n_p ** 2
    g.close()
    out = {"metric": "element-matrix entries assembled/sec (reassembly loop)", "value": entries / (ms_graph * 1e-3),
           "unit": "entries/s", "n_gpus": 1, "steps": n_steps, "ms_per_step": ms_graph, "higher_is_better": True,
           "dtype": "f64" if args.precision == "fp64" else args.precision, "data": "synthetic", "vs_baseline": None,
           "config": {"workload": w.name, "description": w.description, "n_elem": plan.n_elem, "nnz": plan.nnz,
                      "precision": args.precision},
           "ms_per_step_direct": ms_direct, "graph_equals_direct_bitwise": same, "plan_build_s": plan_s}
    print(json.dumps(out))


def tangent(args):
    """Mass tensor of the Newton Jacobian contracted with a nodal vector (Section 5):
    M o_2 w with m(u) = 1 + 0.5 u^2 (m' = u), w = u - u_prev, on the workload's mesh.
    One step = the per-node coefficient m'(u_h) w_h (qxa_coeff_product) plus the
    mass-matrix assembly of that coefficient into the CSR pattern. Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2204_03893_amd as qxa
    from workloads import WORKLOADS, make_inputs
    w = WORKLOADS[args.workload]
    mesh, rule, u0 = make_inputs(w)
    _, _, u1 = make_inputs(w, stream=1)
    dev = torch.device("cuda", 0)
    m = qxa.Mesh(w.dim, w.order, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rule)
    u = torch.tensor(u0, device=dev)
    wv = torch.tensor(u0 - u1, device=dev)
    law_dm = ("poly2", 0.0, 1.0, 0.0)
    stream = torch.cuda.current_stream()
    T = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    S = torch.empty((plan.n_q_mass, plan.n_elem), dtype=torch.float64, device=dev)

    def step():
        qxa.mass_tensor_product(plan, law_dm, u, wv, T=T, S=S, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    qxa.sync(plan, stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    qxa.sync(plan, stream)
    ms = ev0.elapsed_time(ev1) / args.steps
    # the coefficient kernel alone, then the assembly kernels' own events
    ev0.record(stream)
    for _ in range(args.steps):
        qxa.coeff_product(plan, law_dm, u, wv, S=S, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    k_coeff = ev0.elapsed_time(ev1) / args.steps
    plan.set_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    rep = plan.timing_report()
    plan.set_timing(False)
    kern = {k: v["ms"] / v["n"] for k, v in rep.items()}
    kern["coeff_product"] = k_coeff
    ne, npl, nn, nq = plan.n_elem, plan.n_p, plan.n_nodes, plan.n_q_mass
    n_vert = int(mesh["vertex_mask"].sum())
    ab = {"coeff_product": 4 * npl * ne + 16 * nn + 8 * nq * ne,
          "fused": 4 * npl * ne + 8 * w.dim * n_vert + 8 * nq * ne + 4 * ne * npl * npl + 8 * plan.nnz,
          "fixup": 8 * plan.n_partials + 16 * plan.n_shared}
    dom = max(kern, key=kern.get)
    achieved = ab[dom] / (kern[dom] * 1e-3) / 1e9
    entries = ne * npl ** 2
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(os.cpu_count() or 1, 16)
        t0 = time.perf_counter()
        reps = 0
        while reps < 30 and (reps == 0 or time.perf_counter() - t0 < 10):
            oracle.mass_tensor_product(mesh, rule, law_dm, u0, u0 - u1, nthreads=threads)
            reps += 1
        tot = time.perf_counter() - t0
        cpu = {"value": entries * reps / tot, "unit": "entries/s", "cores": threads, "kind": "oracle",
               "sample": f"{reps} full tensor products of the same workload ({w.name}), {tot:.1f} s"}
    # the conductivity tensor contracted in its second mode (c(u) = 1 + 0.5 u^2, c' = u)
    Tc = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    for _ in range(3):
        qxa.cond_tensor_product(plan, law_dm, u, wv, T=Tc, stream=stream)
    torch.cuda.synchronize()
    plan.set_timing(True)
    ev0.record(stream)
    for _ in range(args.steps):
        qxa.cond_tensor_product(plan, law_dm, u, wv, T=Tc, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    qxa.sync(plan, stream)
    ms_c = ev0.elapsed_time(ev1) / args.steps
    rep_c = plan.timing_report()
    plan.set_timing(False)
    cond = {"ms_per_product": ms_c, "entries_per_s": entries / (ms_c * 1e-3),
            "kernels_ms": {k: v["ms"] / v["n"] for k, v in rep_c.items()},
            "design": "two-pass: local matrices to HBM, then one thread per CSR slot"}
    # the volume load vector f_i = int f phi_i with f = exp(u_h)
    Fv = torch.empty(plan.n_nodes, dtype=torch.float64, device=dev)
    for _ in range(3):
        qxa.load_vector(plan, ("exp", 0.0, 1.0), u, F=Fv, stream=stream)
    torch.cuda.synchronize()
    plan.set_timing(True)
    ev0.record(stream)
    for _ in range(args.steps):
        qxa.load_vector(plan, ("exp", 0.0, 1.0), u, F=Fv, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    qxa.sync(plan, stream)
    ms_f = ev0.elapsed_time(ev1) / args.steps
    rep_f = plan.timing_report()
    plan.set_timing(False)
    load = {"ms_per_vector": ms_f, "element_entries_per_s": ne * npl / (ms_f * 1e-3),
            "kernels_ms": {k: v["ms"] / v["n"] for k, v in rep_f.items()}}
    # isoparametric elements (geometry per quadrature node): M and C with the workload's laws
    Mi = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    Ci = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    for _ in range(3):
        qxa.assemble_iso(plan, w.mass_law, w.stiff_law, u, u, M=Mi, Cv=Ci, stream=stream)
    torch.cuda.synchronize()
    plan.set_timing(True)
    ev0.record(stream)
    for _ in range(args.steps):
        qxa.assemble_iso(plan, w.mass_law, w.stiff_law, u, u, M=Mi, Cv=Ci, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    qxa.sync(plan, stream)
    ms_i = ev0.elapsed_time(ev1) / args.steps
    rep_i = plan.timing_report()
    plan.set_timing(False)
    iso = {"ms_per_assembly": ms_i, "entries_per_s": 2 * entries / (ms_i * 1e-3),
           "kernels_ms": {k: v["ms"] / v["n"] for k, v in rep_i.items()},
           "design": ("one pass: the matrix-core kernel with X formed per quadrature node (B_q from every "
                      "node's position), V = QX in LDS, the plan's units, then the fix-up"
                      if "fused_iso" in rep_i else
                      "two passes: X per quadrature node and V = QX through LDS, pair-major per 64 tile "
                      "positions to HBM, then the fused reduction (the plan's units, chains, carries) and "
                      "the fix-up")}
    out = {"metric": "mass-tensor product entries assembled/sec", "value": entries / (ms * 1e-3),
           "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": w.name + " tensor product", "n_elem": ne, "nnz": plan.nnz,
                      "law_dm": list(law_dm), "entries_per_step": entries},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom,
                        "algorithmic_bytes": ab[dom], "kernel_ms": kern[dom]},
           "kernels_ms": kern, "cpu_baseline": cpu, "cond_tensor_product": cond, "load_vector": load,
           "isoparametric": iso}
    print(json.dumps(out))


def paper_sweep(args):
    """Paper-shaped stand-in for Experiment 1 (Section 6.1): the unit square, P1 and P2
    triangles, constant coefficients, the fewest-point rules exact for them (P1: mass 3
    points, conductivity 1; P2: mass 6 points, conductivity 3), mesh sizes close to the
    paper's six meshes. Times the mass matrix alone, the conductivity matrix alone and both
    (formation + scatter into CSR, plan built beforehand). Context for the paper's tables,
    not a target. Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2204_03893_amd as qxa
    from workloads import rule, structured_mesh
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    rules = {1: (rule(2, 2), rule(2, 1)), 2: (rule(2, 4), rule(2, 2))}
    rows = []
    for order in (1, 2):
        for N in (23, 46, 92, 183, 368, 736):
            mesh = structured_mesh(2, order, N, 0.0)
            m = qxa.Mesh(2, order, mesh["coords"], mesh["conn"])
            t0 = time.perf_counter()
            plan = qxa.Plan(m, *rules[order])
            build_s = time.perf_counter() - t0
            M = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
            Cv = torch.empty_like(M)
            res = {"order": order, "N": N, "n_elem": plan.n_elem, "n_nodes": plan.n_nodes, "nnz": plan.nnz,
                   "plan_build_s": build_s}
            for name, wm, wc in (("mass_ms", True, False), ("cond_ms", False, True), ("both_ms", True, True)):
                def once():
                    qxa.assemble(plan, ("const", 1.0), ("const", 1.0), M=M, Cv=Cv, stream=stream,
                                 want_m=wm, want_c=wc)
                for _ in range(5):
                    once()
                torch.cuda.synchronize()
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
                for _ in range(args.steps):
                    once()
                ev1.record(stream)
                torch.cuda.synchronize()
                res[name] = ev0.elapsed_time(ev1) / args.steps
            qxa.sync(plan, stream)
            res["entries_per_s_both"] = 2 * plan.n_elem * plan.n_p ** 2 / (res["both_ms"] * 1e-3)
            rows.append(res)
            print(json.dumps(res), file=sys.stderr, flush=True)
            del plan, m
    # Experiment 2 stand-in (Section 6.2): 2D P2 on 43 x 43 cells (3,698 triangles), mass
    # coefficient c rho = 2.4e6, a conductivity linear in the temperature (the paper's law is
    # piecewise linear; not among the library's laws), 2,757 reassemblies replayed from a graph
    # while the temperature field is updated in place
    from workloads.fields import random_sinusoids
    mesh = structured_mesh(2, 2, 43, 0.0)
    m = qxa.Mesh(2, 2, mesh["coords"], mesh["conn"])
    plan = qxa.Plan(m, rule(2, 4))
    rng = np.random.default_rng([2204, 62])
    T = torch.tensor(300.0 + 50.0 * random_sinusoids(mesh["coords"], 8, rng), device=dev)
    dT = torch.tensor(0.01 * random_sinusoids(mesh["coords"], 4, rng), device=dev)
    g = qxa.ReassemblyGraph(plan, ("const", 2.4e6), ("poly2", 54.0, -0.033, 0.0), None, T)
    n_rep = 2757
    for _ in range(5):
        g.launch(stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(n_rep):
        T.add_(dT)
        g.launch(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    qxa.sync(plan, stream)
    exp2 = {"n_elem": plan.n_elem, "n_nodes": plan.n_nodes, "reassemblies": n_rep,
            "ms_per_reassembly": ev0.elapsed_time(ev1) / n_rep, "total_ms": ev0.elapsed_time(ev1)}
    g.close()
    big = [r for r in rows if r["order"] == 2 and r["N"] == 736][0]
    out = {"metric": "element-matrix entries assembled/sec (paper-shaped sweep, context)",
           "value": big["entries_per_s_both"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic", "vs_baseline": None,
           "config": {"workload": "unit square, 2D P1/P2, constant coefficients, N = 23..736"},
           "p2_736_mass_matrix_ms": big["mass_ms"], "rows": rows, "exp2_standin": exp2}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="p3_2d_1024")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip timing the other precision forms")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) to calibrate HBM byte counters")
    ap.add_argument("--mode", choices=("assemble", "serving", "reassembly", "tangent", "paper"), default="assemble")
    ap.add_argument("--requests", type=int, default=300, help="serving: requests per offered load")
    ap.add_argument("--new-mesh-fraction", type=float, default=0.7,
                    help="serving: share of requests that bring a mesh the server has not seen")
    ap.add_argument("--pool", type=int, default=48, help="serving: resident meshes")
    ap.add_argument("--max-elements", type=float, default=1e6, help="serving: largest mesh (elements)")
    ap.add_argument("--budget-gib", type=int, default=160, help="serving: device memory budget of the server (GiB)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU sharding is a design "
              "note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}))
        return

    if args.mode == "serving":
        serving(args)
        return
    if args.mode == "reassembly":
        reassembly(args)
        return
    if args.mode == "tangent":
        tangent(args)
        return
    if args.mode == "paper":
        paper_sweep(args)
        return

    import paper_2204_03893_amd as qxa
    from workloads import WORKLOADS, make_inputs

    w = WORKLOADS[args.workload]
    mesh, rule, u = make_inputs(w)
    dev = torch.device("cuda", 0)
    m = qxa.Mesh(w.dim, w.order, mesh["coords"], mesh["conn"])
    t0 = time.perf_counter()
    plan = qxa.Plan(m, rule)
    plan_s = time.perf_counter() - t0
    uf = torch.tensor(u, device=dev)
    M = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    Cv = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        qxa.assemble(plan, w.mass_law, w.stiff_law, uf, uf, precision=args.precision, M=M, Cv=Cv, stream=stream)

    for _ in range(args.warmup):
        step()
    qxa.sync(plan, stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    qxa.sync(plan, stream)
    ms = ev0.elapsed_time(ev1) / args.steps

    # per-kernel durations with events recorded by the library on the launch stream
    plan.set_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    rep = plan.timing_report()
    plan.set_timing(False)
    kern = {k: v["ms"] / v["n"] for k, v in rep.items()}
    dom = max(kern, key=kern.get)

    # single assemblies between events: warm, and after writing 1 GiB so that the
    # 256 MB MALL holds none of the assembly's data (median, p10, p90 of the reps)
    def single_reps(n, flush):
        scratch = torch.empty(1 << 27, dtype=torch.float64, device=dev) if flush else None
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for k in range(n):
            if flush:
                scratch.fill_(float(k))
            a.record(stream)
            step()
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        del scratch
        q = np.percentile(ts, [10, 50, 90])
        return {"reps": n, "p10_ms": float(q[0]), "median_ms": float(q[1]), "p90_ms": float(q[2])}

    n_single = max(1, min(50, args.steps))
    single = {"warm": single_reps(n_single, False), "mall_flushed": single_reps(n_single, True)}
    qxa.sync(plan, stream)
    ab = algorithmic_bytes(dom, w, plan, mesh)
    achieved = ab / (kern[dom] * 1e-3) / 1e9
    entries = 2 * plan.n_elem * plan.n_p ** 2
    fb = floor_bytes(w, plan, mesh)
    per_kernel = {}
    for k, t in kern.items():
        b = algorithmic_bytes(k, w, plan, mesh)
        per_kernel[k] = {"ms": t, "algorithmic_bytes": b, "achieved_gbs": b / (t * 1e-3) / 1e9,
                         "frac": b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
    path = {"bytes": fb, "ms": ms, "achieved_gbs": fb / (ms * 1e-3) / 1e9,
            "frac": fb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    # every precision form of the kernel on the same workload: time per assembly and
    # row-scaled error against this run's FP64 values (max_ij |v - v64| / max_k |v64_ik|;
    # the FP64 path itself is held to 1e-12 of the oracle by the test suite)
    forms = {}
    if not args.no_forms:
        rp, _ = plan.pattern()
        rows = torch.repeat_interleave(torch.arange(plan.n_nodes, device=dev), torch.diff(rp))
        M64, C64 = torch.empty_like(M), torch.empty_like(Cv)
        qxa.assemble(plan, w.mass_law, w.stiff_law, uf, uf, precision="fp64", M=M64, Cv=C64, stream=stream)

        def row_err(x, ref):
            rmax = torch.zeros(plan.n_nodes, dtype=torch.float64, device=dev)
            rmax.scatter_reduce_(0, rows, ref.abs(), reduce="amax")
            rmax = torch.where(rmax == 0, torch.ones_like(rmax), rmax)
            return float(((x - ref).abs() / rmax[rows]).max())

        M2, C2 = torch.empty_like(M), torch.empty_like(Cv)
        for form in ("fp64", "fp32", "f16x2", "bf16x3", "bf16x2"):
            def fstep():
                qxa.assemble(plan, w.mass_law, w.stiff_law, uf, uf, precision=form, M=M2, Cv=C2, stream=stream)
            try:
                fstep()
            except qxa.QxaError as e:
                forms[form] = {"supported": False, "reason": str(e)}
                continue
            n_f = max(1, min(50, args.steps))
            for _ in range(3):
                fstep()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(n_f):
                fstep()
            b.record(stream)
            torch.cuda.synchronize()
            qxa.sync(plan, stream)
            forms[form] = {"supported": True, "ms": a.elapsed_time(b) / n_f, "steps": n_f,
                           "row_scaled_err_vs_fp64": {"M": row_err(M2, M64), "C": row_err(C2, C64)}}
        del rows, M64, C64, M2, C2

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, mesh, rule, u)

    out = {
        "metric": "element-matrix entries assembled/sec",
        "value": entries / (ms * 1e-3),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else args.precision,
        "data": "synthetic",
        "config": {"workload": w.name, "description": w.description, "n_elem": plan.n_elem,
                   "n_nodes": plan.n_nodes, "nnz": plan.nnz, "entries_per_step": entries,
                   "precision": args.precision, "n_tiles": plan.n_tiles, "n_shared": plan.n_shared,
                   "n_partials": plan.n_partials, "n_outputs": plan.n_outputs, "n_units": plan.n_units,
                   "n_pair_units": plan.n_pair_units,
                   "n_chains": plan.n_chains, "n_carry_reads": plan.n_carry_reads, "carry_cap": plan.carry_cap,
                   "carry_used": plan.carry_used, "n_fix_slots": plan.n_fix_slots,
                   "n_ext_units": plan.n_ext_units},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, w.name, args.precision), "kernel": dom,
                     "algorithmic_bytes": ab, "kernel_ms": kern[dom], "path": path, "per_kernel": per_kernel},
        "path_floor": {"bytes": fb, "frac_of_hbm_peak": path["frac"]},
        "kernels_ms": kern,
        "precision_forms": forms,
        "single_assembly": single,
        "plan_build_s": plan_s,
        "wall_s_timed_region": wall,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
