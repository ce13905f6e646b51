"""Python binding of libqxa (loop-free FEM assembly, V = Q X, on MI355X).

Argument marshalling only: every step of the assembly runs in the HIP
kernels of libqxa.so. torch is used for device memory and streams. There is
no CPU fallback: if the library is not built, importing the binding's
functions raises.

Coefficient laws are tuples:
    ("const", value) | ("identity",) | ("poly2", a0, a1, a2) | ("exp", a0, a1)
and a non-constant law takes a device field: nodal values [n_nodes] (the law
is applied to u_h = phi^T u at each quadrature node), or values per
quadrature node [n_q, n_elem] with qpoint=True.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqxa.so")

FP64, FP32, F16X2, BF16X2, BF16X3 = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "f16x2": F16X2, "bf16x2": BF16X2, "bf16x3": BF16X3}
_LAW = {"identity": 0, "poly2": 1, "exp": 2}


class QxaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qxa error {code}: {msg}")
        self.code = code


class _Quad(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_q", C.c_int), ("points", C.c_void_p), ("weights", C.c_void_p)]


class _Coeff(C.Structure):
    _fields_ = [("kind", C.c_int), ("law", C.c_int), ("value", C.c_double), ("a", C.c_double * 3),
                ("field", C.c_void_p), ("tensor", C.c_void_p), ("tensor_q", C.c_void_p)]


class _PlanInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("order", C.c_int), ("n_p", C.c_int), ("n_q_mass", C.c_int),
                ("n_q_stiff", C.c_int), ("n_nodes", C.c_int64), ("n_elem", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("device_bytes", C.c_size_t),
                ("build_ms", C.c_double), ("n_tiles", C.c_int64), ("n_shared", C.c_int64),
                ("n_partials", C.c_int64), ("n_outputs", C.c_int64), ("n_units", C.c_int64), ("n_pair_units", C.c_int64),
                ("n_chains", C.c_int64), ("n_carry_reads", C.c_int64), ("n_fix_slots", C.c_int64),
                ("n_ext_units", C.c_int64), ("n_empty_units", C.c_int64), ("carry_cap", C.c_int),
                ("carry_used", C.c_int), ("n_q_mass_kernel", C.c_int), ("n_q_stiff_kernel", C.c_int)]


_TILE_FIELDS = ("nnz", "n_tiles", "n_shared", "n_partials", "n_outputs", "n_units", "n_pair_units", "n_chains",
                "n_carry_reads", "n_fix_slots", "n_ext_units", "n_empty_units", "carry_cap", "carry_used",
                "n_q_mass", "n_q_stiff", "n_q_mass_kernel", "n_q_stiff_kernel")


class _ServerOpts(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget_bytes", C.c_size_t), ("max_inflight", C.c_int),
                ("n_streams", C.c_int), ("batch_tile_limit", C.c_int64), ("queue_capacity", C.c_int),
                ("plan_cache_entries", C.c_int), ("plan_builders", C.c_int)]


class _Job(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("mass_rule", _Quad), ("stiff_rule", _Quad), ("mass", _Coeff),
                ("stiff", _Coeff), ("precision", C.c_int), ("user_tag", C.c_uint64)]


class _Completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("user_tag", C.c_uint64), ("status", C.c_int), ("plan_cached", C.c_int),
                ("batched", C.c_int), ("n_nodes", C.c_int64), ("nnz", C.c_int64), ("M", C.c_void_p),
                ("C", C.c_void_p), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("queue_ms", C.c_double),
                ("run_ms", C.c_double), ("total_ms", C.c_double), ("plan_ms", C.c_double),
                ("message", C.c_char * 160)]


SERVER_STATS = ("submitted", "completed", "plan_hits", "plan_builds", "evictions", "launches", "batched_launches",
                "max_batch", "bytes_in_use", "peak_bytes", "queued", "in_flight", "budget_bytes")

_lib = None


def lib():
    """Load libqxa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2204_03893_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64, ci = C.c_void_p, C.c_int64, C.c_int
        L.qxa_last_error.restype = C.c_char_p
        L.qxa_version.restype = C.c_char_p
        L.qxa_mesh_create.argtypes = [ci, ci, ci, i64, vp, i64, vp, ci, C.POINTER(vp)]
        L.qxa_mesh_destroy.argtypes = [vp]
        L.qxa_plan_create.argtypes = [vp, C.POINTER(_Quad), C.POINTER(_Quad), C.POINTER(vp)]
        L.qxa_plan_destroy.argtypes = [vp]
        L.qxa_plan_get_info.argtypes = [vp, C.POINTER(_PlanInfo)]
        L.qxa_plan_copy_pattern.argtypes = [vp, vp, vp, vp]
        L.qxa_quad_builtin.argtypes = [C.c_int, C.c_int, C.POINTER(_Quad)]
        L.qxa_pattern_host.argtypes = [ci, ci, i64, i64, vp, vp, vp, C.POINTER(i64)]
        L.qxa_plan_check_host.argtypes = [ci, ci, i64, vp, i64, vp, C.POINTER(_Quad), C.POINTER(_Quad), i64, ci,
                                          C.POINTER(_PlanInfo)]
        L.qxa_plan_check_host_corrupted.argtypes = [ci, ci, i64, vp, i64, vp, i64, ci, ci]
        L.qxa_assemble.argtypes = [vp, C.POINTER(_Coeff), C.POINTER(_Coeff), ci, vp, vp, vp]
        L.qxa_element_matrices.argtypes = [vp, C.POINTER(_Coeff), C.POINTER(_Coeff), ci, vp, vp, vp]
        L.qxa_element_matrices_noalloc.argtypes = [vp, C.POINTER(_Coeff), C.POINTER(_Coeff), ci, vp, vp, vp]
        L.qxa_coeff_product.argtypes = [vp, ci, C.POINTER(_Coeff), vp, vp, vp]
        L.qxa_cond_tensor_product.argtypes = [vp, C.POINTER(_Coeff), vp, vp, vp]
        L.qxa_load_vector.argtypes = [vp, C.POINTER(_Coeff), vp, vp]
        L.qxa_assemble_iso.argtypes = [vp, C.POINTER(_Coeff), C.POINTER(_Coeff), vp, vp, vp]
        L.qxa_sync.argtypes = [vp, vp]
        L.qxa_plan_set_timing.argtypes = [vp, ci]
        L.qxa_graph_create.argtypes = [vp, C.POINTER(_Coeff), C.POINTER(_Coeff), ci, vp, vp, C.POINTER(vp)]
        L.qxa_graph_launch.argtypes = [vp, vp]
        L.qxa_graph_destroy.argtypes = [vp]
        L.qxa_plan_timing_report.argtypes = [vp, C.c_char_p, C.c_size_t]
        L.qxa_server_create.argtypes = [C.POINTER(_ServerOpts), C.POINTER(vp)]
        L.qxa_server_submit.argtypes = [vp, C.POINTER(_Job), C.POINTER(C.c_uint64)]
        L.qxa_server_poll.argtypes = [vp, C.POINTER(_Completion), ci, C.POINTER(ci)]
        L.qxa_server_copy_result.argtypes = [vp, C.c_uint64, vp, vp, vp]
        L.qxa_server_release.argtypes = [vp, C.c_uint64]
        L.qxa_server_pause.argtypes = [vp, ci]
        L.qxa_server_drop_mesh.argtypes = [vp, vp]
        L.qxa_server_stats.argtypes = [vp, C.POINTER(i64), ci]
        L.qxa_server_destroy.argtypes = [vp]
        for name in ("qxa_mesh_create", "qxa_mesh_destroy", "qxa_plan_create", "qxa_plan_destroy",
                     "qxa_plan_get_info", "qxa_plan_copy_pattern", "qxa_assemble", "qxa_element_matrices",
                     "qxa_element_matrices_noalloc",
                     "qxa_sync", "qxa_pattern_host", "qxa_plan_check_host", "qxa_plan_check_host_corrupted", "qxa_plan_set_timing", "qxa_plan_timing_report", "qxa_graph_create", "qxa_graph_launch",
                     "qxa_graph_destroy", "qxa_server_create", "qxa_server_submit", "qxa_server_poll",
                     "qxa_server_copy_result", "qxa_server_release", "qxa_server_pause", "qxa_server_drop_mesh", "qxa_server_stats",
                     "qxa_server_destroy"):
            getattr(L, name).restype = ci
        _lib = L
    return _lib


def check(code):
    if code != 0:
        raise QxaError(code, lib().qxa_last_error().decode())
    return code


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _n_local(dim, order):
    n = 1
    for k in range(1, dim + 1):
        n = n * (order + k) // k
    return n


def _dev_arg(t, name, numel, device, dtype="float64"):
    """Checks a tensor handed to the kernels as a raw device pointer: a contiguous torch
    tensor of `dtype` on cuda:`device` with exactly `numel` elements (ValueError otherwise).
    Nothing is launched before every argument of a call has passed."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor on cuda:{device}, got {type(t).__name__}")
    want = getattr(torch, dtype)
    if t.dtype != want:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {want}")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name}: on {t.device}, expected cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    return t


def _field_len(n_nodes, n_q, n_elem, qpoint):
    return n_q * n_elem if qpoint else n_nodes


class Mesh:
    """Library-owned copy of a simplex mesh (coords [dim, n_nodes], conn [n_p, n_elem])."""

    def __init__(self, dim, order, coords, conn, device=0):
        import torch
        self.dim, self.order = int(dim), int(order)
        self.handle = C.c_void_p()
        if isinstance(coords, torch.Tensor):
            X = coords.contiguous().to(torch.float64)
            Cn = conn.contiguous().to(torch.int32)
            mem = 1 if X.is_cuda else 0
            xp, cp = X.data_ptr(), Cn.data_ptr()
            keep = (X, Cn)
        else:
            X = np.ascontiguousarray(coords, dtype=np.float64)
            Cn = np.ascontiguousarray(conn, dtype=np.int32)
            mem = 0
            xp, cp = X.ctypes.data, Cn.ctypes.data
            keep = (X, Cn)
        if X.ndim != 2 or X.shape[0] != self.dim or Cn.ndim != 2:
            raise ValueError(f"coords must be [dim={self.dim}, n_nodes] and conn [n_p, n_elem]")
        if Cn.shape[0] != _n_local(self.dim, self.order):
            raise ValueError(f"conn has {Cn.shape[0]} rows; a P{self.order} simplex in {self.dim}D has "
                             f"{_n_local(self.dim, self.order)} nodes")
        self.n_nodes = int(X.shape[1])
        self.n_elem = int(Cn.shape[1])
        self.n_p = int(Cn.shape[0])
        check(lib().qxa_mesh_create(int(device), self.dim, self.order, self.n_nodes, C.c_void_p(xp), self.n_elem,
                                    C.c_void_p(cp), mem, C.byref(self.handle)))
        del keep
        self.device = device

    def close(self):
        if self.handle:
            lib().qxa_mesh_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _quad(rule, dim):
    pts, w = rule
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, dim)
    w = np.ascontiguousarray(w, dtype=np.float64)
    q = _Quad(dim, w.size, pts.ctypes.data, w.ctypes.data)
    return q, (pts, w)


class Plan:
    """Per-mesh plan: reference tables, CSR pattern, element-entry -> slot permutation."""

    def __init__(self, mesh: Mesh, rule_m, rule_c=None):
        rule_c = rule_m if rule_c is None else rule_c
        qm, km = _quad(rule_m, mesh.dim)
        qc, kc = _quad(rule_c, mesh.dim)
        self.mesh = mesh
        self.handle = C.c_void_p()
        check(lib().qxa_plan_create(mesh.handle, C.byref(qm), C.byref(qc), C.byref(self.handle)))
        info = _PlanInfo()
        check(lib().qxa_plan_get_info(self.handle, C.byref(info)))
        self.info = info
        self.nnz = int(info.nnz)
        self.n_nodes = int(info.n_nodes)
        self.n_elem = int(info.n_elem)
        self.n_p = int(info.n_p)
        self.n_q_mass = int(info.n_q_mass)
        self.n_q_stiff = int(info.n_q_stiff)
        self.build_ms = float(info.build_ms)
        self.device_bytes = int(info.device_bytes)
        self.n_tiles = int(info.n_tiles)
        self.n_shared = int(info.n_shared)
        self.n_partials = int(info.n_partials)
        self.n_outputs = int(info.n_outputs)
        self.n_units = int(info.n_units)
        self.n_pair_units = int(info.n_pair_units)
        self.n_chains = int(info.n_chains)
        self.n_carry_reads = int(info.n_carry_reads)
        self.n_fix_slots = int(info.n_fix_slots)
        self.n_ext_units = int(info.n_ext_units)
        self.n_empty_units = int(info.n_empty_units)
        self.carry_cap = int(info.carry_cap)
        self.carry_used = int(info.carry_used)

    def pattern(self):
        """(row_ptr int64, col_idx int32) as device tensors."""
        import torch
        dev = torch.device("cuda", self.mesh.device)
        rp = torch.empty(self.n_nodes + 1, dtype=torch.int64, device=dev)
        ci = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        check(lib().qxa_plan_copy_pattern(self.handle, _ptr(rp), _ptr(ci), _stream_ptr(None)))
        return rp, ci

    def set_timing(self, on: bool):
        check(lib().qxa_plan_set_timing(self.handle, int(bool(on))))

    def timing_report(self):
        """{kernel: {"n": launches, "ms": total ms}} from events recorded around each launch."""
        import json
        buf = C.create_string_buffer(4096)
        check(lib().qxa_plan_timing_report(self.handle, buf, 4096))
        return json.loads(buf.value.decode())

    def close(self):
        if self.handle:
            lib().qxa_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def quad_builtin(dim: int, degree: int):
    """The library's built-in symmetric rule of at least this degree: (points [n_q, dim],
    weights [n_q]) as new numpy arrays (qxa_quad_builtin)."""
    q = _Quad()
    check(lib().qxa_quad_builtin(int(dim), int(degree), C.byref(q)))
    pts = np.ctypeslib.as_array(C.cast(q.points, C.POINTER(C.c_double)), shape=(q.n_q * q.dim,)).copy()
    wts = np.ctypeslib.as_array(C.cast(q.weights, C.POINTER(C.c_double)), shape=(q.n_q,)).copy()
    return pts.reshape(q.n_q, q.dim), wts


def pattern_host(dim, order, n_nodes, conn):
    """CSR pattern built by the library's host code (no GPU): (row_ptr, col_idx) numpy arrays."""
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nnz = C.c_int64()
    check(lib().qxa_pattern_host(dim, order, n_nodes, conn.shape[1], conn.ctypes.data, None, None, C.byref(nnz)))
    rp = np.zeros(n_nodes + 1, dtype=np.int64)
    ci = np.zeros(nnz.value, dtype=np.int32)
    check(lib().qxa_pattern_host(dim, order, n_nodes, conn.shape[1], conn.ctypes.data, rp.ctypes.data,
                                 ci.ctypes.data, C.byref(nnz)))
    return rp, ci


def plan_check_host(dim, order, coords, conn, chains=0, carry_cap=-1, rule_m=None, rule_c=None):
    """Host-only plan build + check (the plan executed with exact integer sums);
    returns the plan's figures as a dict (the tile-plan fields of qxa_plan_info and the
    rule sizes). Rules default to the built-in one of degree 2 * order."""
    X = np.ascontiguousarray(coords, dtype=np.float64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    info = _PlanInfo()
    qm = _quad(rule_m, dim) if rule_m is not None else None
    qc = _quad(rule_c, dim) if rule_c is not None else None
    check(lib().qxa_plan_check_host(dim, order, X.shape[1], X.ctypes.data, conn.shape[1], conn.ctypes.data,
                                    C.byref(qm[0]) if qm else None, C.byref(qc[0]) if qc else None,
                                    int(chains), int(carry_cap), C.byref(info)))
    return {name: int(getattr(info, name)) for name in _TILE_FIELDS}


def plan_check_host_corrupted(dim, order, coords, conn, mutation, chains=0, carry_cap=-1):
    """Test support for the plan check: the plan of plan_check_host with one deliberate
    corruption (1 a CSR output retargeted, 2 an entry dropped, 3 an LDS index past the
    staged pairs, 4 two outputs' entries exchanged, 5 a partial written twice, 6 a fix-up mirror
    slot changed), then checked. Returns (status, message)."""
    X = np.ascontiguousarray(coords, dtype=np.float64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    st = lib().qxa_plan_check_host_corrupted(dim, order, X.shape[1], X.ctypes.data, conn.shape[1], conn.ctypes.data,
                                             int(chains), int(carry_cap), int(mutation))
    return st, (lib().qxa_last_error().decode() if st else "")


def make_coeff(law, field=None, qpoint=False, tensor=None, tensor_q=None, sizes=None, name="coefficient"):
    """Build the ABI coefficient struct; returns (struct, keepalive). tensor: upper triangle
    (row-major) of a constant symmetric conductivity tensor K, for conductivity coefficients;
    tensor_q: device float64 [n_q][d(d+1)/2][n_elem], a tensor per quadrature node
    (isoparametric path only). sizes = (dim, n_nodes, n_q, n_elem, device) checks the
    device arrays against the plan they are used with."""
    if sizes is not None:
        dim, n_nodes, n_q, n_elem, device = sizes
        if law[0] != "const":
            _dev_arg(field, f"{name} field", _field_len(n_nodes, n_q, n_elem, qpoint), device)
        _dev_arg(tensor_q, f"{name} tensor_q", n_q * (dim * (dim + 1) // 2) * n_elem, device)
        if tensor is not None and np.asarray(tensor).size != dim * (dim + 1) // 2:
            raise ValueError(f"{name} tensor: expected the {dim * (dim + 1) // 2} upper-triangle entries")
    c = _Coeff()
    c.a[0] = c.a[1] = c.a[2] = 0.0
    kt = None
    if tensor is not None:
        kt = np.ascontiguousarray(tensor, dtype=np.float64)
        c.tensor = kt.ctypes.data
    if tensor_q is not None:
        kt = (kt, tensor_q)
        c.tensor_q = tensor_q.data_ptr()
    if law[0] == "const":
        c.kind, c.law, c.value, c.field = 0, 0, float(law[1]), None
        return c, kt
    c.law = _LAW[law[0]]
    for k, v in enumerate(law[1:]):
        c.a[k] = float(v)
    if field is None:
        raise ValueError("non-constant coefficient law needs a device field")
    c.kind = 2 if qpoint else 1
    c.field = field.data_ptr()
    c.value = 0.0
    return c, (field, kt)


def _precision(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _sizes(plan, which):
    """(dim, n_nodes, n_q, n_elem, device) of a plan for coefficients on its mass
    ("mass") or stiffness ("stiff") rule."""
    nq = plan.n_q_mass if which == "mass" else plan.n_q_stiff
    return (plan.mesh.dim, plan.n_nodes, nq, plan.n_elem, plan.mesh.device)


def assemble(plan: Plan, law_m, law_c, field_m=None, field_c=None, precision="fp64", M=None, Cv=None,
             stream=None, want_m=True, want_c=True, qpoint=False, tensor=None):
    """One assembly into CSR value arrays (device float64 tensors of length nnz)."""
    import torch
    dev = torch.device("cuda", plan.mesh.device)
    _dev_arg(M, "M", plan.nnz, plan.mesh.device)
    _dev_arg(Cv, "Cv", plan.nnz, plan.mesh.device)
    cm, k1 = make_coeff(law_m, field_m, qpoint, sizes=_sizes(plan, "mass"), name="mass")
    cc, k2 = make_coeff(law_c, field_c, qpoint, tensor, sizes=_sizes(plan, "stiff"), name="conductivity")
    if want_m and M is None:
        M = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    if want_c and Cv is None:
        Cv = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    check(lib().qxa_assemble(plan.handle, C.byref(cm), C.byref(cc), _precision(precision),
                             _ptr(M if want_m else None), _ptr(Cv if want_c else None), _stream_ptr(stream)))
    return M, Cv


def coeff_product(plan: Plan, law, u, v, rule="mass", S=None, stream=None):
    """S[q][e] = law(u_h(x_q)) * v_h(x_q) at the quadrature nodes of the plan's mass (or
    stiffness) rule: the coefficient of the mass tensor contracted with v (qxa_coeff_product)."""
    import torch
    which = {"mass": 0, "stiffness": 1}[rule]
    nq = plan.n_q_mass if which == 0 else plan.n_q_stiff
    sz = _sizes(plan, "mass" if which == 0 else "stiff")
    _dev_arg(u, "u", plan.n_nodes, plan.mesh.device)
    _dev_arg(v, "v", plan.n_nodes, plan.mesh.device)
    _dev_arg(S, "S", nq * plan.n_elem, plan.mesh.device)
    if S is None:
        S = torch.empty((nq, plan.n_elem), dtype=torch.float64, device=torch.device("cuda", plan.mesh.device))
    c, keep = make_coeff(law, u, sizes=sz, name="law")
    check(lib().qxa_coeff_product(plan.handle, which, C.byref(c), _ptr(v), _ptr(S), _stream_ptr(stream)))
    return S


def mass_tensor_product(plan: Plan, law_dm, u, v, T=None, S=None, stream=None):
    """The mass tensor of the Newton Jacobian (M_ijk = int m'(u_h) phi_i phi_j phi_k)
    contracted with v in its second mode, in the plan's CSR pattern: the mass matrix of
    the per-node coefficient law_dm(u_h) * v_h. Returns the value array (and S)."""
    S = coeff_product(plan, law_dm, u, v, "mass", S=S, stream=stream)
    T, _ = assemble(plan, ("identity",), ("const", 1.0), S, None, M=T, stream=stream, want_c=False, qpoint=True)
    return T, S


def cond_tensor_product(plan: Plan, law_dc, u, v, T=None, stream=None, tensor=None):
    """The conductivity tensor of the Newton Jacobian (C_ijk = int c'(u_h) grad phi_i .
    grad phi_j phi_k) contracted with v in its second mode, as values in the plan's CSR
    pattern (row i, column k; not symmetric)."""
    import torch
    _dev_arg(u, "u", plan.n_nodes, plan.mesh.device)
    _dev_arg(v, "v", plan.n_nodes, plan.mesh.device)
    _dev_arg(T, "T", plan.nnz, plan.mesh.device)
    if T is None:
        T = torch.empty(plan.nnz, dtype=torch.float64, device=torch.device("cuda", plan.mesh.device))
    c, keep = make_coeff(law_dc, u, tensor=tensor, sizes=_sizes(plan, "stiff"), name="law")
    check(lib().qxa_cond_tensor_product(plan.handle, C.byref(c), _ptr(v), _ptr(T), _stream_ptr(stream)))
    return T


def assemble_iso(plan: Plan, law_m, law_c, field_m=None, field_c=None, M=None, Cv=None, stream=None,
                 want_m=True, want_c=True, qpoint=False, tensor=None, tensor_q=None):
    """Isoparametric (curved) elements: M and C with the geometry evaluated per quadrature
    node from every node's position (qxa_assemble_iso, FP64). tensor_q: optional device
    conductivity tensor per quadrature node, float64 [n_q][d(d+1)/2][n_elem]."""
    import torch
    dev = torch.device("cuda", plan.mesh.device)
    _dev_arg(M, "M", plan.nnz, plan.mesh.device)
    _dev_arg(Cv, "Cv", plan.nnz, plan.mesh.device)
    cm, k1 = make_coeff(law_m, field_m, qpoint, sizes=_sizes(plan, "mass"), name="mass")
    cc, k2 = make_coeff(law_c, field_c, qpoint, tensor, tensor_q, sizes=_sizes(plan, "stiff"), name="conductivity")
    if want_m and M is None:
        M = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    if want_c and Cv is None:
        Cv = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    check(lib().qxa_assemble_iso(plan.handle, C.byref(cm), C.byref(cc), _ptr(M if want_m else None),
                                 _ptr(Cv if want_c else None), _stream_ptr(stream)))
    return M, Cv


def load_vector(plan: Plan, law_f, field=None, F=None, stream=None, qpoint=False):
    """Volume load vector F_i = int f phi_i (device float64 [n_nodes]) on the plan's mass rule."""
    import torch
    _dev_arg(F, "F", plan.n_nodes, plan.mesh.device)
    c, keep = make_coeff(law_f, field, qpoint, sizes=_sizes(plan, "mass"), name="load")
    if F is None:
        F = torch.empty(plan.n_nodes, dtype=torch.float64, device=torch.device("cuda", plan.mesh.device))
    check(lib().qxa_load_vector(plan.handle, C.byref(c), _ptr(F), _stream_ptr(stream)))
    return F


def reaction_matrix(plan: Plan, law_a, field=None, A=None, stream=None, qpoint=False):
    """Reaction matrix A_ij = int a phi_j phi_i: the mass matrix of the coefficient a."""
    A, _ = assemble(plan, law_a, ("const", 1.0), field, None, M=A, stream=stream, want_c=False, qpoint=qpoint)
    return A


def element_matrices(plan: Plan, law_m, law_c, field_m=None, field_c=None, precision="fp64", stream=None,
                     qpoint=False):
    """Formation only: V_m, V_c as device tensors [n_p*n_p, n_elem]."""
    import torch
    dev = torch.device("cuda", plan.mesh.device)
    n2 = plan.n_p * plan.n_p
    Vm = torch.empty((n2, plan.n_elem), dtype=torch.float64, device=dev)
    Vc = torch.empty((n2, plan.n_elem), dtype=torch.float64, device=dev)
    cm, k1 = make_coeff(law_m, field_m, qpoint, sizes=_sizes(plan, "mass"), name="mass")
    cc, k2 = make_coeff(law_c, field_c, qpoint, sizes=_sizes(plan, "stiff"), name="conductivity")
    check(lib().qxa_element_matrices(plan.handle, C.byref(cm), C.byref(cc), _precision(precision), _ptr(Vm),
                                     _ptr(Vc), _stream_ptr(stream)))
    return Vm, Vc


def element_matrices_noalloc(plan: Plan, law_m, law_c, field_m=None, field_c=None, precision="fp64", Vm=None,
                             Vc=None, stream=None, qpoint=False):
    """Formation only, through the allocation-free entry point (staging in the library's
    fixed device scratch). Vm, Vc: caller tensors [n_p*n_p, n_elem] (allocated here if None)."""
    import torch
    dev = torch.device("cuda", plan.mesh.device)
    n2 = plan.n_p * plan.n_p
    if Vm is None:
        Vm = torch.empty((n2, plan.n_elem), dtype=torch.float64, device=dev)
    if Vc is None:
        Vc = torch.empty((n2, plan.n_elem), dtype=torch.float64, device=dev)
    _dev_arg(Vm, "Vm", n2 * plan.n_elem, plan.mesh.device)
    _dev_arg(Vc, "Vc", n2 * plan.n_elem, plan.mesh.device)
    cm, k1 = make_coeff(law_m, field_m, qpoint, sizes=_sizes(plan, "mass"), name="mass")
    cc, k2 = make_coeff(law_c, field_c, qpoint, sizes=_sizes(plan, "stiff"), name="conductivity")
    check(lib().qxa_element_matrices_noalloc(plan.handle, C.byref(cm), C.byref(cc), _precision(precision),
                                             _ptr(Vm), _ptr(Vc), _stream_ptr(stream)))
    return Vm, Vc


class ReassemblyGraph:
    """One assembly captured in a HIP graph; update the fields in place, then launch()."""

    def __init__(self, plan: Plan, law_m, law_c, field_m=None, field_c=None, precision="fp64", M=None, Cv=None,
                 qpoint=False):
        import torch
        dev = torch.device("cuda", plan.mesh.device)
        self.plan = plan
        _dev_arg(M, "M", plan.nnz, plan.mesh.device)
        _dev_arg(Cv, "Cv", plan.nnz, plan.mesh.device)
        cm, self._k1 = make_coeff(law_m, field_m, qpoint, sizes=_sizes(plan, "mass"), name="mass")
        cc, self._k2 = make_coeff(law_c, field_c, qpoint, sizes=_sizes(plan, "stiff"), name="conductivity")
        self.M = M if M is not None else torch.empty(plan.nnz, dtype=torch.float64, device=dev)
        self.Cv = Cv if Cv is not None else torch.empty(plan.nnz, dtype=torch.float64, device=dev)
        self.handle = C.c_void_p()
        check(lib().qxa_graph_create(plan.handle, C.byref(cm), C.byref(cc), _precision(precision), _ptr(self.M),
                                     _ptr(self.Cv), C.byref(self.handle)))

    def launch(self, stream=None):
        check(lib().qxa_graph_launch(self.handle, _stream_ptr(stream)))
        return self.M, self.Cv

    def close(self):
        if self.handle:
            lib().qxa_graph_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sync(plan: Plan, stream=None):
    check(lib().qxa_sync(plan.handle, _stream_ptr(stream)))


class Server:
    """Continuous-batching assembly server of the library (a worker thread in libqxa).

    submit() returns a ticket; poll() returns completions (dicts); result()
    copies a completed job's CSR values into new device tensors; every polled
    ticket must be released. Coefficient fields are kept alive here until
    their job completes.
    """

    def __init__(self, device=0, hbm_budget=4 << 30, max_inflight=64, n_streams=4, batch_tile_limit=512,
                 queue_capacity=65536, plan_cache_entries=0, plan_builders=0):
        o = _ServerOpts(int(device), int(hbm_budget), int(max_inflight), int(n_streams), int(batch_tile_limit),
                        int(queue_capacity), int(plan_cache_entries), int(plan_builders))
        self.device = device
        self.handle = C.c_void_p()
        check(lib().qxa_server_create(C.byref(o), C.byref(self.handle)))
        self._keep = {}
        self._nnz = {}
        self._meshes = {}  # resident plans refer to their meshes: keep them until close()

    def submit(self, mesh: Mesh, rule_m, rule_c=None, law_m=("const", 1.0), law_c=("const", 1.0), field_m=None,
               field_c=None, precision="fp64", tag=0, qpoint=False, tensor=None):
        rule_c = rule_m if rule_c is None else rule_c
        qm, km = _quad(rule_m, mesh.dim)
        qc, kc = _quad(rule_c, mesh.dim)
        if mesh.device != self.device:
            raise ValueError(f"mesh on device {mesh.device}, server on {self.device}")
        cm, k1 = make_coeff(law_m, field_m, qpoint, sizes=(mesh.dim, mesh.n_nodes, qm.n_q, mesh.n_elem, self.device),
                            name="mass")
        cc, k2 = make_coeff(law_c, field_c, qpoint, tensor,
                            sizes=(mesh.dim, mesh.n_nodes, qc.n_q, mesh.n_elem, self.device), name="conductivity")
        job = _Job(mesh.handle, qm, qc, cm, cc, _precision(precision), int(tag))
        t = C.c_uint64()
        check(lib().qxa_server_submit(self.handle, C.byref(job), C.byref(t)))
        self._keep[t.value] = (k1, k2)
        self._meshes[id(mesh)] = mesh
        return t.value

    def poll(self, max_n=256):
        buf = (_Completion * max_n)()
        n = C.c_int()
        check(lib().qxa_server_poll(self.handle, buf, max_n, C.byref(n)))
        out = []
        for c in buf[:n.value]:
            self._keep.pop(c.ticket, None)
            self._nnz[c.ticket] = int(c.nnz)
            out.append({"ticket": c.ticket, "tag": c.user_tag, "status": c.status, "plan_cached": bool(c.plan_cached),
                        "batched": c.batched, "n_nodes": c.n_nodes, "nnz": c.nnz, "queue_ms": c.queue_ms,
                        "run_ms": c.run_ms, "total_ms": c.total_ms, "plan_ms": c.plan_ms,
                        "message": c.message.decode()})
        return out

    def result(self, ticket, stream=None):
        """(M, C) of a completed job copied into new float64 device tensors (on `stream`)."""
        import torch
        nnz = self._nnz[ticket]
        dev = torch.device("cuda", self.device)
        M = torch.empty(nnz, dtype=torch.float64, device=dev)
        Cv = torch.empty(nnz, dtype=torch.float64, device=dev)
        check(lib().qxa_server_copy_result(self.handle, C.c_uint64(ticket), _ptr(M), _ptr(Cv), _stream_ptr(stream)))
        return M, Cv

    def release(self, ticket):
        self._nnz.pop(ticket, None)
        check(lib().qxa_server_release(self.handle, C.c_uint64(ticket)))

    def drop_mesh(self, mesh: Mesh):
        """Free the server's plans of a mesh whose jobs are all released (QxaError
        QXA_E_BUSY otherwise); the mesh may then be closed."""
        check(lib().qxa_server_drop_mesh(self.handle, mesh.handle))
        self._meshes.pop(id(mesh), None)

    def pause(self, paused=True):
        """Stop (True) or resume (False) admission; submissions keep queueing."""
        check(lib().qxa_server_pause(self.handle, int(bool(paused))))

    def wait(self, n, timeout_s=60.0):
        """Poll until n completions have arrived (raises TimeoutError)."""
        import time
        out, t0 = [], time.perf_counter()
        while len(out) < n:
            got = self.poll()
            out += got
            if not got:
                if time.perf_counter() - t0 > timeout_s:
                    raise TimeoutError(f"{len(out)} of {n} jobs completed in {timeout_s} s: {self.stats()}")
                time.sleep(0.0005)
        return out

    def stats(self):
        v = (C.c_int64 * len(SERVER_STATS))()
        check(lib().qxa_server_stats(self.handle, v, len(SERVER_STATS)))
        return dict(zip(SERVER_STATS, list(v)))

    def close(self):
        if self.handle:
            lib().qxa_server_destroy(self.handle)
            self.handle = C.c_void_p()
            self._keep.clear()
            self._meshes.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
