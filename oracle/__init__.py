"""CPU FP64 reference (the oracle) for FEM mass/conductivity assembly.

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package. The library under test never
imports it, and this package never imports the library.

The C implementation (oracle.c) follows Algorithm 1 of the paper (a loop over
elements and quadrature nodes, then the addition of local matrices into the
global matrix at N_e x N_e). This module is only argument marshalling.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Coeff(C.Structure):
    _fields_ = [("kind", C.c_int), ("law", C.c_int), ("value", C.c_double),
                ("a", C.c_double * 3), ("field", C.c_void_p), ("tensor", C.c_void_p),
                ("tensor_q", C.c_void_p)]


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(build())
        lib.oracle_set_fault.argtypes = [C.c_int]
        lib.oracle_n_local.argtypes = [C.c_int, C.c_int]
        lib.oracle_local_nodes.argtypes = [C.c_int, C.c_int, _D]
        lib.oracle_basis.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D, _D]
        lib.oracle_pattern_rows.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, _I32, _I64]
        lib.oracle_pattern_rows.restype = C.c_int64
        lib.oracle_pattern_cols.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, _I32, _I64, _I32]
        common = [C.c_int, C.c_int, C.c_int64, _D, C.c_int64, _I32, C.c_int, _D, _D, C.c_int, _D, _D,
                  C.POINTER(_Coeff), C.POINTER(_Coeff)]
        lib.oracle_assemble.argtypes = common + [_I64, _I32, _D, _D, C.c_int, C.POINTER(C.c_int64)]
        lib.oracle_last_timing.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.oracle_assemble_iso.argtypes = common + [_I64, _I32, _D, _D, C.c_int, C.POINTER(C.c_int64)]
        lib.oracle_assemble_rows.argtypes = common + [C.c_int64, _I64, _I64, _I32, _D, _D, C.c_int,
                                                      C.POINTER(C.c_int64)]
        lib.oracle_rows_pattern.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, _I32, C.c_int64, _I64,
                                            _I64, C.c_void_p]
        lib.oracle_rows_pattern.restype = C.c_int64
        lib.oracle_element_matrices.argtypes = common + [C.c_int64, _I64, _D, _D]
        lib.oracle_qpoint_coeff.argtypes = [C.c_int, C.c_int, C.c_int64, _I32, C.c_int, _D, C.POINTER(_Coeff),
                                            C.c_int64, _I64, _D]
        lib.oracle_mass_tensor_product.argtypes = [C.c_int, C.c_int, C.c_int64, _D, C.c_int64, _I32, C.c_int, _D,
                                                   _D, C.POINTER(_Coeff), _D, _I64, _I32, _D, C.c_int,
                                                   C.POINTER(C.c_int64)]
        lib.oracle_cond_tensor_product.argtypes = lib.oracle_mass_tensor_product.argtypes
        lib.oracle_load_vector.argtypes = [C.c_int, C.c_int, C.c_int64, _D, C.c_int64, _I32, C.c_int, _D, _D,
                                           C.POINTER(_Coeff), _D, C.POINTER(C.c_int64)]
        _lib = lib
    return _lib


@contextlib.contextmanager
def planted_fault(code: int):
    """Plant a known mistake in the oracle (for tests showing that pins catch it)."""
    lib = _load()
    lib.oracle_set_fault(code)
    try:
        yield
    finally:
        lib.oracle_set_fault(0)


def _coeff(law, field=None, qpoint=None):
    """law: ("const", v) | ("identity",) | ("poly2", a0, a1, a2) | ("exp", a0, a1)."""
    c = _Coeff()
    c.a[0] = c.a[1] = c.a[2] = 0.0
    keep = None
    if law[0] == "const":
        c.kind, c.law, c.value, c.field = 0, 0, float(law[1]), None
    else:
        c.law = {"identity": 0, "poly2": 1, "exp": 2}[law[0]]
        for k, v in enumerate(law[1:]):
            c.a[k] = float(v)
        if qpoint is not None:
            keep = np.ascontiguousarray(qpoint, dtype=np.float64)
            c.kind = 2
        else:
            keep = np.ascontiguousarray(field, dtype=np.float64)
            c.kind = 1
        c.field = keep.ctypes.data
    return c, keep


def n_local(dim, order):
    return _load().oracle_n_local(dim, order)


def local_nodes(dim, order):
    n = n_local(dim, order)
    out = np.zeros(n * dim)
    _load().oracle_local_nodes(dim, order, out)
    return out.reshape(n, dim)


def basis(dim, order, pts):
    """Reference Lagrange basis values phi [n_pts, n_p] and gradients [n_pts, n_p, dim]."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, dim)
    n = n_local(dim, order)
    phi = np.zeros(pts.shape[0] * n)
    dphi = np.zeros(pts.shape[0] * n * dim)
    rc = _load().oracle_basis(dim, order, pts.shape[0], pts.reshape(-1), phi, dphi)
    if rc < 0:
        raise RuntimeError(f"oracle_basis failed ({rc})")
    return phi.reshape(-1, n), dphi.reshape(-1, n, dim)


def pattern(mesh):
    lib = _load()
    conn = np.ascontiguousarray(mesh["conn"], dtype=np.int32)
    n_nodes = int(mesh["coords"].shape[1])
    row_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    nnz = lib.oracle_pattern_rows(mesh["dim"], mesh["order"], n_nodes, conn.shape[1], conn.reshape(-1), row_ptr)
    if nnz < 0:
        raise ValueError(f"oracle pattern failed ({nnz})")
    col_idx = np.zeros(int(nnz), dtype=np.int32)
    rc = lib.oracle_pattern_cols(mesh["dim"], mesh["order"], n_nodes, conn.shape[1], conn.reshape(-1), row_ptr,
                                 col_idx)
    if rc:
        raise ValueError(f"oracle pattern failed ({rc})")
    return row_ptr, col_idx


def _common(mesh, rule_m, rule_c, law_m, law_c, field_m, field_c, qpoint_m=None, qpoint_c=None, tensor_c=None,
            tensor_q=None):
    conn = np.ascontiguousarray(mesh["conn"], dtype=np.int32)
    coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
    pm, wm = (np.ascontiguousarray(a, dtype=np.float64) for a in rule_m)
    pc, wc = (np.ascontiguousarray(a, dtype=np.float64) for a in rule_c)
    cm, km = _coeff(law_m, field_m, qpoint_m)
    cc, kc = _coeff(law_c, field_c, qpoint_c)
    if tensor_c is not None:
        kc = (kc, np.ascontiguousarray(tensor_c, dtype=np.float64))
        cc.tensor = kc[1].ctypes.data
    if tensor_q is not None:
        kc = (kc, np.ascontiguousarray(tensor_q, dtype=np.float64))
        cc.tensor_q = kc[1].ctypes.data
    args = [mesh["dim"], mesh["order"], coords.shape[1], coords.reshape(-1), conn.shape[1], conn.reshape(-1),
            wm.size, pm.reshape(-1), wm, wc.size, pc.reshape(-1), wc, C.byref(cm), C.byref(cc)]
    return args, (conn, coords, pm, wm, pc, wc, cm, cc, km, kc)


def assemble(mesh, rule_m, rule_c, law_m, law_c, field_m=None, field_c=None, nthreads=0,
             qpoint_m=None, qpoint_c=None, tensor_c=None, tensor_q=None):
    """Full CSR assembly: returns (row_ptr int64, col_idx int32, M float64, C float64).
    tensor_c: upper triangle (row-major) of a constant symmetric conductivity tensor K
    (anisotropic conductivity c K), or None for the isotropic case. tensor_q: instead,
    a tensor per quadrature node of the conductivity rule, [n_q][d(d+1)/2][n_elem]."""
    row_ptr, col_idx = pattern(mesh)
    M = np.zeros(col_idx.size)
    Cv = np.zeros(col_idx.size)
    args, keep = _common(mesh, rule_m, rule_c, law_m, law_c, field_m, field_c, qpoint_m, qpoint_c, tensor_c,
                         tensor_q)
    bad = C.c_int64(-1)
    rc = _load().oracle_assemble(*args, row_ptr, col_idx, M, Cv, int(nthreads), C.byref(bad))
    if rc:
        raise ValueError(f"oracle assemble failed ({rc}), element {bad.value}")
    return row_ptr, col_idx, M, Cv


def assemble_rows(mesh, rows, rule_m, rule_c, law_m, law_c, field_m=None, field_c=None, nthreads=0,
                  qpoint_m=None, qpoint_c=None):
    """Selected rows: returns (sub row_ptr, col_idx, M, C) with rows in the given order."""
    lib = _load()
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    conn = np.ascontiguousarray(mesh["conn"], dtype=np.int32)
    n_nodes = int(mesh["coords"].shape[1])
    sub_ptr = np.zeros(rows.size + 1, dtype=np.int64)
    tot = lib.oracle_rows_pattern(mesh["dim"], mesh["order"], n_nodes, conn.shape[1], conn.reshape(-1), rows.size,
                                  rows, sub_ptr, None)
    if tot < 0:
        raise ValueError(f"oracle rows pattern failed ({tot})")
    cols = np.zeros(int(tot), dtype=np.int32)
    lib.oracle_rows_pattern(mesh["dim"], mesh["order"], n_nodes, conn.shape[1], conn.reshape(-1), rows.size, rows,
                            sub_ptr, cols.ctypes.data)
    M = np.zeros(cols.size)
    Cv = np.zeros(cols.size)
    args, keep = _common(mesh, rule_m, rule_c, law_m, law_c, field_m, field_c, qpoint_m, qpoint_c)
    bad = C.c_int64(-1)
    rc = lib.oracle_assemble_rows(*args, rows.size, rows, sub_ptr, cols, M, Cv, int(nthreads), C.byref(bad))
    if rc:
        raise ValueError(f"oracle assemble_rows failed ({rc}), element {bad.value}")
    return sub_ptr, cols, M, Cv


def element_matrices(mesh, elems, rule_m, rule_c, law_m, law_c, field_m=None, field_c=None,
                     qpoint_m=None, qpoint_c=None):
    """Full local matrices [n_sel, n_p, n_p] (M_e, C_e) of selected elements."""
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    n = n_local(mesh["dim"], mesh["order"])
    Me = np.zeros(elems.size * n * n)
    Ce = np.zeros(elems.size * n * n)
    args, keep = _common(mesh, rule_m, rule_c, law_m, law_c, field_m, field_c, qpoint_m, qpoint_c)
    rc = _load().oracle_element_matrices(*args, elems.size, elems, Me, Ce)
    if rc:
        raise ValueError(f"oracle element_matrices failed ({rc})")
    return Me.reshape(-1, n, n), Ce.reshape(-1, n, n)


def qpoint_coeff(mesh, elems, rule, law, field=None):
    """Coefficient values at the quadrature nodes of selected elements [n_sel, n_q]."""
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    conn = np.ascontiguousarray(mesh["conn"], dtype=np.int32)
    pts, w = rule
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    c, keep = _coeff(law, field)
    out = np.zeros(elems.size * w.size)
    rc = _load().oracle_qpoint_coeff(mesh["dim"], mesh["order"], conn.shape[1], conn.reshape(-1), w.size,
                                     pts.reshape(-1), C.byref(c), elems.size, elems, out)
    if rc:
        raise ValueError("oracle_qpoint_coeff failed")
    return out.reshape(-1, w.size)


def _tensor_product(fn, mesh, rule, law, u, v, nthreads, tensor=None):
    row_ptr, col_idx = pattern(mesh)
    out = np.zeros(col_idx.size)
    conn = np.ascontiguousarray(mesh["conn"], dtype=np.int32)
    coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
    pts, w = (np.ascontiguousarray(a, dtype=np.float64) for a in rule)
    c, keep = _coeff(law, u)
    kt = None
    if tensor is not None:
        kt = np.ascontiguousarray(tensor, dtype=np.float64)
        c.tensor = kt.ctypes.data
    vv = np.ascontiguousarray(v, dtype=np.float64)
    bad = C.c_int64(-1)
    rc = getattr(_load(), fn)(mesh["dim"], mesh["order"], coords.shape[1], coords.reshape(-1), conn.shape[1],
                              conn.reshape(-1), w.size, pts.reshape(-1), w, C.byref(c), vv, row_ptr, col_idx, out,
                              int(nthreads), C.byref(bad))
    if rc:
        raise ValueError(f"oracle {fn} failed ({rc}), element {bad.value}")
    return row_ptr, col_idx, out


def cond_tensor_product(mesh, rule, law_dc, u, v, nthreads=0, tensor=None):
    """The conductivity tensor of Section 5 (C_ijk = int c'(u_h) grad phi_i . grad phi_j phi_k)
    contracted with v in its second mode, in the CSR pattern (row i, column k; not symmetric)."""
    return _tensor_product("oracle_cond_tensor_product", mesh, rule, law_dc, u, v, nthreads, tensor)


def mass_tensor_product(mesh, rule, law_dm, u, v, nthreads=0):
    """The mass tensor of Section 5 (M_ijk = int m'(u_h) phi_i phi_j phi_k) contracted with
    the nodal vector v in its second mode, in the CSR pattern: (row_ptr, col_idx, values).
    law_dm is the law of m' applied to the interpolated field u."""
    row_ptr, col_idx = pattern(mesh)
    out = np.zeros(col_idx.size)
    conn = np.ascontiguousarray(mesh["conn"], dtype=np.int32)
    coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
    pts, w = (np.ascontiguousarray(a, dtype=np.float64) for a in rule)
    c, keep = _coeff(law_dm, u)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    bad = C.c_int64(-1)
    rc = _load().oracle_mass_tensor_product(mesh["dim"], mesh["order"], coords.shape[1], coords.reshape(-1),
                                            conn.shape[1], conn.reshape(-1), w.size, pts.reshape(-1), w,
                                            C.byref(c), vv, row_ptr, col_idx, out, int(nthreads), C.byref(bad))
    if rc:
        raise ValueError(f"oracle mass_tensor_product failed ({rc}), element {bad.value}")
    return row_ptr, col_idx, out


def load_vector(mesh, rule, law_f, field=None, qpoint=None):
    """Volume load vector F_i = int f phi_i over the mesh (float64 [n_nodes])."""
    conn = np.ascontiguousarray(mesh["conn"], dtype=np.int32)
    coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
    pts, w = (np.ascontiguousarray(a, dtype=np.float64) for a in rule)
    c, keep = _coeff(law_f, field, qpoint)
    F = np.zeros(coords.shape[1])
    bad = C.c_int64(-1)
    rc = _load().oracle_load_vector(mesh["dim"], mesh["order"], coords.shape[1], coords.reshape(-1), conn.shape[1],
                                    conn.reshape(-1), w.size, pts.reshape(-1), w, C.byref(c), F, C.byref(bad))
    if rc:
        raise ValueError(f"oracle load_vector failed ({rc}), element {bad.value}")
    return F


def assemble_iso(mesh, rule_m, rule_c, law_m, law_c, field_m=None, field_c=None, nthreads=0, tensor_c=None,
                 qpoint_m=None, qpoint_c=None, tensor_q=None):
    """Isoparametric assembly (the element map uses the P-order basis and every node's
    position): returns (row_ptr, col_idx, M, C)."""
    row_ptr, col_idx = pattern(mesh)
    M = np.zeros(col_idx.size)
    Cv = np.zeros(col_idx.size)
    args, keep = _common(mesh, rule_m, rule_c, law_m, law_c, field_m, field_c, qpoint_m, qpoint_c, tensor_c,
                         tensor_q)
    bad = C.c_int64(-1)
    rc = _load().oracle_assemble_iso(*args, row_ptr, col_idx, M, Cv, int(nthreads), C.byref(bad))
    if rc:
        raise ValueError(f"oracle assemble_iso failed ({rc}), element {bad.value}")
    return row_ptr, col_idx, M, Cv


def last_timing():
    """(formation_s, assembly_s) of the last assemble() call: wall-clock seconds of the
    element-matrix loop and of the global assembly (the paper's two timings)."""
    f, a = C.c_double(0.0), C.c_double(0.0)
    _load().oracle_last_timing(C.byref(f), C.byref(a))
    return f.value, a.value
