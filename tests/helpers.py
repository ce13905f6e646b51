"""Shared test helpers (comparison metrics; no assembly arithmetic)."""
import numpy as np

# Row-scaled error bounds of the reduced-precision contraction forms against the FP64
# oracle. FP32, F16 hi+lo (with per-element power-of-two scaling of X) and the
# three-term BF16 split carry 22-24-bit operands with FP32 accumulation; measured
# 2-5e-7 on the 3D P2 and 2D P3 workloads, so each is held to the 1e-6 target.
# The two-term BF16 split carries ~16 bits (measured 1.2-1.5e-5): its own bound.
FORM_BOUNDS = {"fp32": 1e-6, "f16x2": 1e-6, "bf16x3": 1e-6, "bf16x2": 5e-5}


def row_scaled_error(got, ref, row_ptr):
    """max_ij |v_ij - o_ij| / max_k |o_ik| (entrywise relative error is undefined on cancelled zeros)."""
    if ref.size == 0:
        return 0.0
    rows = np.repeat(np.arange(row_ptr.size - 1), np.diff(row_ptr))
    rmax = np.zeros(row_ptr.size - 1)
    np.maximum.at(rmax, rows, np.abs(ref))          # rows without entries keep 0
    rmax = np.where(rmax == 0, 1.0, rmax)
    return float(np.max(np.abs(got - ref) / rmax[rows]))


def sampled_rows_error(got_full, row_ptr_full, rows, sub_ptr, ref_vals):
    """Row-scaled error on selected rows: got_full is the full CSR value array."""
    err = 0.0
    for k, r in enumerate(rows):
        g = got_full[row_ptr_full[r]:row_ptr_full[r + 1]]
        o = ref_vals[sub_ptr[k]:sub_ptr[k + 1]]
        m = np.max(np.abs(o)) if o.size else 1.0
        err = max(err, float(np.max(np.abs(g - o)) / (m if m > 0 else 1.0)))
    return err


def transpose_slots(row_ptr, col_idx):
    """Index of slot (j,i) for every slot (i,j) of a structurally symmetric CSR."""
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    key = rows.astype(np.int64) * n + col_idx
    tkey = col_idx.astype(np.int64) * n + rows
    order = np.argsort(key)
    pos = np.searchsorted(key[order], tkey)
    return order[pos]


def frobenius_error(got, ref):
    """||got - ref||_F / ||ref||_F."""
    n = float(np.linalg.norm(ref))
    return float(np.linalg.norm(got - ref)) / (n if n > 0 else 1.0)


_INPUTS = {}


def workload_inputs(name):
    """make_inputs of a named full-size workload, generated once per test process (the
    2D P3 one takes tens of seconds)."""
    from workloads import WORKLOADS, make_inputs
    if name not in _INPUTS:
        _INPUTS[name] = make_inputs(WORKLOADS[name])
    return _INPUTS[name]
