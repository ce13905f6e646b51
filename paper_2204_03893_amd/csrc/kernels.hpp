// Kernel argument blocks and launchers (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/qxa.h"
#include "kernels_common.hpp"
#include "plan_format.hpp"
#include "qxa_internal.hpp"

namespace qxa {

// (dim, order, n_q mass, n_q stiffness) combinations with compiled kernels:
// one rule for both matrices (degree 2P), the lower-degree stiffness rule
// (degree 2P-2) that constant coefficients allow, and one size per shape
// that any other rule of at most kMaxRule2D / kMaxRule3D nodes is padded to
// (zero-weight copies of its node 0; a rule is padded to the compiled
// combination of least work that holds it).
#define QXA_FORM_CASES_TUNED(X)                                                                               \
    X(2, 1, 3, 3) X(2, 2, 6, 6) X(2, 3, 12, 12) X(3, 1, 4, 4) X(3, 2, 11, 11) X(3, 3, 24, 24) X(2, 1, 3, 1)   \
        X(2, 2, 6, 3) X(2, 3, 12, 6) X(3, 1, 4, 1) X(3, 2, 11, 4) X(3, 3, 24, 11)
#define QXA_FORM_CASES_PADDED(X) \
    X(2, 1, 16, 16) X(2, 2, 16, 16) X(2, 3, 16, 16) X(3, 1, 32, 32) X(3, 2, 32, 32) X(3, 3, 32, 32)
#define QXA_FORM_CASES(X) QXA_FORM_CASES_TUNED(X) QXA_FORM_CASES_PADDED(X)

// Elements per tile of the fused kernels. Vector-ALU variant (P1): one lane
// per element. Matrix-core variant (P2, P3): 4 producer waves of 16 elements
// (two LDS buffers of both matrices, 2 * 2 * NS * (T + 1) values, next to
// Q^T); 3D P3 (NS = 210) keeps one 16-element group whose row blocks eight
// producer waves split, two each.
constexpr int tile_size(int D, int P)
{
    return (D == 3 && P == 3) ? 16 : (P >= 2) ? 64 : 256;
}

constexpr size_t kLdsBytes = 160 * 1024;  // LDS of a workgroup (gfx950)

// LDS bytes of the matrix-core variant with Q^T staged on chip: the two
// buffers of (V_m, V_c) in the staging type (es bytes), Q^T in K steps of
// `kstep_bytes` per 16-row block (`ks` steps), and the basis and weight tables.
constexpr size_t staged_lds_bytes(int D, int P, int nqm, int nqc, int es, int ks, int kstep_bytes)
{
    const int np = D == 2 ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6, ns = np * (np + 1) / 2;
    return size_t(4) * es * ns * (tile_size(D, P) + 1) + size_t(ks) * ((ns + 15) / 16) * kstep_bytes +
           (size_t(nqm + nqc) * np + nqm + nqc) * 8;
}

// Matrix-core variant of a shape and rule sizes: P >= 2, and for the shapes
// that stage Q^T in LDS (T != 16) the FP64 form must fit a workgroup's LDS
// (16 x 16 x 4 steps: ceil(n_q,m / 4) + d(d+1)/2 ceil(n_q,c / 4), 512 bytes
// per 16-row block each). Larger rules run on the vector-ALU variant.
constexpr bool mfma_variant(int D, int P, int nqm, int nqc)
{
    return P >= 2 && (tile_size(D, P) == 16 ||
                      staged_lds_bytes(D, P, nqm, nqc, 8, (nqm + 3) / 4 + D * (D + 1) / 2 * ((nqc + 3) / 4), 512) <=
                          kLdsBytes);
}

bool fused_uses_mfma(int D, int P, int nqm, int nqc);

// Split 16-bit forms: Q^T staged in LDS (not the T = 16 shape), and the
// three-term BF16 form (the largest) fits with FP32 staging: K steps of 32
// per 16-row block, 1 KiB per term, mass steps ceil(ceil(n_q,m / 4) / 8),
// conductivity ceil(ceil(n_q,c / 4) / floor(8 / (d(d+1)/2))).
constexpr bool split_ok(int D, int P, int nqm, int nqc)
{
    return mfma_variant(D, P, nqm, nqc) && tile_size(D, P) != 16 && nqm > 0 && nqc > 0 &&
           staged_lds_bytes(D, P, nqm, nqc, 4,
                            ((nqm + 3) / 4 + 7) / 8 + ((nqc + 3) / 4 + 8 / (D * (D + 1) / 2) - 1) / (8 / (D * (D + 1) / 2)),
                            3 * 1024) <= kLdsBytes;
}

struct FormArgs {
    FormInputs in;
    const int32_t *conn;  // [np][n_elem]
    const void *Qm, *Qc;  // compute-type tables [ns][nqm], [ns][nqc][ng]
    double *Vm, *Vc;      // [ns][n_elem] outputs (either may be null)
};

struct FusedArgs {
    FormInputs in;
    const int32_t *tconn;       // [np][n_elem], tile order
    const int32_t *elem_order;  // tile position -> element id
    const void *Qm, *Qc;
    const void *Qfrag;          // Q^T in MFMA B-operand order (matrix-core variant)
    int64_t qfrag_vec16;        // size of Qfrag in 16-byte units
    double qinv_m, qinv_c;      // inverse power-of-two scales of the FP16 Q tables (1 otherwise)
    const uint32_t *rec;        // output units (plan_format.hpp)
    const int64_t *rec_ptr;     // [n_tiles + 1]
    const int64_t *rec_mid;     // [n_tiles] first single unit of each tile
    int carry_cap;              // LDS carry entries of a workgroup
    int pad0;
    double *sink;               // write target of idle lanes (at least 1024 doubles)
    double *M, *C;              // CSR values (either may be null)
    double *part;               // [n_partials][2] partials of shared slots (mass, conductivity)
    uint32_t bytes_vals;        // 8 * nnz (buffer-store bound of M and C)
    uint32_t bytes_part;        // 16 * n_partials (buffer-store bound of part)
    int buf_ok;                 // both bounds below 2^31: the stores may go through buffer resources
    // isoparametric kernels only (null otherwise)
    const double *dphi;         // [n_q][np][dim] reference gradients at the (shared) rule's nodes
    const double *Kq;           // [nq_kq][ng][n_elem] conductivity tensor per node, mesh order (or null)
    int nq_kq;                  // nodes of the caller's stiffness rule
    int pad1;
};

// Jobs of one launch: a single assembly is carried by value in `one`
// (n_jobs == 0); a batch of assemblies that share a kernel (same shape,
// rules and precision form) is a device array `jobs` with the running tile
// count tile_end[j] (exclusive prefix). Workgroups map a global tile index
// to (job, tile of the job). The tiles are cut into chains (a job's chains
// in its plan's order, jobs one after the other); a workgroup takes whole
// chains, so that its tiles are one range of global tiles.
struct JobTable {
    FusedArgs one;
    const FusedArgs *jobs;
    const int64_t *tile_end;
    int n_jobs;
    int64_t n_tiles;
    int buf_stores;             // every job has buf_ok
    const int64_t *chain_ptr;   // [n_chains + 1] first (global) tile of each chain
    int64_t n_chains;
};

struct FixupArgs {
    int64_t n_fix;
    const int32_t *fix_target;  // [n_fix] shared upper slot (ascending)
    const int32_t *fix_mirror;  // [n_fix] its mirror slot (== target on the diagonal)
    const int64_t *part_ptr;    // [n_fix + 1] partial ranges, ascending tile order
    const double *part;         // [n_partials][2]: (mass, conductivity) partial pairs
    double *M, *C;
};

struct FixupTable {
    FixupArgs one;
    const FixupArgs *jobs;
    const int64_t *fix_end;  // running count of fix-up outputs (exclusive prefix)
    int n_jobs;
    int64_t n_fix;
};

bool form_supported(int D, int P, int nqm, int nqc);
// Tile-plan parameters of the fused kernel of a shape: tile size, chains (the
// workgroups of one launch on a device with `cus` compute units) and the LDS
// carry entries left beside the kernel's other LDS (`lds_max` bytes per
// workgroup) for every precision form with Q^T sizes qfrag_vec16[form].
TileParams fused_tile_params(int D, int P, int nqm, int nqc, int cus, size_t lds_max, const int64_t (&qfrag_vec16)[5]);
hipError_t launch_form(const FormArgs &a, int D, int P, int nqm, int nqc, int precision, hipStream_t st);
hipError_t launch_fused(const JobTable &jt, int D, int P, int nqm, int nqc, int precision, hipStream_t st);
hipError_t launch_fixup(const FixupTable &ft, hipStream_t st);
// The isoparametric assembly in one pass (the matrix-core kernel with X formed
// per quadrature node from every node's position): shapes whose kernel stages
// Q^T in LDS, one rule for both matrices (nqm == nqc, identical tables), FP64.
// fused_iso_fits: compiled, and the kernel's LDS with the plan's carry entries
// fits a workgroup.
bool fused_iso_fits(int D, int P, int nqm, int nqc, int64_t qfrag_vec16, int carry_cap);
hipError_t launch_fused_iso(const JobTable &jt, int D, int P, int nqm, int nqc, hipStream_t st);
// Reduction of externally formed local matrices with the plan's units: Tm, Tc are
// [n_elem / 64][NS][64] pair-major blocks of 64 tile positions (either may be null).
hipError_t launch_staged_reduce(const JobTable &jt, int D, int P, const double *Tm, const double *Tc, hipStream_t st);

// Argument blocks of one assembly with `plan` (validates the coefficients and
// the precision form). part: [2][n_partials] partial sums; flags: one int.
qxa_status make_fused_args(qxa_plan p, const qxa_coeff *mass, const qxa_coeff *stiff, int precision, double *M,
                           double *C, double *part, int *flags, FusedArgs &a, FixupArgs &f);

}  // namespace qxa
