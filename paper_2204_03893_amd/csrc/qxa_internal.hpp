// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qxa.h"

namespace qxa {

constexpr int kMaxNp = 20;  // P3 tetrahedra
constexpr int kMaxNq = 64;

inline int n_local(int dim, int order)
{
    int n = 1;
    for (int k = 1; k <= dim; ++k) n = n * (order + k) / k;
    return n;
}
inline int n_sym(int np) { return np * (np + 1) / 2; }
inline int n_geo(int dim) { return dim * (dim + 1) / 2; }

// Error reporting ---------------------------------------------------------
qxa_status fail(qxa_status code, const std::string &msg);
qxa_status hip_fail(hipError_t e, const char *what);
#define QXA_HIP(call)                                          \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return ::qxa::hip_fail(_e, #call); \
    } while (0)

// Reference element tables (Algorithm 2, Lines 1-3) ---------------------
struct RefTables {
    int dim = 0, order = 0, np = 0, ns = 0, ng = 0;
    int nq_m = 0, nq_c = 0;
    std::vector<double> w_m, w_c;     // quadrature weights
    std::vector<double> phi_m;        // [np][nq_m]: Phi for the mass rule
    std::vector<double> phi_c;        // [np][nq_c]: Phi at the stiffness rule (for u_h)
    std::vector<double> Qm;           // [ns][nq_m]           symmetric-pair rows of Phi (.) Phi
    std::vector<double> Qc;           // [ns][nq_c][ng]       symmetric-pair rows of [J_q (x) J_q], symmetric W
    std::vector<int> pair_a, pair_b;  // sym pair s -> (a, b), a <= b
    bool stiff_const_grad = false;    // J_q identical for all q (P1): Q_c columns repeat
};

// Builds the tables from the rules; returns QXA_OK or an error.
qxa_status build_ref_tables(int dim, int order, const qxa_quad &mr, const qxa_quad &cr, RefTables &out);

// Lagrange basis of the reference simplex in barycentric product form.
void lagrange_eval(int dim, int order, const double *xhat, double *phi, double *dphi /* [np][dim] */);

// Host-built plan data ---------------------------------------------------
struct HostPlan {
    int64_t n_nodes = 0, n_elem = 0, nnz = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col_idx;
    // Element-entry -> CSR slot for every symmetric pair s of every element:
    // perm[s * n_elem + e] = slot of (min(i,j), max(i,j)) (upper triangle).
    std::vector<uint32_t> perm_sym;
    // Segments over all CSR slots: slot t reads the contribution list of its
    // upper-triangle twin src_upper[t]; seg_ptr over upper slots lists the
    // V indices s*n_elem + e in ascending (e, s) order.
    std::vector<uint32_t> seg_ptr;    // [nnz + 1], empty segments for lower slots
    std::vector<uint32_t> seg_val;    // V indices
    std::vector<uint32_t> src_upper;  // [nnz]
};

qxa_status build_host_plan(int dim, int order, int64_t n_nodes, int64_t n_elem, const int32_t *conn, HostPlan &hp);

}  // namespace qxa

// Opaque handles ------------------------------------------------------------
struct qxa_mesh_s {
    int device = 0;
    int dim = 0, order = 0, np = 0;
    int64_t n_nodes = 0, n_elem = 0;
    double *d_coords = nullptr;   // [dim][n_nodes]
    int32_t *d_conn = nullptr;    // [np][n_elem]
    std::vector<int32_t> h_conn;  // host copy for plan building
    size_t device_bytes = 0;
};

struct qxa_plan_s {
    qxa_mesh mesh = nullptr;
    qxa::RefTables ref;
    int64_t nnz = 0;
    int64_t *d_row_ptr = nullptr;
    int32_t *d_col_idx = nullptr;
    uint32_t *d_seg_ptr = nullptr;
    uint32_t *d_seg_val = nullptr;
    uint32_t *d_src_upper = nullptr;
    double *d_tables = nullptr;   // device copy of w, Phi, Qm, Qc (FP64)
    float *d_tables_f = nullptr;  // FP32 copy
    size_t off_wm = 0, off_wc = 0, off_phim = 0, off_phic = 0, off_qm = 0, off_qc = 0;
    double *d_V = nullptr;        // [2][ns][n_elem] element-matrix buffer (two-pass path)
    int *d_flags = nullptr;       // device status flags (non-finite)
    size_t device_bytes = 0;
    double build_ms = 0.0;
    // optional per-kernel event timing
    bool timing = false;
    struct Rec {
        const char *name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
};

namespace qxa {
// Records events around a launch when the plan has timing enabled.
struct TimedLaunch {
    qxa_plan p;
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(qxa_plan p_, const char *n, hipStream_t s_) : p(p_), name(n), s(s_)
    {
        if (p->timing) {
            hipEventCreate(&a);
            hipEventCreate(&b);
            hipEventRecord(a, s);
        }
    }
    ~TimedLaunch()
    {
        if (p->timing) {
            hipEventRecord(b, s);
            p->recs.push_back({name, a, b});
        }
    }
};
}  // namespace qxa
