// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/qxa.h"
#include "plan_format.hpp"

namespace qxa {

constexpr int kMaxNp = 20;  // P3 tetrahedra
constexpr int kMaxNq = 64;
constexpr int kSinkDoubles = 1024;

inline int n_local(int dim, int order)
{
    int n = 1;
    for (int k = 1; k <= dim; ++k) n = n * (order + k) / k;
    return n;
}
inline int n_sym(int np) { return np * (np + 1) / 2; }
inline int n_geo(int dim) { return dim * (dim + 1) / 2; }

// Host plan building blocks ------------------------------------------------
// Allocator that default-initialises (leaves trivial elements unset), for
// large host arrays that are filled in parallel right after they are sized.
template <class T>
struct DefaultInit : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = DefaultInit<U>;
    };
    DefaultInit() = default;
    template <class U>
    DefaultInit(const DefaultInit<U> &) noexcept
    {
    }
    template <class U>
    void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value)
    {
        ::new (static_cast<void *>(p)) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a)
    {
        ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
    }
};
template <class T>
using hvec = std::vector<T, DefaultInit<T>>;

// Host threads of the plan builders (at most 16).
inline unsigned host_threads() { return std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

// f(lo, hi) over [0, n) cut into one contiguous range per host thread.
template <class F>
void parallel_for(int64_t n, F &&f, int64_t serial_below = 2048)
{
    const unsigned nt = host_threads();
    if (n < serial_below || nt == 1) {
        f(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t lo = std::min<int64_t>(n, t * chunk), hi = std::min<int64_t>(n, lo + chunk);
        if (lo < hi) th.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto &x : th) x.join();
}

// Sort of a random-access range on the host threads: ranges sorted in
// parallel, then merged pairwise (the result equals std::sort's for a strict
// weak order without ties).
template <class It>
void parallel_sort(It first, It last)
{
    const int64_t n = last - first;
    const unsigned nt = host_threads();
    if (n < (int64_t(1) << 16) || nt == 1) {
        std::sort(first, last);
        return;
    }
    int64_t w = (n + nt - 1) / nt;
    parallel_for(nt, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) std::sort(first + std::min(n, k * w), first + std::min(n, (k + 1) * w));
    }, 0);
    for (; w < n; w *= 2) {
        const int64_t pairs = (n + 2 * w - 1) / (2 * w);
        parallel_for(pairs, [&](int64_t a, int64_t b) {
            for (int64_t k = a; k < b; ++k) {
                const int64_t lo = k * 2 * w, mid = std::min(n, lo + w), hi = std::min(n, lo + 2 * w);
                if (mid < hi) std::inplace_merge(first + lo, first + mid, first + hi);
            }
        }, 0);
    }
}

// Error reporting ---------------------------------------------------------
qxa_status fail(qxa_status code, const std::string &msg);
qxa_status hip_fail(hipError_t e, const char *what);
#define QXA_HIP(call)                                          \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return ::qxa::hip_fail(_e, #call); \
    } while (0)

// Reference element tables of Algorithm 2 (Phi, J_q, Q) ---------------------
// Built-in symmetric quadrature rules (rules_builtin.cpp, generated).
struct BuiltinRule {
    int dim, degree, n_q;
    const double *points, *weights;
};
extern const BuiltinRule k_builtin_rules[];
extern const int k_n_builtin_rules;

struct RefTables {
    int dim = 0, order = 0, np = 0, ns = 0, ng = 0;
    int nq_m = 0, nq_c = 0;        // nodes of the compiled rules (the tables below)
    int nq_m_in = 0, nq_c_in = 0;  // nodes of the caller's rules (a prefix of the compiled ones)
    std::vector<double> w_m, w_c;     // quadrature weights
    std::vector<double> phi_m;        // [np][nq_m]: Phi for the mass rule
    std::vector<double> phi_c;        // [np][nq_c]: Phi at the stiffness rule (for u_h)
    std::vector<double> dphi_c;       // [nq_c][np][dim]: J_q, reference gradients at the stiffness rule
    std::vector<double> dphi_m;       // [nq_m][np][dim]: the same at the mass rule (curved geometry)
    std::vector<double> Qm;           // [ns][nq_m]           symmetric-pair rows of Phi (.) Phi
    std::vector<double> Qc;           // [ns][nq_c][ng]       symmetric-pair rows of [J_q (x) J_q], symmetric W
    std::vector<int> pair_a, pair_b;  // sym pair s -> (a, b), a <= b
    bool stiff_const_grad = false;    // J_q identical for all q (P1): Q_c columns repeat
};

// Builds the tables from the rules, each padded to the compiled size chosen by
// compiled_rule_sizes; returns QXA_OK or an error.
qxa_status build_ref_tables(int dim, int order, const qxa_quad &mr, const qxa_quad &cr, RefTables &out);

// Largest rules the compiled kernels take (in nodes).
constexpr int kMaxRule2D = 16, kMaxRule3D = 32;
// The compiled (mass, stiffness) rule sizes of least work (n_q,m + d(d+1)/2
// n_q,c) that hold rules of nqm and nqc nodes; false if none does.
bool compiled_rule_sizes(int dim, int order, int nqm, int nqc, int &cm, int &cc);

// Lagrange basis of the reference simplex in barycentric product form.
void lagrange_eval(int dim, int order, const double *xhat, double *phi, double *dphi /* [np][dim] */);

// Host-built plan data ---------------------------------------------------
struct HostPlan {
    int64_t n_nodes = 0, n_elem = 0, nnz = 0;
    std::vector<int64_t> row_ptr;
    hvec<int32_t> col_idx;
    // Element-entry -> CSR slot for every symmetric pair s of every element:
    // perm[s * n_elem + e] = slot of (min(i,j), max(i,j)) (upper triangle).
    hvec<uint32_t> perm_sym;
    hvec<uint32_t> mirror;            // [nnz]: slot of (j, i) for slot (i, j)
};

qxa_status build_host_plan(int dim, int order, int64_t n_nodes, int64_t n_elem, const int32_t *conn, HostPlan &hp);

// Tile decomposition for the fused kernel.
struct TileParams {
    int T = 64;            // elements per tile
    int64_t chains = 256;  // chains (workgroups of one launch) the tiles are split into
    int carry_cap = 0;     // LDS carry entries of a workgroup
    bool pair_units = true;
    // > 1: chains of runs of run_len consecutive tiles, one chain per workgroup, the
    // workgroups of one XCD on neighbouring runs at the same time (build_tile_plan)
    int run_len = 0;
};

struct TilePlan {
    int T = 0;
    int64_t n_tiles = 0;
    hvec<int32_t> elem_order;         // tile position -> element id (Morton order of centroids)
    hvec<int32_t> tconn;              // [np][n_elem] connectivity in tile order
    // Chain c holds tiles chain_ptr[c] .. chain_ptr[c+1] - 1; a workgroup
    // processes whole chains, so carries never cross a chain.
    std::vector<int64_t> chain_ptr;   // [n_chains + 1]
    int carry_cap = 0, carry_used = 0;
    // Output units of tile t (plan_format.hpp): rec_ptr[t] .. rec_ptr[t+1] - 1,
    // pair units up to rec_mid[t]. Outputs are ordered CSR outputs first in
    // ascending slot order (upper and mirror entries separately), then carry
    // outputs, then partials; among single units, outputs of several units
    // come first.
    hvec<uint32_t> rec;               // [4 * n_units]
    std::vector<int64_t> rec_ptr;     // [n_tiles + 1] (in units)
    std::vector<int64_t> rec_mid;     // [n_tiles]
    // Partials of shared upper slot k (CSR order) are part_ptr[k] ..
    // part_ptr[k+1] - 1, in ascending tile order.
    std::vector<int64_t> part_ptr;    // [n_shared + 1]
    // fix-up: shared upper slot k (ascending CSR order) and its mirror slot
    std::vector<int32_t> fix_target;  // [n_shared]
    std::vector<int32_t> fix_mirror;  // [n_shared]
    int64_t n_shared = 0;
    int64_t n_partials = 0;
    int64_t n_outputs = 0;            // outputs of all tiles
    int64_t n_carry_reads = 0;        // outputs that read a carry entry
    int64_t n_ext_units = 0;          // single units continued in the next unit
    int64_t n_empty_units = 0;        // units that store nothing (holes of that layout)
};

qxa_status build_tile_plan(int dim, int order, int64_t n_nodes, int64_t n_elem, const int32_t *conn,
                           const double *coords, const HostPlan &hp, const TileParams &prm, TilePlan &tp);
qxa_status check_tile_plan(int np, int64_t n_elem, const HostPlan &hp, const TilePlan &tp);
// The tile-plan figures of qxa_plan_info (n_tiles .. carry_used); other fields untouched.
void tile_plan_stats(const TilePlan &tp, qxa_plan_info &o);

// First-fit sub-allocator over one device allocation (256-byte granules,
// free ranges coalesced). Thread-safe. Serves the server's resident plans and
// job buffers so that their total never exceeds the budget it was given and
// no allocation or free in the serving loop synchronises the device.
class DevArena {
public:
    ~DevArena();
    qxa_status init(size_t bytes);
    void *alloc(size_t bytes);  // nullptr when no free range is large enough
    void release(void *p);
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t capacity() const { return cap_; }
    static size_t granule(size_t bytes) { return (bytes + 255) & ~size_t(255); }

private:
    std::mutex mu_;
    char *base_ = nullptr;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;            // offset -> length
    std::unordered_map<size_t, size_t> live_;  // offset -> length
};

// Everything of a plan that is computed on the host (reference tables, CSR
// pattern, tile plan, operand-ordered Q^T), before any device allocation.
struct PlanStaging {
    int device = 0;
    RefTables ref;
    HostPlan hp;
    TilePlan tp;
    bool mfma = false;
    std::vector<uint8_t> frag[5];
    double f16_qinv[2] = {1.0, 1.0};
    std::vector<double> tab;
    std::vector<float> tabf;
    size_t off_wm = 0, off_wc = 0, off_phim = 0, off_phic = 0, off_qm = 0, off_qc = 0, off_dphic = 0, off_dphim = 0;
};

qxa_status plan_stage(qxa_mesh mesh, const qxa_quad &mr, const qxa_quad &cr, PlanStaging &out);
// Uploads a staged plan. With an arena every buffer comes from it (QXA_E_NOMEM
// when it is full) and the plan keeps no scratch of its own (own_scratch =
// false: the caller brings partial-sum and flag buffers per assembly).
qxa_status plan_upload(qxa_mesh mesh, const PlanStaging &stg, DevArena *arena, bool own_scratch, qxa_plan *out);
// Device bytes of a staged plan's largest arrays (a lower bound of its size).
size_t plan_bytes_lower_bound(const PlanStaging &stg);

}  // namespace qxa

// Opaque handles ------------------------------------------------------------
struct qxa_mesh_s {
    uint64_t serial = 0;          // unique per mesh created in this process
    int device = 0;
    int dim = 0, order = 0, np = 0;
    int64_t n_nodes = 0, n_elem = 0;
    double *d_coords = nullptr;   // [dim][n_nodes]
    int32_t *d_conn = nullptr;    // [np][n_elem]
    std::vector<int32_t> h_conn;  // host copy for plan building
    std::vector<double> h_coords; // host copy for plan building (element order)
    size_t device_bytes = 0;
};

struct qxa_plan_s {
    qxa_mesh mesh = nullptr;
    int device = 0;                  // destroy never reads the mesh (it may be gone)
    qxa::DevArena *arena = nullptr;  // device buffers come from here when set
    qxa::RefTables ref;
    int64_t nnz = 0;
    int64_t *d_row_ptr = nullptr;
    int32_t *d_col_idx = nullptr;
    // fused-path tile plan (device copies)
    int tile_T = 0;
    int64_t n_tiles = 0, n_shared = 0, n_partials = 0, n_chains = 0;
    int carry_cap = 0;
    qxa_plan_info stats{};  // tile-plan figures reported by qxa_plan_get_info
    int32_t *d_tconn = nullptr, *d_elem_order = nullptr;
    uint32_t *d_rec = nullptr;
    int64_t *d_rec_ptr = nullptr, *d_rec_mid = nullptr;
    int64_t *d_chain_ptr = nullptr;
    std::vector<int64_t> h_chain_ptr;  // host copy (batched launches concatenate the chains of their jobs)
    int64_t *d_part_ptr = nullptr;
    int32_t *d_fix_target = nullptr, *d_fix_mirror = nullptr;
    int64_t n_fix = 0;
    double *d_sink = nullptr;     // write target of idle lanes (kSinkDoubles)
    double *d_part = nullptr;     // [2][n_partials]
    // Q^T in MFMA operand order, one block per precision form (FP64, FP32,
    // F16X2, BF16X2, BF16X3), sizes in 16-byte units
    void *d_qfrag[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int64_t qfrag_vec16[5] = {0, 0, 0, 0, 0};
    double f16_qinv[2] = {1.0, 1.0};  // FP16 tables are stored as Q * 2^k (mass, stiffness)
    double *d_tables = nullptr;   // device copy of w, Phi, Qm, Qc (FP64)
    float *d_tables_f = nullptr;  // FP32 copy
    size_t off_wm = 0, off_wc = 0, off_phim = 0, off_phic = 0, off_qm = 0, off_qc = 0, off_dphic = 0, off_dphim = 0;
    double *d_Tiso = nullptr;     // [2][n_elem / 64][ns][64] isoparametric local matrices of the tile positions (first use)
    double *d_V = nullptr;        // [2][ns][n_elem] formation-only buffer (allocated on first use)
    // conductivity tensor product (built on first use): local matrices [n_elem][np][np]
    // and, per CSR slot (both triangles), its element entries (index into d_T) in
    // ascending element order
    double *d_T = nullptr;
    int32_t *d_ns_ptr = nullptr;  // [nnz + 1]
    int32_t *d_ns_items = nullptr;
    // load vector (built on first use): element vectors [np][n_elem] and, per node,
    // its element entries in ascending element order
    double *d_Fe = nullptr;
    int32_t *d_nf_ptr = nullptr;  // [n_nodes + 1]
    int32_t *d_nf_items = nullptr;
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
