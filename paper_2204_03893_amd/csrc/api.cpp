// C-ABI of the assembly library: argument validation, ownership, launches.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "kernels_twopass.hpp"
#include "qxa_internal.hpp"

namespace qxa {

static thread_local std::string g_err;

qxa_status fail(qxa_status code, const std::string &msg)
{
    g_err = msg;
    return code;
}

qxa_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? QXA_E_NOMEM : QXA_E_HIP;
}

template <class T>
static qxa_status dev_alloc(T **p, size_t count, size_t &acct)
{
    *p = nullptr;
    if (count == 0) return QXA_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    acct += count * sizeof(T);
    return QXA_OK;
}

template <class T>
static qxa_status upload(T **p, const T *src, size_t count, size_t &acct)
{
    qxa_status st = dev_alloc(p, count, acct);
    if (st || count == 0) return st;
    QXA_HIP(hipMemcpy(*p, src, count * sizeof(T), hipMemcpyHostToDevice));
    return QXA_OK;
}

// Plan buffers: from the plan's arena when it has one, else hipMalloc.
template <class T>
static qxa_status plan_alloc(qxa_plan p, T **ptr, size_t count)
{
    if (!p->arena) return dev_alloc(ptr, count, p->device_bytes);
    *ptr = nullptr;
    if (count == 0) return QXA_OK;
    *ptr = static_cast<T *>(p->arena->alloc(count * sizeof(T)));
    if (!*ptr) return fail(QXA_E_NOMEM, "device memory budget exhausted");
    p->device_bytes += DevArena::granule(count * sizeof(T));
    return QXA_OK;
}
template <class T>
static qxa_status plan_upload_buf(qxa_plan p, T **ptr, const T *src, size_t count)
{
    qxa_status st = plan_alloc(p, ptr, count);
    if (st || count == 0) return st;
    QXA_HIP(hipMemcpy(*ptr, src, count * sizeof(T), hipMemcpyHostToDevice));
    return QXA_OK;
}
static void plan_free(qxa_plan p, void *ptr)
{
    if (!ptr) return;
    if (p->arena) p->arena->release(ptr);
    else hipFree(ptr);
}
// Frees the buffers a lazily built map consists of and clears their pointers, so that
// a build that failed part-way is redone on the next call instead of being used.
template <class... T>
static void plan_drop(qxa_plan p, T **...ptrs)
{
    (plan_free(p, *ptrs), ...);
    ((*ptrs = nullptr), ...);
}

// n_nodes, n_elem: the field's length for the nodal and per-(q, e) kinds (a field of
// zero length may be null); nq: the rows of a per-(q, e) field (the caller's rule).
static qxa_status to_coeff(const qxa_coeff *c, CoeffDev &out, const char *which, int64_t n_nodes, int64_t n_elem,
                           int nq)
{
    if (!c) {
        out = CoeffDev{0, 0, 0.0, 0.0, 0.0, 0.0, nullptr, nq, 0};
        return QXA_OK;
    }
    if (c->kind < 0 || c->kind > 2) return fail(QXA_E_INVALID, std::string(which) + " coefficient: bad kind");
    if (c->law < 0 || c->law > 2) return fail(QXA_E_INVALID, std::string(which) + " coefficient: bad law");
    if (c->kind != 0 && !c->field && (c->kind == 1 ? n_nodes : n_elem) > 0)
        return fail(QXA_E_INVALID, std::string(which) + " coefficient: null field");
    if (c->kind == 0 && !std::isfinite(c->value))
        return fail(QXA_E_NONFINITE, std::string(which) + " coefficient: non-finite constant");
    if (c->tensor_q)
        return fail(QXA_E_UNSUPPORTED, std::string(which) +
                                           " coefficient: a tensor per quadrature node is taken by the "
                                           "isoparametric path (qxa_assemble_iso) only");
    out = CoeffDev{c->kind, c->law, c->value, c->a[0], c->a[1], c->a[2], c->field, nq, 0};
    return QXA_OK;
}

// The conductivity tensor of a stiffness coefficient (host array, d(d+1)/2 upper
// entries); the mass coefficient has none.
static qxa_status to_tensor(const qxa_coeff *mass, const qxa_coeff *stiff, int dim, int &aniso, double (&K)[6])
{
    aniso = 0;
    for (int g = 0; g < 6; ++g) K[g] = 0.0;
    if (mass && mass->tensor) return fail(QXA_E_INVALID, "mass coefficient: a tensor applies to conductivity only");
    if (!stiff || !stiff->tensor) return QXA_OK;
    const int ng = dim * (dim + 1) / 2;
    for (int g = 0; g < ng; ++g) {
        if (!std::isfinite(stiff->tensor[g])) return fail(QXA_E_NONFINITE, "conductivity tensor: non-finite entry");
        K[g] = stiff->tensor[g];
    }
    aniso = 1;
    return QXA_OK;
}

static uint16_t bf16_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return uint16_t(u >> 16);
}
static float bf16_value(uint16_t b)
{
    const uint32_t u = uint32_t(b) << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}
static uint16_t f16_bits(float x)
{
    const _Float16 h = _Float16(x);
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}
static float f16_value(uint16_t b)
{
    _Float16 h;
    std::memcpy(&h, &b, 2);
    return float(h);
}

// Q^T fragments in MFMA B-operand order for every precision form.
//   FP64 / FP32 (16x16x4): [ks][nb][lane], lane l of block (ks, nb) holds
//     Q[s = 16 nb + l % 16][k = 4 ks + l / 16];
//   split forms (16x16x32): [component][ks][nb][lane][8], lane l holds
//     Q[s = 16 nb + l % 16][k = 32 ks + 8 (l / 16) + t], t = 0..7, as the
//     hi / lo (/ mid) terms of its 16-bit split.
// Mass block first, then conductivity. The K order is chosen so that the four
// lanes holding one element need the weighted coefficients of nodes
// q = 4 m + j only (j = l / 16):
//   16x16x4: mass k = q; conductivity k = g * NQP + q, NQP = n_q rounded up to 4;
//   16x16x32: segment (ks, j) of 8 slots holds QPS = 8 / G groups of G slots,
//     slot t = node q = 4 (QPS ks + t / G) + j, component t % G (G = 1 for the
//     mass, d(d+1)/2 for the conductivity), unused slots zero.
// Zero outside the tables.
int qc_pad(int nq) { return (nq + 3) / 4 * 4; }
int split_blocks(int nq, int G) { return ((nq + 3) / 4 + 8 / G - 1) / (8 / G); }

static void build_qfrags(const RefTables &T, std::vector<uint8_t> (&out)[5], double (&f16_qinv)[2])
{
    const int nb_ = (T.ns + 15) / 16, kc = T.nq_c * T.ng;
    // FP16 keeps 5 exponent bits: each table is scaled by 2^k so that its largest
    // entry lies in [2^13, 2^14), keeping small products out of the subnormals
    double f16_scale[2];
    for (int blk = 0; blk < 2; ++blk) {
        const std::vector<double> &Q = blk == 0 ? T.Qm : T.Qc;
        double mx = 0.0;
        for (double x : Q) mx = std::max(mx, std::fabs(x));
        const int e = mx > 0.0 ? std::ilogb(mx) : 0;
        f16_scale[blk] = std::ldexp(1.0, 13 - e);
        f16_qinv[blk] = std::ldexp(1.0, e - 13);
    }
    // entry (s, q, g) of the mass (blk 0, g = 0) or conductivity (blk 1) table
    auto qent = [&](int blk, int s, int q, int g) -> double {
        if (s >= T.ns) return 0.0;
        if (blk == 0) return q < T.nq_m && g == 0 ? T.Qm[size_t(s) * T.nq_m + q] : 0.0;
        if (q >= T.nq_c || g >= T.ng) return 0.0;
        return T.Qc[size_t(s) * kc + size_t(q) * T.ng + g];
    };
    // entry (s, k) in the K order of the 16x16x4 forms
    auto qval = [&](int blk, int s, int k) -> double {
        if (blk == 0) return qent(0, s, k, 0);
        const int nqp = qc_pad(T.nq_c);
        return qent(1, s, k % nqp, k / nqp);
    };
    // entry (s, k) in the K order of the split forms
    auto qval_split = [&](int blk, int s, int k) -> double {
        const int G = blk == 0 ? 1 : T.ng, qps = 8 / G;
        const int ks = k / 32, j = (k % 32) / 8, t = k % 8, u = t / G;
        if (u >= qps) return 0.0;
        return qent(blk, s, 4 * (qps * ks + u) + j, t % G);
    };
    // plain forms
    for (int f = 0; f < 2; ++f) {
        std::vector<uint8_t> &o = out[f];
        for (int blk = 0; blk < 2; ++blk) {
            const int kb = blk == 0 ? T.nq_m : T.ng * qc_pad(T.nq_c);
            const int ks_n = (kb + 3) / 4;
            for (int ks = 0; ks < ks_n; ++ks)
                for (int nb = 0; nb < nb_; ++nb)
                    for (int l = 0; l < 64; ++l) {
                        const double v = qval(blk, 16 * nb + l % 16, 4 * ks + l / 16);
                        if (f == 0) {
                            const uint8_t *b = reinterpret_cast<const uint8_t *>(&v);
                            o.insert(o.end(), b, b + 8);
                        } else {
                            const float x = float(v);
                            const uint8_t *b = reinterpret_cast<const uint8_t *>(&x);
                            o.insert(o.end(), b, b + 4);
                        }
                    }
        }
        while (o.size() % 16) o.push_back(0);
    }
    // split forms: F16X2 (index 2), BF16X2 (3), BF16X3 (4)
    for (int f = 2; f < 5; ++f) {
        const int nc = f == 4 ? 3 : 2;
        std::vector<uint8_t> &o = out[f];
        for (int blk = 0; blk < 2; ++blk) {
            const int ks_n = blk == 0 ? split_blocks(T.nq_m, 1) : split_blocks(T.nq_c, T.ng);
            for (int c = 0; c < nc; ++c)
                for (int ks = 0; ks < ks_n; ++ks)
                    for (int nb = 0; nb < nb_; ++nb)
                        for (int l = 0; l < 64; ++l)
                            for (int t = 0; t < 8; ++t) {
                                double v = qval_split(blk, 16 * nb + l % 16, 32 * ks + 8 * (l / 16) + t);
                                uint16_t comp[3];
                                if (f == 2) {
                                    v *= f16_scale[blk];
                                    comp[0] = f16_bits(float(v));
                                    comp[1] = f16_bits(float(v - double(f16_value(comp[0]))));
                                } else {
                                    comp[0] = bf16_bits(float(v));
                                    const double r1 = v - double(bf16_value(comp[0]));
                                    comp[1] = bf16_bits(float(r1));
                                    comp[2] = bf16_bits(float(r1 - double(bf16_value(comp[1]))));
                                }
                                o.push_back(uint8_t(comp[c] & 0xff));
                                o.push_back(uint8_t(comp[c] >> 8));
                            }
        }
    }
}

// Device scratch of the allocation-free formation entry point: the pair-major
// element matrices V_m, V_c (2 * n_sym * n_elem doubles) live here instead of a
// buffer allocated by the plan. Every GPU the library runs on holds its own copy
// for the life of the process. In host code `scratch` only names the symbol:
// kernels get the per-device address resolved by hipGetSymbolAddress.
constexpr size_t kScratchDoubles = size_t(8) << 20;  // 64 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[64] = {};  // per device, resolved once at mesh creation

// Resolves this device's scratch address (the device must be current). Once per device.
static qxa_status resolve_scratch(int device)
{
    if (device < 0 || device >= 64) return fail(QXA_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return QXA_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = static_cast<double *>(ptr);
    return QXA_OK;
}

static double *scratch_of(int device)
{
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace qxa

using namespace qxa;

extern "C" {

const char *qxa_last_error(void) { return g_err.c_str(); }
const char *qxa_version(void) { return "qxa 0.1 (gfx950)"; }

qxa_status qxa_mesh_create(int device, int dim, int order, int64_t n_nodes, const double *coords, int64_t n_elem,
                           const int32_t *conn, int mem, qxa_mesh *out)
{
    if (!out) return fail(QXA_E_INVALID, "out is null");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(QXA_E_INVALID, "dim must be 2 or 3");
    if (order < 1 || order > 3) return fail(QXA_E_INVALID, "order must be 1, 2 or 3");
    if (n_nodes < dim + 1 || n_elem < 0) return fail(QXA_E_INVALID, "bad sizes");
    if (n_nodes >= (int64_t(1) << 31)) return fail(QXA_E_UNSUPPORTED, "more than 2^31 nodes");
    if (!coords || (n_elem > 0 && !conn)) return fail(QXA_E_INVALID, "null coords/conn");
    if (mem != QXA_MEM_HOST && mem != QXA_MEM_DEVICE) return fail(QXA_E_INVALID, "bad mem flag");
    QXA_HIP(hipSetDevice(device));
    {
        const qxa_status sst = resolve_scratch(device);  // set-up of this device's scratch address
        if (sst) return sst;
    }
    const int np = n_local(dim, order);
    std::vector<double> hx;
    std::vector<int32_t> hc;
    const double *X = coords;
    const int32_t *Cn = conn;
    if (mem == QXA_MEM_DEVICE) {
        hx.resize(size_t(dim) * n_nodes);
        hc.resize(size_t(np) * n_elem);
        QXA_HIP(hipMemcpy(hx.data(), coords, hx.size() * sizeof(double), hipMemcpyDeviceToHost));
        if (n_elem) QXA_HIP(hipMemcpy(hc.data(), conn, hc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        X = hx.data();
        Cn = hc.data();
    }
    for (size_t k = 0; k < size_t(dim) * n_nodes; ++k)
        if (!std::isfinite(X[k])) return fail(QXA_E_NONFINITE, "non-finite node coordinate at index " + std::to_string(k));
    for (int64_t e = 0; e < n_elem; ++e) {
        int32_t v[kMaxNp];
        for (int i = 0; i < np; ++i) {
            v[i] = Cn[size_t(i) * n_elem + e];
            if (v[i] < 0 || v[i] >= n_nodes)
                return fail(QXA_E_INDEX, "element " + std::to_string(e) + ": node index out of range");
            for (int j = 0; j < i; ++j)
                if (v[j] == v[i]) return fail(QXA_E_INDEX, "element " + std::to_string(e) + ": repeated node");
        }
        // |det B_e| against the longest edge from vertex 0 (B_e invertible, Section 3)
        double B[3][3], lmax = 0.0;
        for (int c = 0; c < dim; ++c) {
            double l2 = 0.0;
            for (int r = 0; r < dim; ++r) {
                B[r][c] = X[size_t(r) * n_nodes + v[c + 1]] - X[size_t(r) * n_nodes + v[0]];
                l2 += B[r][c] * B[r][c];
            }
            lmax = std::max(lmax, std::sqrt(l2));
        }
        const double det = dim == 2 ? B[0][0] * B[1][1] - B[0][1] * B[1][0]
                                    : B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                                          B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                                          B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
        if (!(std::fabs(det) > 1e-14 * std::pow(lmax, dim)))
            return fail(QXA_E_DEGENERATE, "element " + std::to_string(e) + " is degenerate (|det B_e| ~ 0)");
    }
    static std::atomic<uint64_t> serial{0};
    auto *m = new qxa_mesh_s();
    m->serial = ++serial;
    m->device = device;
    m->dim = dim;
    m->order = order;
    m->np = np;
    m->n_nodes = n_nodes;
    m->n_elem = n_elem;
    m->h_conn.assign(Cn, Cn + size_t(np) * n_elem);
    m->h_coords.assign(X, X + size_t(dim) * n_nodes);
    qxa_status st = upload(&m->d_coords, X, size_t(dim) * n_nodes, m->device_bytes);
    if (!st) st = upload(&m->d_conn, Cn, size_t(np) * n_elem, m->device_bytes);
    if (st) {
        qxa_mesh_destroy(m);
        return st;
    }
    *out = m;
    return QXA_OK;
}

qxa_status qxa_mesh_destroy(qxa_mesh m)
{
    if (!m) return QXA_OK;
    hipSetDevice(m->device);
    hipFree(m->d_coords);
    hipFree(m->d_conn);
    delete m;
    return QXA_OK;
}

qxa_status qxa_plan_destroy(qxa_plan p)
{
    if (!p) return QXA_OK;
    hipSetDevice(p->device);
    void *bufs[] = {p->d_row_ptr, p->d_col_idx, p->d_tconn, p->d_elem_order, p->d_rec, p->d_rec_ptr, p->d_rec_mid,
                    p->d_chain_ptr,
                    p->d_part_ptr, p->d_fix_target, p->d_fix_mirror, p->d_sink, p->d_part, p->d_qfrag[0],
                    p->d_qfrag[1], p->d_qfrag[2], p->d_qfrag[3], p->d_qfrag[4], p->d_tables, p->d_tables_f,
                    p->d_V, p->d_flags, p->d_T, p->d_ns_ptr, p->d_ns_items, p->d_Fe, p->d_nf_ptr, p->d_nf_items, p->d_Tiso};
    for (void *b : bufs) plan_free(p, b);
    delete p;
    return QXA_OK;
}

}  // extern "C"

namespace qxa {

qxa_status plan_stage(qxa_mesh mesh, const qxa_quad &mr, const qxa_quad &cr, PlanStaging &g)
{
    qxa_status st = build_ref_tables(mesh->dim, mesh->order, mr, cr, g.ref);
    if (st) return st;
    const RefTables &T = g.ref;
    if (!form_supported(T.dim, T.order, T.nq_m, T.nq_c))
        return fail(QXA_E_UNSUPPORTED, "no kernel built for dim=" + std::to_string(T.dim) + " order=" +
                                           std::to_string(T.order) + " n_q(mass)=" + std::to_string(T.nq_m) +
                                           " n_q(stiffness)=" + std::to_string(T.nq_c));
    g.mfma = fused_uses_mfma(T.dim, T.order, T.nq_m, T.nq_c);
    if (g.mfma) build_qfrags(T, g.frag, g.f16_qinv);
    if (!split_ok(T.dim, T.order, T.nq_m, T.nq_c))
        for (int f = QXA_F16X2; f <= QXA_BF16X3; ++f) g.frag[f].clear();
    st = build_host_plan(mesh->dim, mesh->order, mesh->n_nodes, mesh->n_elem, mesh->h_conn.data(), g.hp);
    if (st) return st;
    int cus = 256, lds = 160 * 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, mesh->device) != hipSuccess) cus = 256;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, mesh->device) != hipSuccess)
        lds = 160 * 1024;
    (void)hipGetLastError();
    int64_t qv16[5];
    for (int f = 0; f < 5; ++f) qv16[f] = int64_t(g.frag[f].size() / 16);
    const TileParams prm = fused_tile_params(T.dim, T.order, T.nq_m, T.nq_c, cus, size_t(lds), qv16);
    st = build_tile_plan(mesh->dim, mesh->order, mesh->n_nodes, mesh->n_elem, mesh->h_conn.data(),
                         mesh->h_coords.data(), g.hp, prm, g.tp);
    if (!st) st = check_tile_plan(T.np, mesh->n_elem, g.hp, g.tp);
    if (st) return st;
    // reference tables: FP64 block and an FP32 copy
    auto put = [&](const std::vector<double> &v) {
        size_t off = g.tab.size();
        g.tab.insert(g.tab.end(), v.begin(), v.end());
        while (g.tab.size() % 4) g.tab.push_back(0.0);
        return off;
    };
    g.off_wm = put(T.w_m);
    g.off_wc = put(T.w_c);
    g.off_phim = put(T.phi_m);
    g.off_phic = put(T.phi_c);
    g.off_qm = put(T.Qm);
    g.off_qc = put(T.Qc);
    g.off_dphic = put(T.dphi_c);
    g.off_dphim = put(T.dphi_m);
    g.tabf.assign(g.tab.begin(), g.tab.end());
    return QXA_OK;
}

size_t plan_bytes_lower_bound(const PlanStaging &g)
{
    const HostPlan &hp = g.hp;
    const TilePlan &tp = g.tp;
    return sizeof(int64_t) * (hp.row_ptr.size() + tp.rec_ptr.size() + tp.rec_mid.size()) +
           sizeof(int32_t) * (hp.col_idx.size() + tp.tconn.size() + tp.elem_order.size()) +
           sizeof(uint32_t) * tp.rec.size();
}

qxa_status plan_upload(qxa_mesh mesh, const PlanStaging &g, DevArena *arena, bool own_scratch, qxa_plan *out)
{
    *out = nullptr;
    QXA_HIP(hipSetDevice(mesh->device));
    auto *p = new qxa_plan_s();
    p->mesh = mesh;
    p->device = mesh->device;
    p->arena = arena;
    p->ref = g.ref;
    const HostPlan &hp = g.hp;
    const TilePlan &tp = g.tp;
    p->nnz = hp.nnz;
    p->tile_T = tp.T;
    p->n_tiles = tp.n_tiles;
    p->n_shared = tp.n_shared;
    p->n_fix = int64_t(tp.fix_target.size());
    p->n_partials = tp.n_partials;
    p->n_chains = int64_t(tp.chain_ptr.size()) - 1;
    p->carry_cap = tp.carry_cap;
    p->h_chain_ptr = tp.chain_ptr;
    tile_plan_stats(tp, p->stats);
    qxa_status st = plan_upload_buf(p, &p->d_row_ptr, hp.row_ptr.data(), hp.row_ptr.size());
    if (!st) st = plan_upload_buf(p, &p->d_col_idx, hp.col_idx.data(), hp.col_idx.size());
    if (!st) st = plan_upload_buf(p, &p->d_tconn, tp.tconn.data(), tp.tconn.size());
    if (!st) st = plan_upload_buf(p, &p->d_elem_order, tp.elem_order.data(), tp.elem_order.size());
    if (!st) st = plan_upload_buf(p, &p->d_rec, tp.rec.data(), tp.rec.size());
    if (!st) st = plan_upload_buf(p, &p->d_rec_ptr, tp.rec_ptr.data(), tp.rec_ptr.size());
    if (!st) st = plan_upload_buf(p, &p->d_rec_mid, tp.rec_mid.data(), tp.rec_mid.size());
    if (!st) st = plan_upload_buf(p, &p->d_chain_ptr, tp.chain_ptr.data(), tp.chain_ptr.size());
    if (!st) st = plan_upload_buf(p, &p->d_part_ptr, tp.part_ptr.data(), tp.part_ptr.size());
    if (!st) st = plan_upload_buf(p, &p->d_fix_target, tp.fix_target.data(), tp.fix_target.size());
    if (!st) st = plan_upload_buf(p, &p->d_fix_mirror, tp.fix_mirror.data(), tp.fix_mirror.size());
    if (!st) st = plan_alloc(p, &p->d_sink, size_t(kSinkDoubles));
    if (!st && own_scratch) st = plan_alloc(p, &p->d_part, size_t(2) * tp.n_partials);
    if (g.mfma) {
        p->f16_qinv[0] = g.f16_qinv[0];
        p->f16_qinv[1] = g.f16_qinv[1];
        for (int f = 0; f < 5 && !st; ++f) {
            p->qfrag_vec16[f] = int64_t(g.frag[f].size() / 16);
            st = plan_upload_buf(p, reinterpret_cast<uint8_t **>(&p->d_qfrag[f]), g.frag[f].data(), g.frag[f].size());
        }
    }
    p->off_wm = g.off_wm;
    p->off_wc = g.off_wc;
    p->off_phim = g.off_phim;
    p->off_phic = g.off_phic;
    p->off_dphic = g.off_dphic;
    p->off_dphim = g.off_dphim;
    p->off_qm = g.off_qm;
    p->off_qc = g.off_qc;
    if (!st) st = plan_upload_buf(p, &p->d_tables, g.tab.data(), g.tab.size());
    if (!st) st = plan_upload_buf(p, &p->d_tables_f, g.tabf.data(), g.tabf.size());
    if (!st && own_scratch) {
        st = plan_alloc(p, &p->d_flags, 1);
        if (!st) {
            hipError_t e = hipMemset(p->d_flags, 0, sizeof(int));
            if (e != hipSuccess) st = hip_fail(e, "hipMemset");
        }
    }
    if (st) {
        qxa_plan_destroy(p);
        return st;
    }
    *out = p;
    return QXA_OK;
}

}  // namespace qxa

extern "C" {

qxa_status qxa_plan_create(qxa_mesh mesh, const qxa_quad *mr, const qxa_quad *cr, qxa_plan *out)
{
    if (!out) return fail(QXA_E_INVALID, "out is null");
    *out = nullptr;
    if (!mesh || !mr || !cr) return fail(QXA_E_INVALID, "null mesh or rule");
    const auto t0 = std::chrono::steady_clock::now();
    QXA_HIP(hipSetDevice(mesh->device));
    PlanStaging g;
    qxa_status st = plan_stage(mesh, *mr, *cr, g);
    if (!st) st = plan_upload(mesh, g, nullptr, true, out);
    if (st) return st;
    (*out)->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return QXA_OK;
}

qxa_status qxa_plan_get_info(qxa_plan p, qxa_plan_info *out)
{
    if (!p || !out) return fail(QXA_E_INVALID, "null plan or out");
    *out = p->stats;
    out->dim = p->ref.dim;
    out->order = p->ref.order;
    out->n_p = p->ref.np;
    out->n_q_mass = p->ref.nq_m_in;
    out->n_q_stiff = p->ref.nq_c_in;
    out->n_q_mass_kernel = p->ref.nq_m;
    out->n_q_stiff_kernel = p->ref.nq_c;
    out->n_nodes = p->mesh->n_nodes;
    out->n_elem = p->mesh->n_elem;
    out->nnz = p->nnz;
    out->row_ptr = p->d_row_ptr;
    out->col_idx = p->d_col_idx;
    out->device_bytes = p->device_bytes;
    out->build_ms = p->build_ms;
    return QXA_OK;
}

qxa_status qxa_pattern_host(int dim, int order, int64_t n_nodes, int64_t n_elem, const int32_t *conn,
                            int64_t *row_ptr, int32_t *col_idx, int64_t *nnz)
{
    if (!nnz || (n_elem > 0 && !conn)) return fail(QXA_E_INVALID, "null argument");
    if ((dim != 2 && dim != 3) || order < 1 || order > 3 || n_nodes < 1 || n_elem < 0)
        return fail(QXA_E_INVALID, "bad dim/order/sizes");
    const int np = n_local(dim, order);
    for (size_t k = 0; k < size_t(np) * n_elem; ++k)
        if (conn[k] < 0 || conn[k] >= n_nodes) return fail(QXA_E_INDEX, "node index out of range");
    HostPlan hp;
    qxa_status st = build_host_plan(dim, order, n_nodes, n_elem, conn, hp);
    if (st) return st;
    *nnz = hp.nnz;
    if (row_ptr) std::memcpy(row_ptr, hp.row_ptr.data(), sizeof(int64_t) * hp.row_ptr.size());
    if (row_ptr && col_idx) std::memcpy(col_idx, hp.col_idx.data(), sizeof(int32_t) * hp.col_idx.size());
    return QXA_OK;
}

// One deliberate corruption of a built tile plan (tests of the plan check):
// true if the plan has what the mutation needs.
static bool corrupt_tile_plan(int mutation, int np, TilePlan &tp)
{
    const uint32_t T = uint32_t(tp.T), ns = uint32_t(n_sym(np));
    auto is_csr = [](uint32_t c) { return int32_t(c) >= 0 && int32_t(c) < kCodeCarry; };
    for (int64_t t = 0; t < tp.n_tiles; ++t) {
        const int64_t r0 = tp.rec_ptr[t], rm = tp.rec_mid[t];
        if (rm - r0 < 2) continue;
        uint32_t *A = &tp.rec[4 * r0], *B = &tp.rec[4 * (r0 + 1)];
        switch (mutation) {
        case 1:  // a CSR output retargeted to the slot of another output of the tile
            if (!is_csr(A[0]) || !is_csr(B[0])) continue;
            A[0] = B[0];
            return true;
        case 2:  // an entry of an output dropped (marked absent)
            if ((A[1] & 0xffffu) == T) continue;
            A[1] = (A[1] & 0xffff0000u) | T;
            return true;
        case 3:  // an LDS index past the staged pairs
            A[1] = (A[1] & 0xffff0000u) | (ns * (T + 1));
            return true;
        case 4:  // two outputs' entries exchanged
            if ((A[1] & 0xffffu) == (B[1] & 0xffffu)) continue;
            std::swap(A[1], B[1]);
            return true;
        default: break;
        }
    }
    if (mutation == 5 && tp.n_partials > 1) {  // a partial written twice, another never
        for (int64_t r = 0; r + 1 < int64_t(tp.rec.size() / 4); ++r) {
            uint32_t *R = &tp.rec[4 * r];
            const int32_t c = int32_t(R[0]);
            if (c < 0) {
                R[0] = uint32_t(c == -1 ? -2 : -1);
                return true;
            }
        }
    }
    if (mutation == 6 && tp.n_shared > 0) {  // a fix-up mirror slot pointing elsewhere
        tp.fix_mirror[0] = tp.fix_mirror[0] == 0 ? 1 : 0;
        return true;
    }
    return false;
}

static qxa_status plan_check_host_impl(int dim, int order, int64_t n_nodes, const double *coords, int64_t n_elem,
                                       const int32_t *conn, const qxa_quad *mass_rule, const qxa_quad *stiff_rule,
                                       int64_t chains, int carry_cap, int mutation, qxa_plan_info *out)
{
    if (!coords || (n_elem > 0 && !conn)) return fail(QXA_E_INVALID, "null argument");
    if ((dim != 2 && dim != 3) || order < 1 || order > 3 || n_nodes < 1 || n_elem < 0)
        return fail(QXA_E_INVALID, "bad dim/order/sizes");
    const int np = n_local(dim, order);
    for (size_t k = 0; k < size_t(np) * n_elem; ++k)
        if (conn[k] < 0 || conn[k] >= n_nodes) return fail(QXA_E_INDEX, "node index out of range");
    qxa_quad rule{};
    qxa_status st = qxa_quad_builtin(dim, 2 * order, &rule);
    RefTables T;
    if (!st) st = build_ref_tables(dim, order, mass_rule ? *mass_rule : rule, stiff_rule ? *stiff_rule : rule, T);
    if (st) return st;
    std::vector<uint8_t> frag[5];
    double qinv[2];
    if (fused_uses_mfma(dim, order, T.nq_m, T.nq_c)) build_qfrags(T, frag, qinv);
    int64_t qv16[5];
    for (int f = 0; f < 5; ++f) qv16[f] = int64_t(frag[f].size() / 16);
    TileParams prm = fused_tile_params(dim, order, T.nq_m, T.nq_c, 256, size_t(160) * 1024, qv16);
    if (chains > 0) {  // an explicit chain count: runs of consecutive tiles, no run layout
        prm.chains = chains;
        prm.run_len = 0;
    }
    if (carry_cap >= 0) prm.carry_cap = std::min(carry_cap, 65535);
    HostPlan hp;
    st = build_host_plan(dim, order, n_nodes, n_elem, conn, hp);
    if (st) return st;
    TilePlan tp;
    st = build_tile_plan(dim, order, n_nodes, n_elem, conn, coords, hp, prm, tp);
    if (!st && mutation && !corrupt_tile_plan(mutation, np, tp))
        return fail(QXA_E_UNSUPPORTED, "plan check: the plan has nothing this mutation changes");
    if (!st) st = check_tile_plan(np, n_elem, hp, tp);
    if (st) return st;
    if (out) {
        *out = qxa_plan_info{};
        out->dim = dim;
        out->order = order;
        out->n_p = np;
        out->n_q_mass = T.nq_m_in;
        out->n_q_stiff = T.nq_c_in;
        out->n_q_mass_kernel = T.nq_m;
        out->n_q_stiff_kernel = T.nq_c;
        out->n_nodes = n_nodes;
        out->n_elem = n_elem;
        out->nnz = hp.nnz;
        tile_plan_stats(tp, *out);
    }
    return QXA_OK;
}

qxa_status qxa_plan_check_host(int dim, int order, int64_t n_nodes, const double *coords, int64_t n_elem,
                               const int32_t *conn, const qxa_quad *mass_rule, const qxa_quad *stiff_rule,
                               int64_t chains, int carry_cap, qxa_plan_info *out)
{
    return plan_check_host_impl(dim, order, n_nodes, coords, n_elem, conn, mass_rule, stiff_rule, chains, carry_cap, 0,
                                out);
}

qxa_status qxa_plan_check_host_corrupted(int dim, int order, int64_t n_nodes, const double *coords, int64_t n_elem,
                                         const int32_t *conn, int64_t chains, int carry_cap, int mutation)
{
    if (mutation < 1 || mutation > 6) return fail(QXA_E_INVALID, "plan check: mutation is 1..6");
    return plan_check_host_impl(dim, order, n_nodes, coords, n_elem, conn, nullptr, nullptr, chains, carry_cap,
                                mutation, nullptr);
}

qxa_status qxa_quad_builtin(int dim, int degree, qxa_quad *out)
{
    if (!out) return fail(QXA_E_INVALID, "null output");
    if (dim != 2 && dim != 3) return fail(QXA_E_INVALID, "dim must be 2 or 3");
    const BuiltinRule *best = nullptr;
    for (int k = 0; k < k_n_builtin_rules; ++k) {
        const BuiltinRule &r = k_builtin_rules[k];
        if (r.dim == dim && r.degree >= degree && (!best || r.degree < best->degree)) best = &r;
    }
    if (!best) return fail(QXA_E_UNSUPPORTED, "no built-in rule of that degree (at most 6)");
    *out = qxa_quad{dim, best->n_q, best->points, best->weights};
    return QXA_OK;
}

qxa_status qxa_plan_copy_pattern(qxa_plan p, int64_t *row_ptr, int32_t *col_idx, void *stream)
{
    if (!p) return fail(QXA_E_INVALID, "null plan");
    QXA_HIP(hipSetDevice(p->mesh->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (row_ptr)
        QXA_HIP(hipMemcpyAsync(row_ptr, p->d_row_ptr, sizeof(int64_t) * (p->mesh->n_nodes + 1),
                               hipMemcpyDeviceToDevice, s));
    if (col_idx && p->nnz)
        QXA_HIP(hipMemcpyAsync(col_idx, p->d_col_idx, sizeof(int32_t) * p->nnz, hipMemcpyDeviceToDevice, s));
    return QXA_OK;
}

static qxa_status fill_inputs(qxa_plan p, const qxa_coeff *mass, const qxa_coeff *stiff, int precision,
                              FormInputs &in, const void **Qm, const void **Qc)
{
    if (precision < QXA_FP64 || precision > QXA_BF16X3) return fail(QXA_E_INVALID, "unknown precision form");
    if (precision > QXA_FP32 && !split_ok(p->ref.dim, p->ref.order, p->ref.nq_m, p->ref.nq_c))
        return fail(QXA_E_UNSUPPORTED,
                    "split 16-bit forms run on the matrix cores with Q staged on chip (2D P2/P3 and 3D P2, with "
                    "rules whose tables fit there); use QXA_FP32 as the reduced-precision form here");
    const int64_t nn = p->mesh->n_nodes, ne = p->mesh->n_elem;
    qxa_status st = to_coeff(mass, in.cm, "mass", nn, ne, p->ref.nq_m_in);
    if (!st) st = to_coeff(stiff, in.cc, "stiffness", nn, ne, p->ref.nq_c_in);
    if (!st) st = to_tensor(mass, stiff, p->ref.dim, in.aniso, in.K);
    if (st) return st;
    const qxa_mesh m = p->mesh;
    in.n_nodes = m->n_nodes;
    in.n_elem = m->n_elem;
    in.coords = m->d_coords;
    in.w_m = p->d_tables + p->off_wm;
    in.w_c = p->d_tables + p->off_wc;
    in.phi_m = p->d_tables + p->off_phim;
    in.phi_c = p->d_tables + p->off_phic;
    in.flags = p->d_flags;
    if (precision == QXA_FP32) {
        *Qm = p->d_tables_f + p->off_qm;
        *Qc = p->d_tables_f + p->off_qc;
    } else {
        *Qm = p->d_tables + p->off_qm;
        *Qc = p->d_tables + p->off_qc;
    }
    return QXA_OK;
}

}  // extern "C"

namespace qxa {

qxa_status make_fused_args(qxa_plan p, const qxa_coeff *mass, const qxa_coeff *stiff, int precision, double *M,
                           double *C, double *part, int *flags, FusedArgs &a, FixupArgs &f)
{
    a = FusedArgs{};
    qxa_status st = fill_inputs(p, mass, stiff, precision, a.in, &a.Qm, &a.Qc);
    if (st) return st;
    a.in.flags = flags;
    a.tconn = p->d_tconn;
    a.elem_order = p->d_elem_order;
    a.rec = p->d_rec;
    a.rec_ptr = p->d_rec_ptr;
    a.rec_mid = p->d_rec_mid;
    a.carry_cap = p->carry_cap;
    a.sink = p->d_sink;
    a.M = M;
    a.C = C;
    a.Qfrag = p->d_qfrag[precision];
    a.qfrag_vec16 = p->qfrag_vec16[precision];
    a.qinv_m = precision == QXA_F16X2 ? p->f16_qinv[0] : 1.0;
    a.qinv_c = precision == QXA_F16X2 ? p->f16_qinv[1] : 1.0;
    a.part = part;
    // buffer stores address 31-bit byte offsets; larger arrays (or QXA_FLAT_STORES
    // set, which tests use to cover that path on small meshes) take plain stores
    const int64_t lim = (int64_t(1) << 31) - 16;
    a.buf_ok = 8 * p->nnz <= lim && 16 * p->n_partials <= lim && !std::getenv("QXA_FLAT_STORES");
    a.bytes_vals = a.buf_ok ? uint32_t(8 * p->nnz) : 0u;
    a.bytes_part = a.buf_ok ? uint32_t(16 * p->n_partials) : 0u;
    f = FixupArgs{p->n_fix, p->d_fix_target, p->d_fix_mirror, p->d_part_ptr, part, M, C};
    return QXA_OK;
}

}  // namespace qxa

extern "C" {

qxa_status qxa_assemble(qxa_plan p, const qxa_coeff *mass, const qxa_coeff *stiff, int precision, double *M_vals,
                        double *C_vals, void *stream)
{
    if (!p) return fail(QXA_E_INVALID, "null plan");
    if (!p->d_flags) return fail(QXA_E_INVALID, "plan is owned by a server");
    FusedArgs a;
    FixupArgs f;
    qxa_status st = make_fused_args(p, mass, stiff, precision, M_vals, C_vals, p->d_part, p->d_flags, a, f);
    if (st) return st;
    if (!M_vals && !C_vals) return QXA_OK;
    QXA_HIP(hipSetDevice(p->mesh->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // launch errors are read back with hipGetLastError: drop one left behind by
    // an unrelated earlier call on this thread so it is not blamed on the launch
    const hipError_t stale = hipGetLastError();
    if (stale != hipSuccess && std::getenv("QXA_DEBUG"))
        std::fprintf(stderr, "qxa: cleared an earlier HIP error before launching: %s\n", hipGetErrorString(stale));
    {
        TimedLaunch tl(p, "fused", s);
        const JobTable jt{a, nullptr, nullptr, 0, p->n_tiles, a.buf_ok, p->d_chain_ptr, p->n_chains};
        QXA_HIP(launch_fused(jt, p->ref.dim, p->ref.order, p->ref.nq_m, p->ref.nq_c, precision, s));
    }
    TimedLaunch tl(p, "fixup", s);
    const FixupTable ft{f, nullptr, nullptr, 0, p->n_fix};
    QXA_HIP(launch_fixup(ft, s));
    return QXA_OK;
}

qxa_status qxa_element_matrices(qxa_plan p, const qxa_coeff *mass, const qxa_coeff *stiff, int precision, double *Vm,
                                double *Vc, void *stream)
{
    if (!p) return fail(QXA_E_INVALID, "null plan");
    if (precision != QXA_FP64 && precision != QXA_FP32)
        return fail(QXA_E_UNSUPPORTED, "the formation-only entry point computes in FP64 or FP32");
    FormArgs a{};
    qxa_status st = fill_inputs(p, mass, stiff, precision, a.in, &a.Qm, &a.Qc);
    if (st) return st;
    if (!Vm && !Vc) return QXA_OK;
    QXA_HIP(hipSetDevice(p->mesh->device));
    const size_t ns = size_t(p->ref.ns), ne = size_t(p->mesh->n_elem);
    if (!p->d_V && ne) {
        st = plan_alloc(p, &p->d_V, 2 * ns * ne);
        if (st) return st;
    }
    a.conn = p->mesh->d_conn;
    a.Vm = Vm ? p->d_V : nullptr;
    a.Vc = Vc ? p->d_V + ns * ne : nullptr;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    QXA_HIP(launch_form(a, p->ref.dim, p->ref.order, p->ref.nq_m, p->ref.nq_c, precision, s));
    ExpandArgs x{p->mesh->n_elem, p->ref.np, a.Vm, a.Vc, Vm, Vc};
    QXA_HIP(launch_expand(x, s));
    return QXA_OK;
}

qxa_status qxa_element_matrices_noalloc(qxa_plan p, const qxa_coeff *mass, const qxa_coeff *stiff, int precision,
                                        double *Vm, double *Vc, void *stream)
{
    if (!p) return fail(QXA_E_INVALID, "null plan");
    if (precision != QXA_FP64 && precision != QXA_FP32)
        return fail(QXA_E_UNSUPPORTED, "the formation-only entry point computes in FP64 or FP32");
    FormArgs a{};
    qxa_status st = fill_inputs(p, mass, stiff, precision, a.in, &a.Qm, &a.Qc);
    if (st) return st;
    if (!Vm && !Vc) return QXA_OK;
    const size_t ns = size_t(p->ref.ns), ne = size_t(p->mesh->n_elem);
    if (2 * ns * ne > kScratchDoubles)
        return fail(QXA_E_UNSUPPORTED, "allocation-free formation: 2 * n_sym * n_elem = " + std::to_string(2 * ns * ne) +
                                           " doubles exceeds the scratch of " + std::to_string(kScratchDoubles) +
                                           " (64 MiB); use qxa_element_matrices");
    if (ne == 0) return QXA_OK;
    if (!p->d_flags) return fail(QXA_E_INVALID, "plan is owned by a server");
    double *sc = scratch_of(p->mesh->device);
    if (!sc) return fail(QXA_E_INVALID, "scratch address of the plan's device was not resolved");
    QXA_HIP(hipSetDevice(p->mesh->device));
    a.conn = p->mesh->d_conn;
    a.Vm = Vm ? sc : nullptr;
    a.Vc = Vc ? sc + ns * ne : nullptr;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    QXA_HIP(launch_form(a, p->ref.dim, p->ref.order, p->ref.nq_m, p->ref.nq_c, precision, s));
    ExpandArgs x{p->mesh->n_elem, p->ref.np, a.Vm, a.Vc, Vm, Vc};
    QXA_HIP(launch_expand(x, s));
    return QXA_OK;
}

qxa_status qxa_coeff_product(qxa_plan p, int rule, const qxa_coeff *c, const double *v, double *S, void *stream)
{
    if (!p || !c) return fail(QXA_E_INVALID, "null argument");
    // arrays of zero length may be null
    if ((!v && p->mesh->n_nodes) || (!S && p->mesh->n_elem)) return fail(QXA_E_INVALID, "null argument");
    if (rule != 0 && rule != 1) return fail(QXA_E_INVALID, "rule: 0 (mass rule) or 1 (stiffness rule)");
    if (!p->d_flags) return fail(QXA_E_INVALID, "plan is owned by a server");
    if (c->kind != QXA_COEFF_NODAL) return fail(QXA_E_INVALID, "the first factor is a nodal field through a law");
    if (c->tensor) return fail(QXA_E_INVALID, "the first factor has no tensor");
    CoeffProductArgs a{};
    qxa_status st = to_coeff(c, a.c, "first factor", p->mesh->n_nodes, p->mesh->n_elem, 0);
    if (st) return st;
    if (p->mesh->n_elem == 0) return QXA_OK;
    QXA_HIP(hipSetDevice(p->mesh->device));
    a.n_elem = p->mesh->n_elem;
    a.conn = p->mesh->d_conn;
    a.phi = p->d_tables + (rule == 0 ? p->off_phim : p->off_phic);
    a.v = v;
    a.S = S;
    a.flags = p->d_flags;
    const int nq = rule == 0 ? p->ref.nq_m : p->ref.nq_c;
    a.nq_out = rule == 0 ? p->ref.nq_m_in : p->ref.nq_c_in;
    QXA_HIP(launch_coeff_product(a, p->ref.dim, p->ref.order, nq, reinterpret_cast<hipStream_t>(stream)));
    return QXA_OK;
}

}  // extern "C"

namespace qxa {

// Entries of every CSR slot (both triangles) for the nonsymmetric local matrices
// T[(e * np + a) * np + b] (element-major): the slot of (N_e(a), N_e(b)) is the upper slot of the
// pair or its mirror. Counting sort in element order, so each slot lists its
// entries by ascending element, then (a, b): a fixed summation order.
static qxa_status build_slot_entries(qxa_plan p)
{
    const qxa_mesh m = p->mesh;
    const int np = p->ref.np;
    const int64_t ne = m->n_elem;
    if (int64_t(np) * np * ne >= (int64_t(1) << 31))
        return fail(QXA_E_UNSUPPORTED, "conductivity tensor product: more than 2^31 element entries");
    HostPlan hp;
    qxa_status st = build_host_plan(m->dim, m->order, m->n_nodes, ne, m->h_conn.data(), hp);
    if (st) return st;
    const int32_t *conn = m->h_conn.data();
    auto slot = [&](int64_t e, int a, int b) -> uint32_t {
        const int lo = std::min(a, b), hi = std::max(a, b);
        const int s = lo * np - lo * (lo - 1) / 2 + (hi - lo);
        const uint32_t up = hp.perm_sym[size_t(s) * ne + e];
        return conn[size_t(a) * ne + e] <= conn[size_t(b) * ne + e] ? up : hp.mirror[up];
    };
    std::vector<int64_t> ptr(hp.nnz + 1, 0);
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) ++ptr[slot(e, a, b) + 1];
    for (int64_t t = 0; t < hp.nnz; ++t) ptr[t + 1] += ptr[t];
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    std::vector<int32_t> items(static_cast<size_t>(ptr[hp.nnz]));
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) items[size_t(fill[slot(e, a, b)]++)] = int32_t((e * np + a) * np + b);
    // offsets below 2^31 (checked above): 4 bytes per slot for the gather to read
    const std::vector<int32_t> ptr32(ptr.begin(), ptr.end());
    st = plan_upload_buf(p, &p->d_ns_ptr, ptr32.data(), ptr32.size());
    if (!st) st = plan_upload_buf(p, &p->d_ns_items, items.data(), items.size());
    if (st) plan_drop(p, &p->d_ns_ptr, &p->d_ns_items);
    return st;
}


// Element entries of every node (a * n_elem + e with N_e(a) = node), ascending element.
static qxa_status build_node_entries(qxa_plan p)
{
    const qxa_mesh m = p->mesh;
    const int np = p->ref.np;
    const int64_t ne = m->n_elem, nn = m->n_nodes;
    if (int64_t(np) * ne >= (int64_t(1) << 31)) return fail(QXA_E_UNSUPPORTED, "load vector: more than 2^31 entries");
    const int32_t *conn = m->h_conn.data();
    std::vector<int64_t> ptr(nn + 1, 0);
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < np; ++a) ++ptr[conn[size_t(a) * ne + e] + 1];
    for (int64_t i = 0; i < nn; ++i) ptr[i + 1] += ptr[i];
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    std::vector<int32_t> items(static_cast<size_t>(ptr[nn]));
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < np; ++a) items[size_t(fill[conn[size_t(a) * ne + e]]++)] = int32_t(a * ne + e);
    const std::vector<int32_t> ptr32(ptr.begin(), ptr.end());  // below 2^31 (checked above)
    qxa_status st = plan_upload_buf(p, &p->d_nf_ptr, ptr32.data(), ptr32.size());
    if (!st) st = plan_upload_buf(p, &p->d_nf_items, items.data(), items.size());
    if (!st) st = plan_alloc(p, &p->d_Fe, size_t(np) * ne);
    if (st) plan_drop(p, &p->d_nf_ptr, &p->d_nf_items, &p->d_Fe);
    return st;
}

}  // namespace qxa

extern "C" {

qxa_status qxa_assemble_iso(qxa_plan p, const qxa_coeff *mass, const qxa_coeff *stiff, double *M_vals, double *C_vals,
                            void *stream)
{
    if (!p) return fail(QXA_E_INVALID, "null plan");
    if (!p->d_flags) return fail(QXA_E_INVALID, "plan is owned by a server");
    IsoArgs a{};
    if (mass && mass->tensor_q) return fail(QXA_E_INVALID, "mass coefficient: a tensor applies to conductivity only");
    if (stiff && stiff->tensor_q && stiff->tensor)
        return fail(QXA_E_INVALID, "conductivity: give either a constant tensor or one per quadrature node");
    qxa_coeff sc{};
    if (stiff) {
        sc = *stiff;
        sc.tensor_q = nullptr;  // validated with the rest; passed to the kernel below
    }
    const void *qm, *qc;
    qxa_status st = fill_inputs(p, mass, stiff ? &sc : nullptr, QXA_FP64, a.in, &qm, &qc);
    if (st) return st;
    a.Kq = stiff ? stiff->tensor_q : nullptr;
    a.nq_kq = p->ref.nq_c_in;
    // the reduction: the plan's units, chains and fix-up, as the fused assembly
    FusedArgs fa;
    FixupArgs fx;
    st = make_fused_args(p, mass, stiff ? &sc : nullptr, QXA_FP64, M_vals, C_vals, p->d_part, p->d_flags, fa, fx);
    if (st) return st;
    const qxa_mesh m = p->mesh;
    if ((!M_vals && !C_vals) || m->n_elem == 0) return QXA_OK;
    QXA_HIP(hipSetDevice(m->device));
    const RefTables &R = p->ref;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // one pass where the shape's matrix-core kernel takes it: one rule for both
    // matrices, and the reference gradients fit in LDS beside the plan's carries
    const bool one_rule = R.nq_m == R.nq_c && R.nq_m_in == R.nq_c_in && R.w_m == R.w_c && R.phi_m == R.phi_c &&
                          R.dphi_m == R.dphi_c;
    if (one_rule && fused_iso_fits(m->dim, m->order, R.nq_m, R.nq_c, fa.qfrag_vec16, fa.carry_cap)) {
        fa.dphi = p->d_tables + p->off_dphim;
        fa.Kq = a.Kq;
        fa.nq_kq = a.nq_kq;
        {
            TimedLaunch tl(p, "fused_iso", s);
            const JobTable jt{fa, nullptr, nullptr, 0, p->n_tiles, fa.buf_ok, p->d_chain_ptr, p->n_chains};
            QXA_HIP(launch_fused_iso(jt, m->dim, m->order, R.nq_m, R.nq_c, s));
        }
        TimedLaunch tl(p, "fixup", s);
        const FixupTable ft{fx, nullptr, nullptr, 0, p->n_fix};
        QXA_HIP(launch_fixup(ft, s));
        return QXA_OK;
    }
    // else two passes; the local-matrix kernel stages positions, fields and X of 64 elements in LDS
    const size_t iso_lds = size_t(kIsoElems) * (R.np * R.dim + 2 * R.np + R.nq_m + R.nq_c * R.ng) * sizeof(double);
    if (iso_lds > kLdsBytes)
        return fail(QXA_E_UNSUPPORTED, "isoparametric assembly: rules of " + std::to_string(R.nq_m) + " and " +
                                           std::to_string(R.nq_c) + " nodes need " + std::to_string(iso_lds) +
                                           " bytes of LDS per workgroup (more than 160 KiB)");
    // symmetric local matrices once per pair, pair-major per block of kIsoElems tile positions
    const int64_t ne_pad = (m->n_elem + kIsoElems - 1) / kIsoElems * kIsoElems;
    if (int64_t(p->ref.ns) * ne_pad >= (int64_t(1) << 31))
        return fail(QXA_E_UNSUPPORTED, "isoparametric assembly: more than 2^31 element entries");
    const size_t nt = size_t(p->ref.ns) * size_t(ne_pad);
    if (!p->d_Tiso) {
        st = plan_alloc(p, &p->d_Tiso, 2 * nt);
        if (st) return st;
    }
    a.tconn = p->d_tconn;
    a.elem_order = p->d_elem_order;
    a.Qm = static_cast<const double *>(qm);
    a.Qc = static_cast<const double *>(qc);
    a.dphi_m = p->d_tables + p->off_dphim;
    a.dphi_c = p->d_tables + p->off_dphic;
    a.Tm = M_vals ? p->d_Tiso : nullptr;
    a.Tc = C_vals ? p->d_Tiso + nt : nullptr;
    {
        TimedLaunch tl(p, "iso_rows", s);
        QXA_HIP(launch_iso(a, m->dim, m->order, p->ref.nq_m, p->ref.nq_c, s));
    }
    {
        TimedLaunch tl(p, "staged_reduce", s);
        const JobTable jt{fa, nullptr, nullptr, 0, p->n_tiles, fa.buf_ok, p->d_chain_ptr, p->n_chains};
        QXA_HIP(launch_staged_reduce(jt, m->dim, m->order, a.Tm, a.Tc, s));
    }
    TimedLaunch tl(p, "fixup", s);
    const FixupTable ft{fx, nullptr, nullptr, 0, p->n_fix};
    QXA_HIP(launch_fixup(ft, s));
    return QXA_OK;
}

qxa_status qxa_load_vector(qxa_plan p, const qxa_coeff *f, double *F, void *stream)
{
    if (!p || !f || (!F && p->mesh->n_nodes)) return fail(QXA_E_INVALID, "null argument");
    if (!p->d_flags) return fail(QXA_E_INVALID, "plan is owned by a server");
    LoadArgs a{};
    const void *qm, *qc;
    qxa_status st = fill_inputs(p, f, nullptr, QXA_FP64, a.in, &qm, &qc);
    if (st) return st;
    const qxa_mesh m = p->mesh;
    QXA_HIP(hipSetDevice(m->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (m->n_elem == 0) {
        if (m->n_nodes) QXA_HIP(hipMemsetAsync(F, 0, sizeof(double) * m->n_nodes, s));
        return QXA_OK;
    }
    if (!p->d_nf_ptr) {
        st = build_node_entries(p);
        if (st) return st;
    }
    a.conn = m->d_conn;
    a.Fe = p->d_Fe;
    {
        TimedLaunch tl(p, "load_elem", s);
        QXA_HIP(launch_load(a, m->dim, m->order, p->ref.nq_m, s));
    }
    TimedLaunch tl(p, "slot_gather", s);
    const SlotGatherArgs g{m->n_nodes, p->d_nf_ptr, p->d_nf_items, p->d_Fe, F};
    QXA_HIP(launch_slot_gather(g, s));
    return QXA_OK;
}

qxa_status qxa_cond_tensor_product(qxa_plan p, const qxa_coeff *c, const double *v, double *T_vals, void *stream)
{
    if (!p || !c) return fail(QXA_E_INVALID, "null argument");
    if ((!v && p->mesh->n_nodes) || (!T_vals && p->nnz)) return fail(QXA_E_INVALID, "null argument");
    if (!p->d_flags) return fail(QXA_E_INVALID, "plan is owned by a server");
    if (c->kind != QXA_COEFF_NODAL) return fail(QXA_E_INVALID, "c' is a nodal field through a law");
    CondTensorArgs a{};
    qxa_status st = to_coeff(c, a.c, "c'", p->mesh->n_nodes, p->mesh->n_elem, 0);
    if (!st) st = to_tensor(nullptr, c, p->ref.dim, a.aniso, a.K);
    if (st) return st;
    if (p->mesh->n_elem == 0) return QXA_OK;
    QXA_HIP(hipSetDevice(p->mesh->device));
    if (!p->d_ns_ptr) {
        st = build_slot_entries(p);
        if (st) return st;
    }
    if (!p->d_T) {
        st = plan_alloc(p, &p->d_T, size_t(p->ref.np) * p->ref.np * p->mesh->n_elem);
        if (st) return st;
    }
    const qxa_mesh m = p->mesh;
    a.n_nodes = m->n_nodes;
    a.n_elem = m->n_elem;
    a.coords = m->d_coords;
    a.conn = m->d_conn;
    a.w = p->d_tables + p->off_wc;
    a.phi = p->d_tables + p->off_phic;
    a.dphi = p->d_tables + p->off_dphic;
    a.v = v;
    a.T = p->d_T;
    a.flags = p->d_flags;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    {
        TimedLaunch tl(p, "cond_tensor_rows", s);
        QXA_HIP(launch_cond_tensor(a, m->dim, m->order, p->ref.nq_c, s));
    }
    TimedLaunch tl(p, "slot_gather", s);
    const SlotGatherArgs g{p->nnz, p->d_ns_ptr, p->d_ns_items, p->d_T, T_vals};
    QXA_HIP(launch_slot_gather(g, s));
    return QXA_OK;
}

qxa_status qxa_plan_set_timing(qxa_plan p, int enable)
{
    if (!p) return fail(QXA_E_INVALID, "null plan");
    p->timing = enable != 0;
    return QXA_OK;
}

qxa_status qxa_plan_timing_report(qxa_plan p, char *buf, size_t cap)
{
    if (!p || !buf || cap == 0) return fail(QXA_E_INVALID, "null plan or buffer");
    QXA_HIP(hipSetDevice(p->mesh->device));
    std::vector<std::pair<std::string, std::pair<int, double>>> acc;
    qxa_status st = QXA_OK;
    for (auto &r : p->recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && st == QXA_OK) st = hip_fail(e, "hipEventElapsedTime");
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
        size_t k = 0;
        while (k < acc.size() && acc[k].first != r.name) ++k;
        if (k == acc.size()) acc.push_back({r.name, {0, 0.0}});
        acc[k].second.first += 1;
        acc[k].second.second += ms;
    }
    p->recs.clear();
    std::string out = "{";
    for (size_t k = 0; k < acc.size(); ++k) {
        char tmp[160];
        std::snprintf(tmp, sizeof(tmp), "%s\"%s\": {\"n\": %d, \"ms\": %.6f}", k ? ", " : "", acc[k].first.c_str(),
                      acc[k].second.first, acc[k].second.second);
        out += tmp;
    }
    out += "}";
    std::snprintf(buf, cap, "%s", out.c_str());
    return st;
}

}  // extern "C"

struct qxa_graph_s {
    qxa_plan plan = nullptr;
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

qxa_status qxa_graph_create(qxa_plan p, const qxa_coeff *mass, const qxa_coeff *stiff, int precision, double *M_vals,
                            double *C_vals, qxa_graph *out)
{
    if (!out) return fail(QXA_E_INVALID, "out is null");
    *out = nullptr;
    if (!p) return fail(QXA_E_INVALID, "null plan");
    QXA_HIP(hipSetDevice(p->mesh->device));
    hipStream_t s = nullptr;
    QXA_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    const bool timing = p->timing;
    p->timing = false;  // no event nodes inside the graph
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    qxa_status st = e == hipSuccess ? QXA_OK : hip_fail(e, "hipStreamBeginCapture");
    hipGraph_t g = nullptr;
    if (!st) {
        st = qxa_assemble(p, mass, stiff, precision, M_vals, C_vals, s);
        const std::string msg = st ? std::string(qxa_last_error()) : std::string();
        e = hipStreamEndCapture(s, &g);
        if (!st && e != hipSuccess) st = hip_fail(e, "hipStreamEndCapture");
        if (st && !msg.empty()) fail(st, msg);
    }
    p->timing = timing;
    hipStreamDestroy(s);
    if (st) {
        if (g) hipGraphDestroy(g);
        return st;
    }
    auto *gr = new qxa_graph_s();
    gr->plan = p;
    gr->device = p->device;
    gr->graph = g;
    e = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        delete gr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = gr;
    return QXA_OK;
}

qxa_status qxa_graph_launch(qxa_graph g, void *stream)
{
    if (!g) return fail(QXA_E_INVALID, "null graph");
    QXA_HIP(hipSetDevice(g->device));
    QXA_HIP(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)));
    return QXA_OK;
}

qxa_status qxa_graph_destroy(qxa_graph g)
{
    if (!g) return QXA_OK;
    hipSetDevice(g->device);
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
    return QXA_OK;
}

qxa_status qxa_sync(qxa_plan p, void *stream)
{
    if (!p) return fail(QXA_E_INVALID, "null plan");
    QXA_HIP(hipSetDevice(p->mesh->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    QXA_HIP(hipStreamSynchronize(s));
    int flag = 0;
    QXA_HIP(hipMemcpy(&flag, p->d_flags, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        QXA_HIP(hipMemset(p->d_flags, 0, sizeof(int)));
        return fail(QXA_E_NONFINITE, "non-finite coefficient value at a quadrature node");
    }
    return QXA_OK;
}

}  // extern "C"
