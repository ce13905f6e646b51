// Reference-element tables of Algorithm 2 (Section 4):
//   Phi = [phi_1 .. phi_nq]  (basis values at the quadrature nodes),
//   J_q  (reference basis gradients at node q),
//   Q_m = Phi (.) Phi        (Khatri-Rao product, n_p^2 x n_q),
//   Q_c = [J_1 (x) J_1, ..., J_nq (x) J_nq]  (n_p^2 x d^2 n_q).
// Only the rows of distinct symmetric pairs (a <= b) are kept: V is the
// vectorisation of a symmetric matrix, so the other rows are duplicates
// (Section 7, first improvement). Q_c is further contracted against the
// symmetric W = vec(A_e): columns (q, a, b) and (q, b, a) are merged into one
// column per a <= b, so X_c = Lambda_c (.) W keeps d(d+1)/2 rows per q.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "qxa_internal.hpp"

namespace qxa {

// Barycentric multi-indices of the local nodes (mesh format of qxa.h).
static int local_alpha(int dim, int P, int alpha[kMaxNp][4])
{
    static const int e2[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    static const int e3[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
    std::memset(alpha, 0, sizeof(int) * kMaxNp * 4);
    int n = 0;
    for (int k = 0; k <= dim; ++k) alpha[n++][k] = P;
    const int ne = dim == 2 ? 3 : 6;
    for (int s = 0; s < ne; ++s) {
        const int a = dim == 2 ? e2[s][0] : e3[s][0];
        const int b = dim == 2 ? e2[s][1] : e3[s][1];
        for (int t = 1; t < P; ++t, ++n) {
            alpha[n][a] = P - t;
            alpha[n][b] = t;
        }
    }
    if (P == 3) {
        if (dim == 2) {
            alpha[n][0] = alpha[n][1] = alpha[n][2] = 1;
            ++n;
        } else {
            const int opp[4] = {3, 0, 1, 2};
            for (int f = 0; f < 4; ++f, ++n)
                for (int k = 0; k < 4; ++k) alpha[n][k] = (k == opp[f]) ? 0 : 1;
        }
    }
    return n;
}

// phi_i(l) = prod_k prod_{j < alpha_ik} (P l_k - j) / (j + 1), with l the
// barycentric coordinates (l_0 = 1 - sum xhat, l_k = xhat_k). The reference
// gradient is d/dxhat_m = d/dl_m - d/dl_0.
void lagrange_eval(int dim, int order, const double *xhat, double *phi, double *dphi)
{
    int alpha[kMaxNp][4];
    const int np = local_alpha(dim, order, alpha);
    double l[4];
    l[0] = 1.0;
    for (int k = 0; k < dim; ++k) {
        l[k + 1] = xhat[k];
        l[0] -= xhat[k];
    }
    for (int i = 0; i < np; ++i) {
        double f[4], df[4];  // per barycentric factor group: value, derivative w.r.t. l_k
        for (int k = 0; k <= dim; ++k) {
            double v = 1.0, dv = 0.0;
            for (int j = 0; j < alpha[i][k]; ++j) {
                const double g = (order * l[k] - j) / (j + 1);
                const double dg = double(order) / (j + 1);
                dv = dv * g + v * dg;
                v *= g;
            }
            f[k] = v;
            df[k] = dv;
        }
        double val = 1.0;
        for (int k = 0; k <= dim; ++k) val *= f[k];
        phi[i] = val;
        double dl[4];
        for (int k = 0; k <= dim; ++k) {
            double p = df[k];
            for (int m = 0; m <= dim; ++m)
                if (m != k) p *= f[m];
            dl[k] = p;
        }
        for (int m = 0; m < dim; ++m) dphi[i * dim + m] = dl[m + 1] - dl[0];
    }
}

static qxa_status check_rule(const qxa_quad &r, int dim, const char *which)
{
    if (r.dim != dim) return fail(QXA_E_INVALID, std::string(which) + " rule dimension does not match the mesh");
    if (r.n_q < 1 || r.n_q > kMaxNq || !r.points || !r.weights)
        return fail(QXA_E_INVALID, std::string(which) + " rule: need 1 <= n_q <= 64 and non-null points/weights");
    double s = 0.0;
    for (int q = 0; q < r.n_q; ++q) {
        if (!std::isfinite(r.weights[q])) return fail(QXA_E_NONFINITE, std::string(which) + " rule weight");
        s += r.weights[q];
        for (int k = 0; k < dim; ++k)
            if (!std::isfinite(r.points[q * dim + k])) return fail(QXA_E_NONFINITE, std::string(which) + " rule point");
    }
    const double vol = dim == 2 ? 0.5 : 1.0 / 6.0;
    if (std::fabs(s - vol) > 1e-12)
        return fail(QXA_E_INVALID, std::string(which) + " rule weights must sum to the reference volume 1/dim!");
    return QXA_OK;
}

qxa_status build_ref_tables(int dim, int order, const qxa_quad &mr, const qxa_quad &cr, RefTables &T)
{
    qxa_status st = check_rule(mr, dim, "mass");
    if (st) return st;
    st = check_rule(cr, dim, "stiffness");
    if (st) return st;
    T.dim = dim;
    T.order = order;
    T.np = n_local(dim, order);
    T.ns = n_sym(T.np);
    T.ng = n_geo(dim);
    T.nq_m_in = mr.n_q;
    T.nq_c_in = cr.n_q;
    if (!compiled_rule_sizes(dim, order, mr.n_q, cr.n_q, T.nq_m, T.nq_c))
        return fail(QXA_E_UNSUPPORTED, "no kernel takes rules of " + std::to_string(mr.n_q) + " (mass) and " +
                                           std::to_string(cr.n_q) + " (stiffness) nodes for dim=" +
                                           std::to_string(dim) + " order=" + std::to_string(order) + " (at most " +
                                           std::to_string(dim == 2 ? kMaxRule2D : kMaxRule3D) + " nodes)");
    // rules padded to the compiled sizes: zero-weight copies of node 0
    std::vector<double> pm(size_t(T.nq_m) * dim), pc(size_t(T.nq_c) * dim);
    for (int q = 0; q < T.nq_m; ++q)
        std::copy(mr.points + (q < mr.n_q ? q : 0) * dim, mr.points + (q < mr.n_q ? q : 0) * dim + dim,
                  pm.begin() + size_t(q) * dim);
    for (int q = 0; q < T.nq_c; ++q)
        std::copy(cr.points + (q < cr.n_q ? q : 0) * dim, cr.points + (q < cr.n_q ? q : 0) * dim + dim,
                  pc.begin() + size_t(q) * dim);
    const double *mpts = pm.data(), *cpts = pc.data();
    const int np = T.np, ns = T.ns, ng = T.ng;
    T.w_m.assign(mr.weights, mr.weights + mr.n_q);
    T.w_c.assign(cr.weights, cr.weights + cr.n_q);
    T.w_m.resize(T.nq_m, 0.0);
    T.w_c.resize(T.nq_c, 0.0);
    T.pair_a.clear();
    T.pair_b.clear();
    for (int a = 0; a < np; ++a)
        for (int b = a; b < np; ++b) {
            T.pair_a.push_back(a);
            T.pair_b.push_back(b);
        }
    // geometric component g -> (c1, c2), c1 <= c2, row-major upper triangle
    int gc1[6], gc2[6];
    {
        int g = 0;
        for (int c1 = 0; c1 < dim; ++c1)
            for (int c2 = c1; c2 < dim; ++c2, ++g) {
                gc1[g] = c1;
                gc2[g] = c2;
            }
    }
    double phi[kMaxNp], dphi[kMaxNp * 3];
    // mass rule: Phi and Q_m
    T.phi_m.assign(size_t(np) * T.nq_m, 0.0);
    T.dphi_m.assign(size_t(T.nq_m) * np * dim, 0.0);
    T.Qm.assign(size_t(ns) * T.nq_m, 0.0);
    for (int q = 0; q < T.nq_m; ++q) {
        lagrange_eval(dim, order, mpts + q * dim, phi, dphi);
        for (int i = 0; i < np; ++i) T.phi_m[size_t(i) * T.nq_m + q] = phi[i];
        std::copy(dphi, dphi + np * dim, T.dphi_m.begin() + size_t(q) * np * dim);
        for (int s = 0; s < ns; ++s) T.Qm[size_t(s) * T.nq_m + q] = phi[T.pair_a[s]] * phi[T.pair_b[s]];
    }
    // stiffness rule: Phi (for u_h) and Q_c
    T.phi_c.assign(size_t(np) * T.nq_c, 0.0);
    T.dphi_c.assign(size_t(T.nq_c) * np * dim, 0.0);
    T.Qc.assign(size_t(ns) * T.nq_c * ng, 0.0);
    std::vector<double> J0;
    T.stiff_const_grad = true;
    for (int q = 0; q < T.nq_c; ++q) {
        lagrange_eval(dim, order, cpts + q * dim, phi, dphi);
        for (int i = 0; i < np; ++i) T.phi_c[size_t(i) * T.nq_c + q] = phi[i];
        std::copy(dphi, dphi + np * dim, T.dphi_c.begin() + size_t(q) * np * dim);
        if (q == 0) J0.assign(dphi, dphi + np * dim);
        else
            for (int k = 0; k < np * dim; ++k)
                if (dphi[k] != J0[k]) T.stiff_const_grad = false;
        for (int s = 0; s < ns; ++s) {
            const int a = T.pair_a[s], b = T.pair_b[s];
            for (int g = 0; g < ng; ++g) {
                const int c1 = gc1[g], c2 = gc2[g];
                double v = dphi[a * dim + c1] * dphi[b * dim + c2];
                if (c1 != c2) v += dphi[a * dim + c2] * dphi[b * dim + c1];
                T.Qc[(size_t(s) * T.nq_c + q) * ng + g] = v;
            }
        }
    }
    return QXA_OK;
}

}  // namespace qxa
