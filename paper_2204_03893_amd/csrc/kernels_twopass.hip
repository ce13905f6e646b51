// Kernels that write local values to HBM and then gather them:
//  - formation (Algorithm 2 up to the element matrices) of the symmetric V_m, V_c for
//    the formation-only entry point, and their expansion to full n_p x n_p matrices;
//  - the per-node coefficient of the mass tensor contracted with a vector and the local
//    matrices of the conductivity tensor contracted with a vector (Section 5);
//  - element load vectors (Section 2);
//  - isoparametric local matrices with a per-node geometry and tensor (Section 7);
//  - the deterministic gathers into CSR slots, nodes, or upper slots and their mirrors.
#include "kernels_twopass.hpp"
#include "kernels_common.hpp"

// This file is built twice: on its own (the rule sizes of QXA_FORM_CASES_TUNED,
// the rule-size choice, the gathers and the dispatch) and through
// kernels_twopass_padded.hip (those of QXA_FORM_CASES_PADDED), so that the two
// sets of kernels compile in parallel.
#ifdef QXA_TWOPASS_PADDED
#define QXA_TWOPASS_CASES QXA_FORM_CASES_PADDED
#define QXA_PART(name) name##_padded
#else
#define QXA_TWOPASS_CASES QXA_FORM_CASES_TUNED
#define QXA_PART(name) name##_tuned
#endif

namespace qxa {

template <int D, int P, int NQM, int NQC, typename CT>
__global__ __launch_bounds__(256) void form_kernel(FormArgs a)
{
    using S = Shape<D, P>;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.in.n_elem) return;
    int32_t v[S::NP];
#pragma unroll
    for (int i = 0; i < S::NP; ++i) v[i] = a.conn[i * a.in.n_elem + e];
    double A[S::NG], lm[NQM], lc[NQC];
    if (!element_setup<D, P, NQM, NQC>(a.in, v, e, A, lm, lc)) atomicOr(a.in.flags, 1);
    const int64_t ne = a.in.n_elem;
    if (a.Vm)
        contract_mass<S::NS, NQM>(reinterpret_cast<const CT *>(a.Qm), lm,
                                  [&](int s, double x) { a.Vm[s * ne + e] = x; });
    if (a.Vc)
        contract_stiff<P, S::NS, NQC, S::NG>(reinterpret_cast<const CT *>(a.Qc), lc, A,
                                             [&](int s, double x) { a.Vc[s * ne + e] = x; });
}
#ifndef QXA_TWOPASS_PADDED

// Symmetric pairs -> full n_p x n_p element matrices [(i*np+j)][n_elem].
__global__ __launch_bounds__(256) void expand_kernel(ExpandArgs a)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.n_elem) return;
    int s = 0;
    for (int i = 0; i < a.np; ++i)
        for (int j = i; j < a.np; ++j, ++s) {
            if (a.Vm) {
                const double x = a.Sm[int64_t(s) * a.n_elem + e];
                a.Vm[int64_t(i * a.np + j) * a.n_elem + e] = x;
                a.Vm[int64_t(j * a.np + i) * a.n_elem + e] = x;
            }
            if (a.Vc) {
                const double x = a.Sc[int64_t(s) * a.n_elem + e];
                a.Vc[int64_t(i * a.np + j) * a.n_elem + e] = x;
                a.Vc[int64_t(j * a.np + i) * a.n_elem + e] = x;
            }
        }
}
#endif
#ifndef QXA_TWOPASS_PADDED

bool compiled_rule_sizes(int D, int P, int nqm, int nqc, int &cm, int &cc)
{
    const int ng = D * (D + 1) / 2;
    int best = -1;
#define X(d, p, m, c)                                                           \
    if (D == d && P == p && nqm <= m && nqc <= c && (best < 0 || m + ng * c < best)) { \
        best = m + ng * c;                                                      \
        cm = m;                                                                 \
        cc = c;                                                                 \
    }
    QXA_FORM_CASES(X)
#undef X
    return best >= 0;
}
#endif
#ifndef QXA_TWOPASS_PADDED

bool form_supported(int D, int P, int nqm, int nqc)
{
#define X(d, p, m, c) \
    if (D == d && P == p && nqm == m && nqc == c) return true;
    QXA_FORM_CASES(X)
#undef X
    return false;
}
#endif

hipError_t QXA_PART(launch_form)(const FormArgs &a, int D, int P, int nqm, int nqc, int precision, hipStream_t st, bool &found)
{
    found = true;
    if (a.in.n_elem == 0) return hipSuccess;
    const dim3 block(256), grid(unsigned((a.in.n_elem + 255) / 256));
#define X(d, p, m, c)                                                                 \
    if (D == d && P == p && nqm == m && nqc == c) {                                   \
        if (precision == 1) form_kernel<d, p, m, c, float><<<grid, block, 0, st>>>(a); \
        else form_kernel<d, p, m, c, double><<<grid, block, 0, st>>>(a);               \
        return hipGetLastError();                                                     \
    }
    QXA_TWOPASS_CASES(X)
#undef X
    found = false;
    return hipErrorInvalidValue;
}

// Coefficient of the mass tensor contracted with v (Section 5): at every
// quadrature node of the rule, s = law(u_h(xhat_q)) * v_h(xhat_q) with u_h and
// v_h interpolated from the element's nodal values (one thread per element,
// S[q][e] stored q-major so that a warp's stores are contiguous).
template <int D, int P, int NQ>
__global__ __launch_bounds__(256) void coeff_product_kernel(CoeffProductArgs a)
{
    using S = Shape<D, P>;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.n_elem) return;
    double u[S::NP], v[S::NP];
#pragma unroll
    for (int i = 0; i < S::NP; ++i) {
        const int32_t node = a.conn[i * a.n_elem + e];
        u[i] = a.c.field[node];
        v[i] = a.v[node];
    }
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double uh = 0.0, vh = 0.0;
#pragma unroll
        for (int i = 0; i < S::NP; ++i) {
            const double ph = uniform_table(a.phi)[i * NQ + q];
            uh = fma(ph, u[i], uh);
            vh = fma(ph, v[i], vh);
        }
        const double s = apply_law(a.c, uh) * vh;
        if (q < a.nq_out) {  // (the caller's rule; the compiled one may be padded)
            ok &= isfinite(s);
            a.S[q * a.n_elem + e] = s;
        }
    }
    if (!ok) atomicOr(a.flags, 1);
}

hipError_t QXA_PART(launch_coeff_product)(const CoeffProductArgs &a, int D, int P, int nq, hipStream_t st, bool &found)
{
    found = true;
    if (a.n_elem == 0) return hipSuccess;
    const dim3 block(256), grid(unsigned((a.n_elem + 255) / 256));
#define X(d, p, m, c)                                                            \
    if (D == d && P == p && nq == m) {                                          \
        coeff_product_kernel<d, p, m><<<grid, block, 0, st>>>(a);                \
        return hipGetLastError();                                                \
    }                                                                            \
    if (D == d && P == p && nq == c) {                                          \
        coeff_product_kernel<d, p, c><<<grid, block, 0, st>>>(a);                \
        return hipGetLastError();                                                \
    }
    QXA_TWOPASS_CASES(X)
#undef X
    found = false;
    return hipErrorInvalidValue;
}

// Local matrices of the conductivity tensor contracted with v in its second mode
// (Section 5): T_e[a][b] = sum_q w_q c'(u_h) |det B_e| (J_q[a] A_e J_q^T v_e) phi_b(xhat_q),
// i.e. the columns of Q = [phi_q (x) J_q] weighted by X[(q, c), e] = lambda_q (A_e J_q^T v_e)_c.
// A block takes 64 elements, one per lane, through LDS: the nodal values of u and v (one
// wave per local node) and the geometry; X (one wave per quadrature node, the reference
// tables as wave-uniform scalars); then, per chunk of kCtRows rows, row a of every element
// (one wave per row: r_a(q) = J_q[a] . X[q, :], then T[a][b] = sum_q phi_b(q) r_a(q)) into
// an LDS stage that the block copies out as contiguous row segments of the element-major
// output [n_elem][n_p][n_p].
constexpr int kCtElems = 64, kCtRows = 8;

template <int D, int P, int NQ>
constexpr size_t ct_lds_doubles()
{
    using S = Shape<D, P>;
    return size_t(kCtElems) * (2 * S::NP + S::NG + 1 + NQ * D) + size_t(kCtElems) * (kCtRows * S::NP + 1);
}

template <int D, int P, int NQ>
__global__ __launch_bounds__(512) void cond_tensor_rows_kernel(CondTensorArgs a)
{
    using S = Shape<D, P>;
    constexpr int NP = S::NP, NG = S::NG, E = kCtElems, STR = kCtRows * NP + 1;
    extern __shared__ double ct_lds[];
    double *sU = ct_lds;          // [NP][E] u at the element's nodes
    double *sV = sU + NP * E;     // [NP][E] v at the element's nodes
    double *sA = sV + NP * E;     // [NG][E] A_e
    double *sB = sA + NG * E;     // [E] |det B_e|
    double *sX = sB + E;          // [NQ * D][E] X
    double *sT = sX + NQ * D * E; // [E][STR] rows of the current chunk
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int nw = int(blockDim.x >> 6);
    const int64_t ne = a.n_elem, e0 = int64_t(blockIdx.x) * E, e = e0 + lane;
    const bool live = e < ne;
    for (int i = wave; i < NP; i += nw) {
        const int32_t node = live ? a.conn[i * ne + e] : 0;
        sU[i * E + lane] = live ? a.c.field[node] : 0.0;
        sV[i * E + lane] = live ? a.v[node] : 0.0;
    }
    if (wave == 0) {
        double x[D + 1][D];
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            const int32_t node = live ? a.conn[k * ne + e] : 0;
#pragma unroll
            for (int c = 0; c < D; ++c) x[k][c] = live ? a.coords[c * a.n_nodes + node] : (c + 1 == k ? 1.0 : 0.0);
        }
        double babs, Au[NG];
        geometry_from<D>(x, babs, Au, a.aniso, a.K);
#pragma unroll
        for (int g = 0; g < NG; ++g) sA[g * E + lane] = Au[g];
        sB[lane] = babs;
    }
    __syncthreads();
    bool ok = true;
    for (int q = wave; q < NQ; q += nw) {
        const auto J = uniform_table(a.dphi + size_t(q) * NP * D);
        const auto phi = uniform_table(a.phi);
        double uh = 0.0, gv[D];
#pragma unroll
        for (int c = 0; c < D; ++c) gv[c] = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const double vi = sV[i * E + lane] - sV[lane];  // v_i - v_0 (the gradients sum to zero)
            uh = fma(phi[i * NQ + q], sU[i * E + lane], uh);
#pragma unroll
            for (int c = 0; c < D; ++c) gv[c] = fma(J[i * D + c], vi, gv[c]);  // J_q^T v_e
        }
        const double lam = uniform_table(a.w)[q] * apply_law(a.c, uh) * sB[lane];
        if (live) ok &= isfinite(lam);
        double A[D][D];
        {
            int g = 0;
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
                for (int c = r; c < D; ++c, ++g) A[r][c] = A[c][r] = sA[g * E + lane];
        }
#pragma unroll
        for (int c = 0; c < D; ++c) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) t = fma(A[c][k], gv[k], t);
            sX[(q * D + c) * E + lane] = lam * t;
        }
    }
    if (!ok) atomicOr(a.flags, 1);
    __syncthreads();
    for (int a0 = 0; a0 < NP; a0 += kCtRows) {
        const int rows = min(kCtRows, NP - a0);
        for (int ar = wave; ar < rows; ar += nw) {
            const int ra = a0 + ar;
            double r[NQ];  // r_a(q) = J_q[a] . X[q, :]
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const auto J = uniform_table(a.dphi + size_t(q) * NP * D);
                double t = 0.0;
#pragma unroll
                for (int c = 0; c < D; ++c) t = fma(J[ra * D + c], sX[(q * D + c) * E + lane], t);
                r[q] = t;
            }
#pragma unroll 1
            for (int b = 0; b < NP; ++b) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) t = fma(uniform_table(a.phi)[b * NQ + q], r[q], t);
                sT[lane * STR + ar * NP + b] = t;
            }
        }
        __syncthreads();
        const int seg = rows * NP;  // element el's rows a0 .. a0 + rows - 1: contiguous in T
        for (int idx = threadIdx.x; idx < E * seg; idx += blockDim.x) {
            const int el = idx / seg, off = idx - el * seg;
            if (e0 + el < ne) a.T[(e0 + el) * (NP * NP) + a0 * NP + off] = sT[el * STR + off];
        }
        __syncthreads();
    }
}

hipError_t QXA_PART(launch_cond_tensor)(const CondTensorArgs &a, int D, int P, int nq, hipStream_t st, bool &found)
{
    found = true;
    if (a.n_elem == 0) return hipSuccess;
    const unsigned blocks = unsigned((a.n_elem + kCtElems - 1) / kCtElems);
#define X(d, p, m, c)                                                                                   \
    if (D == d && P == p && nq == c) {                                                                  \
        cond_tensor_rows_kernel<d, p, c><<<blocks, 512, ct_lds_doubles<d, p, c>() * sizeof(double), st>>>(a); \
        return hipGetLastError();                                                                       \
    }
    QXA_TWOPASS_CASES(X)
#undef X
    found = false;
    return hipErrorInvalidValue;
}

// Element load vectors (Section 2, f_i = int f phi_i; the vector analogue of
// Algorithm 2, V = Phi Lambda): Fe[a][e] = sum_q phi_a(xhat_q) w_q f_q |det B_e|, one
// thread per element.
template <int D, int P, int NQ>
__global__ __launch_bounds__(256) void load_elem_kernel(LoadArgs a)
{
    using S = Shape<D, P>;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t ne = a.in.n_elem;
    if (e >= ne) return;
    double x[D + 1][D];
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        const int32_t node = a.conn[k * ne + e];
#pragma unroll
        for (int c = 0; c < D; ++c) x[k][c] = a.in.coords[c * a.in.n_nodes + node];
    }
    double babs, A[S::NG];
    geometry_from<D>(x, babs, A);
    const CoeffDev &f = a.in.cm;
    double u[S::NP];
    if (f.kind == 1) {
#pragma unroll
        for (int i = 0; i < S::NP; ++i) u[i] = f.field[a.conn[i * ne + e]];
    }
    double fe[S::NP];
#pragma unroll
    for (int i = 0; i < S::NP; ++i) fe[i] = 0.0;
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s;
        if (f.kind == 0) {
            s = f.value;
        } else if (f.kind == 1) {
            double uh = 0.0;
#pragma unroll
            for (int i = 0; i < S::NP; ++i) uh = fma(uniform_table(a.in.phi_m)[i * NQ + q], u[i], uh);
            s = apply_law(f, uh);
        } else {
            s = apply_law(f, qe_value(f, q, ne, e));
        }
        const double lam = uniform_table(a.in.w_m)[q] * s * babs;
        ok &= isfinite(lam);
#pragma unroll
        for (int i = 0; i < S::NP; ++i) fe[i] = fma(uniform_table(a.in.phi_m)[i * NQ + q], lam, fe[i]);
    }
#pragma unroll
    for (int i = 0; i < S::NP; ++i) a.Fe[i * ne + e] = fe[i];
    if (!ok) atomicOr(a.in.flags, 1);
}

hipError_t QXA_PART(launch_load)(const LoadArgs &a, int D, int P, int nq, hipStream_t st, bool &found)
{
    found = true;
    if (a.in.n_elem == 0) return hipSuccess;
    const unsigned grid = unsigned((a.in.n_elem + 255) / 256);
#define X(d, p, m, c)                                                  \
    if (D == d && P == p && nq == m) {                                 \
        load_elem_kernel<d, p, m><<<grid, 256, 0, st>>>(a);            \
        return hipGetLastError();                                      \
    }
    QXA_TWOPASS_CASES(X)
#undef X
    found = false;
    return hipErrorInvalidValue;
}

// Isoparametric elements (curved geometry, Section 7): M_e and C_e with B, |det B| and
// A = B^{-1} K B^{-T} evaluated per quadrature node from every node's position, so X
// holds one column per (q, e): X_m[q] = w_q m_q |det B_q| and X_c[(q, g)] = w_q c_q
// |det B_q| A_q[g]; the contraction V = Q X with the plan's Q_m and Q_c (symmetric pair
// rows) is unchanged. A block of 8 waves takes 64 tile positions (the plan's element
// order), one element per lane, in three phases through LDS: the elements' node positions and nodal
// fields (one wave per local node), X (one wave per quadrature node: B_q, |det B_q|, the
// coefficient, A_q), then V (one wave per pair a <= b, Q read as wave-uniform scalars),
// stored once per pair in a pair-major layout [block][pair][64] so that the lanes of a
// wave write 512 contiguous bytes; the fused kernels' reduction then reads them per tile.

template <int D, int P, int NQM, int NQC>
constexpr size_t iso_lds_doubles()
{
    using S = Shape<D, P>;
    return size_t(kIsoElems) * (S::NP * D + 2 * S::NP + NQM + NQC * S::NG);
}

template <int D, int P, int NQM, int NQC>
__global__ __launch_bounds__(512) void iso_rows_kernel(IsoArgs a)
{
    using S = Shape<D, P>;
    constexpr int NP = S::NP, NG = S::NG, NS = S::NS, E = kIsoElems;
    extern __shared__ double iso_lds[];
    double *sCrd = iso_lds;              // [NP * D][E] node positions
    double *sUm = sCrd + NP * D * E;     // [NP][E] nodal field of the mass coefficient
    double *sUc = sUm + NP * E;          // [NP][E] nodal field of the conductivity coefficient
    double *sXm = sUc + NP * E;          // [NQM][E]
    double *sXc = sXm + NQM * E;         // [NQC * NG][E]
    const FormInputs &in = a.in;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int nw = int(blockDim.x >> 6);
    // lane: tile position p (the output order the fused reduction reads), element e
    const int64_t ne = in.n_elem, p = int64_t(blockIdx.x) * E + lane;
    const bool live = p < ne;
    const int64_t e = live ? int64_t(a.elem_order[p]) : 0;
    for (int i = wave; i < NP; i += nw) {
        const int32_t node = live ? a.tconn[i * ne + p] : 0;
#pragma unroll
        for (int r = 0; r < D; ++r) sCrd[(i * D + r) * E + lane] = live ? in.coords[r * in.n_nodes + node] : 0.0;
        sUm[i * E + lane] = live && in.cm.kind == 1 ? in.cm.field[node] : 0.0;
        sUc[i * E + lane] = live && in.cc.kind == 1 ? in.cc.field[node] : 0.0;
    }
    __syncthreads();
    bool ok = true;
    for (int qq = wave; qq < NQM + NQC; qq += nw) {
        const bool mass = qq < NQM;
        const int q = mass ? qq : qq - NQM;
        if (mass ? !a.Tm : !a.Tc) continue;  // never read
        const auto J = uniform_table((mass ? a.dphi_m : a.dphi_c) + size_t(q) * NP * D);
        double B[D][D];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) B[r][c] = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int r = 0; r < D; ++r) {
                // x_i - x_0: the gradients sum to zero, so this is B_q exactly, without the
                // cancellation of absolute coordinates on small elements
                const double xr = sCrd[(i * D + r) * E + lane] - sCrd[r * E + lane];
#pragma unroll
                for (int c = 0; c < D; ++c) B[r][c] = fma(xr, J[i * D + c], B[r][c]);
            }
        double I[D][D], adet;
        inverse_abs_det<D>(B, I, adet);
        const CoeffDev &cf = mass ? in.cm : in.cc;
        double sv = cf.value;
        if (cf.kind == 1) {
            const auto phi = uniform_table(mass ? in.phi_m : in.phi_c);
            const double *u = mass ? sUm : sUc;
            double uh = 0.0;  // u_h(xhat_q) = phi_q^T u_e
#pragma unroll
            for (int i = 0; i < NP; ++i) uh = fma(phi[i * (mass ? NQM : NQC) + q], u[i * E + lane], uh);
            sv = apply_law(cf, uh);
        } else if (cf.kind == 2) {
            sv = live ? apply_law(cf, qe_value(cf, q, ne, e)) : 0.0;
        }
        const double lam = uniform_table(mass ? in.w_m : in.w_c)[q] * sv * adet;
        if (mass) {
            if (live) {
                ok &= isfinite(lam) && adet > 0.0;
                sXm[q * E + lane] = lam;
            }
        } else {
            double Au[NG];
            if (a.Kq) {  // K_qe: a tensor per quadrature node
                double Kl[NG];
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    Kl[g] = live ? a.Kq[(int64_t(q < a.nq_kq ? q : 0) * NG + g) * ne + e] : 0.0;
                    ok &= isfinite(Kl[g]);
                }
                metric_from_inverse<D>(I, 1, Kl, Au);
            } else {
                metric_from_inverse<D>(I, in.aniso, in.K, Au);
            }
            if (live) {
                ok &= isfinite(lam) && adet > 0.0;
#pragma unroll
                for (int g = 0; g < NG; ++g) sXc[(q * NG + g) * E + lane] = lam * Au[g];
            }
        }
    }
    if (!ok) atomicOr(in.flags, 1);
    __syncthreads();
    if (!live) return;
    // PB pairs per pass: each X value read from LDS serves PB rows of Q
    constexpr int PB = 4;
    for (int sp0 = wave * PB; sp0 < NS; sp0 += nw * PB) {
        int spj[PB];
#pragma unroll
        for (int j = 0; j < PB; ++j) spj[j] = min(sp0 + j, NS - 1);
        if (a.Tm) {
            double v[PB];
#pragma unroll
            for (int j = 0; j < PB; ++j) v[j] = 0.0;
#pragma unroll
            for (int q = 0; q < NQM; ++q) {
                const double x = sXm[q * E + lane];
#pragma unroll
                for (int j = 0; j < PB; ++j) v[j] = fma(uniform_table(a.Qm)[spj[j] * NQM + q], x, v[j]);
            }
#pragma unroll
            for (int j = 0; j < PB; ++j)
                if (sp0 + j < NS) a.Tm[(size_t(blockIdx.x) * NS + sp0 + j) * E + lane] = v[j];
        }
        if (a.Tc) {
            double v[PB];
#pragma unroll
            for (int j = 0; j < PB; ++j) v[j] = 0.0;
#pragma unroll 6
            for (int k = 0; k < NQC * NG; ++k) {
                const double x = sXc[k * E + lane];
#pragma unroll
                for (int j = 0; j < PB; ++j) v[j] = fma(uniform_table(a.Qc)[spj[j] * (NQC * NG) + k], x, v[j]);
            }
#pragma unroll
            for (int j = 0; j < PB; ++j)
                if (sp0 + j < NS) a.Tc[(size_t(blockIdx.x) * NS + sp0 + j) * E + lane] = v[j];
        }
    }
}

hipError_t QXA_PART(launch_iso)(const IsoArgs &a, int D, int P, int nqm, int nqc, hipStream_t st, bool &found)
{
    found = true;
    if (a.in.n_elem == 0) return hipSuccess;
    const unsigned blocks = unsigned((a.in.n_elem + kIsoElems - 1) / kIsoElems);
#define X(d, p, m, c)                                                                                  \
    if (D == d && P == p && nqm == m && nqc == c) {                                                    \
        iso_rows_kernel<d, p, m, c><<<blocks, 512, iso_lds_doubles<d, p, m, c>() * sizeof(double), st>>>(a); \
        return hipGetLastError();                                                                      \
    }
    QXA_TWOPASS_CASES(X)
#undef X
    found = false;
    return hipErrorInvalidValue;
}
#ifndef QXA_TWOPASS_PADDED

// out[t] = sum of src over the entries of slot t, in their stored order (deterministic).
__global__ __launch_bounds__(256) void slot_gather_kernel(SlotGatherArgs a)
{
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (t >= a.n_slots) return;
    const int64_t lo = a.ptr[t], hi = a.ptr[t + 1];
    double s = 0.0;
    // four entries per step: their index and value loads are issued before the adds, which
    // then run in the stored order (the same sum as one entry at a time)
    for (int64_t k = lo; k < hi; k += 4) {
        int32_t i[4];
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) i[j] = a.items[min(k + j, hi - 1)];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = a.src[i[j]];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (k + j < hi) s += v[j];
    }
    a.out[t] = s;
}


hipError_t launch_slot_gather(const SlotGatherArgs &a, hipStream_t st)
{
    if (a.n_slots == 0) return hipSuccess;
    slot_gather_kernel<<<unsigned((a.n_slots + 255) / 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_expand(const ExpandArgs &a, hipStream_t st)
{
    if (a.n_elem == 0) return hipSuccess;
    expand_kernel<<<unsigned((a.n_elem + 255) / 256), 256, 0, st>>>(a);
    return hipGetLastError();
}


hipError_t launch_form_padded(const FormArgs &a, int D, int P, int nqm, int nqc, int precision, hipStream_t st, bool &found);
hipError_t launch_form(const FormArgs &a, int D, int P, int nqm, int nqc, int precision, hipStream_t st)
{
    bool found = false;
    const hipError_t e = launch_form_tuned(a, D, P, nqm, nqc, precision, st, found);
    return found ? e : launch_form_padded(a, D, P, nqm, nqc, precision, st, found);
}
hipError_t launch_coeff_product_padded(const CoeffProductArgs &a, int D, int P, int nq, hipStream_t st, bool &found);
hipError_t launch_coeff_product(const CoeffProductArgs &a, int D, int P, int nq, hipStream_t st)
{
    bool found = false;
    const hipError_t e = launch_coeff_product_tuned(a, D, P, nq, st, found);
    return found ? e : launch_coeff_product_padded(a, D, P, nq, st, found);
}
hipError_t launch_cond_tensor_padded(const CondTensorArgs &a, int D, int P, int nq, hipStream_t st, bool &found);
hipError_t launch_cond_tensor(const CondTensorArgs &a, int D, int P, int nq, hipStream_t st)
{
    bool found = false;
    const hipError_t e = launch_cond_tensor_tuned(a, D, P, nq, st, found);
    return found ? e : launch_cond_tensor_padded(a, D, P, nq, st, found);
}
hipError_t launch_load_padded(const LoadArgs &a, int D, int P, int nq, hipStream_t st, bool &found);
hipError_t launch_load(const LoadArgs &a, int D, int P, int nq, hipStream_t st)
{
    bool found = false;
    const hipError_t e = launch_load_tuned(a, D, P, nq, st, found);
    return found ? e : launch_load_padded(a, D, P, nq, st, found);
}
hipError_t launch_iso_padded(const IsoArgs &a, int D, int P, int nqm, int nqc, hipStream_t st, bool &found);
hipError_t launch_iso(const IsoArgs &a, int D, int P, int nqm, int nqc, hipStream_t st)
{
    bool found = false;
    const hipError_t e = launch_iso_tuned(a, D, P, nqm, nqc, st, found);
    return found ? e : launch_iso_padded(a, D, P, nqm, nqc, st, found);
}
#endif

}  // namespace qxa
