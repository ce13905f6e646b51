// Formation kernel (Algorithm 2, Lines 4-11) writing the symmetric element
// matrices V_m, V_c to a buffer, and the deterministic segmented gather that
// forms the CSR values from it (Line 12). One lane per element in formation;
// one lane per CSR slot in the gather, summing its segment in the plan's
// fixed (element, pair) order, so results are bitwise reproducible.
#include "kernels.hpp"
#include "kernels_common.hpp"

namespace qxa {

template <int D, int P, int NQM, int NQC, typename CT>
__global__ __launch_bounds__(256) void form_kernel(FormArgs a)
{
    constexpr int NP = (D == 2) ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6;
    constexpr int NS = NP * (NP + 1) / 2;
    constexpr int NG = D * (D + 1) / 2;
    constexpr bool FLAT = NQC * NG <= 96;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.n_elem) return;

    int32_t v[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) v[i] = a.conn[i * a.n_elem + e];

    double babs, A[NG];
    element_geometry<D>(a.coords, a.n_nodes, v, babs, A);

    // coefficient values at the quadrature nodes (S_m, S_c, Line 5) and the
    // weighted columns Lambda = S * (w b^T) (Lines 6-7)
    double um[NP];
    const bool need_u = a.cm.kind == 1 || a.cc.kind == 1;
    if (need_u) {
        const double *f = a.cm.kind == 1 ? a.cm.field : a.cc.field;
#pragma unroll
        for (int i = 0; i < NP; ++i) um[i] = f[v[i]];
    }
    bool bad = false;
    double lm[NQM];
#pragma unroll
    for (int q = 0; q < NQM; ++q) {
        double s;
        if (a.cm.kind == 0) {
            s = a.cm.value;
        } else if (a.cm.kind == 1) {
            double uh = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) uh = fma(a.phi_m[i * NQM + q], um[i], uh);
            s = apply_law(a.cm, uh);
        } else {
            s = apply_law(a.cm, a.cm.field[q * a.n_elem + e]);
        }
        lm[q] = a.w_m[q] * s * babs;
        bad |= !isfinite(lm[q]);
    }
    double uc[NP];
    if (a.cc.kind == 1) {
        if (a.cm.kind == 1 && a.cc.field == a.cm.field) {
#pragma unroll
            for (int i = 0; i < NP; ++i) uc[i] = um[i];
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) uc[i] = a.cc.field[v[i]];
        }
    }
    double lc[NQC];
#pragma unroll
    for (int q = 0; q < NQC; ++q) {
        double s;
        if (a.cc.kind == 0) {
            s = a.cc.value;
        } else if (a.cc.kind == 1) {
            double uh = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) uh = fma(a.phi_c[i * NQC + q], uc[i], uh);
            s = apply_law(a.cc, uh);
        } else {
            s = apply_law(a.cc, a.cc.field[q * a.n_elem + e]);
        }
        lc[q] = a.w_c[q] * s * babs;
        bad |= !isfinite(lc[q]);
    }
    if (bad) atomicOr(a.flags, 1);

    const CT *__restrict__ Qm = reinterpret_cast<const CT *>(a.Qm);
    const CT *__restrict__ Qc = reinterpret_cast<const CT *>(a.Qc);
    // V_m = Q_m X_m with X_m = Lambda_m (Lines 8, 10)
    if (a.Vm) {
        CT x[NQM];
#pragma unroll
        for (int q = 0; q < NQM; ++q) x[q] = CT(lm[q]);
#pragma unroll 1
        for (int s = 0; s < NS; ++s) {
            CT acc = CT(0);
#pragma unroll
            for (int q = 0; q < NQM; ++q) acc = fma(Qm[s * NQM + q], x[q], acc);
            a.Vm[s * a.n_elem + e] = double(acc);
        }
    }
    // V_c = Q_c X_c with X_c = Lambda_c (.) W (Lines 9, 11)
    if (a.Vc) {
        if constexpr (P == 1) {
            // constant reference gradients: the n_q column blocks of Q_c coincide,
            // so Q_c X_c = Q_c^(1) (sum_q lambda_q) vec(A_e)
            double ls = 0.0;
#pragma unroll
            for (int q = 0; q < NQC; ++q) ls += lc[q];
            CT x[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) x[g] = CT(ls * A[g]);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                CT acc = CT(0);
#pragma unroll
                for (int g = 0; g < NG; ++g) acc = fma(Qc[s * NQC * NG + g], x[g], acc);
                a.Vc[s * a.n_elem + e] = double(acc);
            }
        } else if constexpr (FLAT) {
            CT x[NQC * NG];
#pragma unroll
            for (int q = 0; q < NQC; ++q)
#pragma unroll
                for (int g = 0; g < NG; ++g) x[q * NG + g] = CT(lc[q] * A[g]);
#pragma unroll 1
            for (int s = 0; s < NS; ++s) {
                CT acc = CT(0);
#pragma unroll
                for (int k = 0; k < NQC * NG; ++k) acc = fma(Qc[s * NQC * NG + k], x[k], acc);
                a.Vc[s * a.n_elem + e] = double(acc);
            }
        } else {
            // same product with X_c = Lambda_c (.) W applied column block by block
            CT l[NQC], w[NG];
#pragma unroll
            for (int q = 0; q < NQC; ++q) l[q] = CT(lc[q]);
#pragma unroll
            for (int g = 0; g < NG; ++g) w[g] = CT(A[g]);
#pragma unroll 1
            for (int s = 0; s < NS; ++s) {
                CT acc = CT(0);
#pragma unroll
                for (int q = 0; q < NQC; ++q) {
                    CT t = CT(0);
#pragma unroll
                    for (int g = 0; g < NG; ++g) t = fma(Qc[(s * NQC + q) * NG + g], w[g], t);
                    acc = fma(t, l[q], acc);
                }
                a.Vc[s * a.n_elem + e] = double(acc);
            }
        }
    }
}

// Deterministic segmented reduction: slot t sums the contributions listed in
// the segment of its upper-triangle twin, in the plan's order.
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= a.nnz) return;
    const uint32_t u = a.src_upper[t];
    const uint32_t lo = a.seg_ptr[u], hi = a.seg_ptr[u + 1];
    double m = 0.0, c = 0.0;
    for (uint32_t k = lo; k < hi; ++k) {
        const uint32_t idx = a.seg_val[k];
        if (a.M) m += a.Vm[idx];
        if (a.C) c += a.Vc[idx];
    }
    if (a.M) a.M[t] = m;
    if (a.C) a.C[t] = c;
}

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

// ---------------------------------------------------------------- dispatch
#define QXA_FORM_CASES(X)                                                                                     \
    X(2, 1, 3, 3) X(2, 2, 6, 6) X(2, 3, 12, 12) X(3, 1, 4, 4) X(3, 2, 11, 11) X(3, 3, 24, 24) X(2, 1, 3, 1)   \
        X(2, 2, 6, 3) X(2, 3, 12, 6) X(3, 1, 4, 1) X(3, 2, 11, 4) X(3, 3, 24, 11)

bool form_supported(int D, int P, int nqm, int nqc)
{
#define X(d, p, m, c) \
    if (D == d && P == p && nqm == m && nqc == c) return true;
    QXA_FORM_CASES(X)
#undef X
    return false;
}

hipError_t launch_form(const FormArgs &a, int D, int P, int nqm, int nqc, int precision, hipStream_t st)
{
    const dim3 block(256), grid(unsigned((a.n_elem + 255) / 256));
    if (a.n_elem == 0) return hipSuccess;
#define X(d, p, m, c)                                                                         \
    if (D == d && P == p && nqm == m && nqc == c) {                                           \
        if (precision == 1) form_kernel<d, p, m, c, float><<<grid, block, 0, st>>>(a);         \
        else form_kernel<d, p, m, c, double><<<grid, block, 0, st>>>(a);                       \
        return hipGetLastError();                                                             \
    }
    QXA_FORM_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_gather(const GatherArgs &a, hipStream_t st)
{
    if (a.nnz == 0) return hipSuccess;
    gather_kernel<<<unsigned((a.nnz + 255) / 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_expand(const ExpandArgs &a, hipStream_t st)
{
    if (a.n_elem == 0) return hipSuccess;
    expand_kernel<<<unsigned((a.n_elem + 255) / 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace qxa
