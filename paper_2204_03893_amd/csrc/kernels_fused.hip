// Fused assembly kernel: Algorithm 2, Lines 4-12 in one pass over the mesh.
//
// One workgroup per tile of T consecutive elements (plan order), one lane per
// element. Each lane computes its element's geometry and weighted coefficient
// columns (Lines 4-7), then for each matrix in turn forms the element
// matrix V = Q X (Lines 8-11, symmetric-pair rows only) into LDS, and the
// workgroup reduces every CSR slot the tile touches over the tile's
// contributions in the plan's fixed order (Line 12). Slots owned by the tile
// are written directly (upper entry and its mirror); slots shared with other
// tiles are written as partials and summed by the fix-up kernel in
// ascending tile order. No float atomics: results are bitwise reproducible.
#include <algorithm>

#include "kernels.hpp"
#include "kernels_common.hpp"

namespace qxa {

// Reduction of one record: sum the contributions (padded LDS indices) of both
// staged matrices in the plan's order and write the target slot or partial.
// Empty inline slots hold the index of a zero kept in LDS, so the six reads
// are issued unconditionally (adding +0.0 leaves every sum unchanged).
__device__ __forceinline__ void reduce_record(const uint4 R, const double *sVm, const double *sVc, uint32_t zero,
                                              const uint16_t *__restrict__ ovf, double *__restrict__ M,
                                              double *__restrict__ C, double *__restrict__ Mpart,
                                              double *__restrict__ Cpart)
{
    uint32_t c[6] = {R.y & 0xffffu, R.y >> 16, R.z & 0xffffu, R.z >> 16, R.w & 0xffffu, R.w >> 16};
    const bool more = c[5] >= 0x8000u && c[5] != 0xffffu;
    const uint32_t c5 = c[5];
#pragma unroll
    for (int q = 1; q < 6; ++q) c[q] = (c[q] >= 0x8000u) ? zero : c[q];
    double vm[6], vc[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        vm[q] = sVm[c[q]];
        vc[q] = sVc[c[q]];
    }
    double am = vm[0], ac = vc[0];
#pragma unroll
    for (int q = 1; q < 6; ++q) {
        am += vm[q];
        ac += vc[q];
    }
    if (more) {
        const uint16_t *o = ovf + (c5 & 0x7fffu);
        const uint32_t n = o[0];
        for (uint32_t q = 1; q <= n; ++q) {
            am += sVm[o[q]];
            ac += sVc[o[q]];
        }
    }
    const int32_t t = int32_t(R.x);
    if (t >= 0) {
        if (M) M[t] = am;
        if (C) C[t] = ac;
    } else {
        if (M) Mpart[-int64_t(t) - 1] = am;
        if (C) Cpart[-int64_t(t) - 1] = ac;
    }
}

constexpr int kPrefetch = 4;  // records per thread loaded before the contraction

__device__ __forceinline__ void prefetch_records(const uint4 *__restrict__ rec, int64_t r0, int64_t r1, int stride,
                                                 uint4 (&pf)[kPrefetch])
{
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) {
        const int64_t k = r0 + threadIdx.x + int64_t(i) * stride;
        pf[i] = k < r1 ? rec[k] : make_uint4(0u, 0u, 0u, 0u);
    }
}

// All records of a tile: the prefetched batch first, then the rest in
// groups of kPrefetch independent loads.
__device__ __forceinline__ void tile_reduce(const uint4 (&pf)[kPrefetch], const FusedArgs &a, int64_t tile,
                                            const double *sVm, const double *sVc, uint32_t zero, int stride)
{
    const int64_t r0 = a.rec_ptr[tile], r1 = a.rec_ptr[tile + 1];
    const uint16_t *ovf = a.ovf + a.ovf_ptr[tile];
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i)
        if (r0 + threadIdx.x + int64_t(i) * stride < r1) reduce_record(pf[i], sVm, sVc, zero, ovf, a.M, a.C, a.Mpart, a.Cpart);
    for (int64_t k0 = r0 + threadIdx.x + int64_t(kPrefetch) * stride; k0 < r1; k0 += int64_t(kPrefetch) * stride) {
        uint4 R[kPrefetch];
#pragma unroll
        for (int i = 0; i < kPrefetch; ++i) {
            const int64_t k = k0 + int64_t(i) * stride;
            R[i] = k < r1 ? a.rec[k] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < kPrefetch; ++i)
            if (k0 + int64_t(i) * stride < r1) reduce_record(R[i], sVm, sVc, zero, ovf, a.M, a.C, a.Mpart, a.Cpart);
    }
}

template <int D, int P, int NQM, int NQC, typename CT, int T>
__global__ __launch_bounds__(T) void fused_kernel(FusedArgs a)
{
    using S = Shape<D, P>;
    extern __shared__ double sV[];  // [2][NS][T + 1] (row stride padded against bank conflicts)
    double *sVm = sV, *sVc = sV + S::NS * (T + 1);
    // the padding column of row 0 is never a contribution: keep a zero there
    if (threadIdx.x == 0) sVm[T] = sVc[T] = 0.0;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t p0 = tile * T;
    const int64_t ne = a.in.n_elem;
    const int lane = threadIdx.x;
    const int64_t p = p0 + lane;
    const bool active = p < ne;
    uint4 pf[kPrefetch];
    prefetch_records(a.rec, a.rec_ptr[tile], a.rec_ptr[tile + 1], T, pf);

    double A[S::NG], lm[NQM], lc[NQC];
    if (active) {
        int32_t v[S::NP];
#pragma unroll
        for (int i = 0; i < S::NP; ++i) v[i] = a.tconn[i * ne + p];
        const int64_t eid = (a.in.cm.kind == 2 || a.in.cc.kind == 2) ? int64_t(a.elem_order[p]) : p;
        if (!element_setup<D, P, NQM, NQC>(a.in, v, eid, A, lm, lc)) atomicOr(a.in.flags, 1);
        contract_mass<S::NS, NQM>(reinterpret_cast<const CT *>(a.Qm), lm,
                                  [&](int s, double x) { sVm[s * (T + 1) + lane] = x; });
        contract_stiff<P, S::NS, NQC, S::NG>(reinterpret_cast<const CT *>(a.Qc), lc, A,
                                             [&](int s, double x) { sVc[s * (T + 1) + lane] = x; });
    }
    lds_barrier();
    tile_reduce(pf, a, tile, sVm, sVc, T, T);
}

// ---------------------------------------------------------------------------
// Matrix-core variant for the dense contractions (P >= 2 with n_p(n_p+1)/2 >= 21
// symmetric rows): V^T = X^T Q^T on 16 x 16 x 4 FP64 (or FP32) MFMA tiles.
// A = X^T fragment (16 elements x 4 k), built per lane from Lambda and W with
// compile-time indices; B = Q^T fragment (4 k x 16 symmetric rows), staged in
// LDS once per workgroup in operand order (precomputed at plan time);
// D = V^T block (16 elements x 16 rows). The workgroup loops over tiles.
typedef double qxa_d4 __attribute__((ext_vector_type(4)));
typedef float qxa_f4 __attribute__((ext_vector_type(4)));

template <typename CT>
struct Mfma;
template <>
struct Mfma<double> {
    using acc_t = qxa_d4;
    // row (element) of accumulator register r held by lane l
    static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<float> {
    using acc_t = qxa_f4;
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <typename T>
__device__ __forceinline__ T sel4(int j, T a0, T a1, T a2, T a3)
{
    return j == 0 ? a0 : (j == 1 ? a1 : (j == 2 ? a2 : a3));
}

// x_m(k) = Lambda_m[k] (k < NQM, else 0)
template <int NQM>
__device__ __forceinline__ double xm_at(const double *lm, int k)
{
    return k < NQM ? lm[k] : 0.0;
}
// x_c(k) = (Lambda_c (.) W)[k] = lambda_q * A_g, k = q*NG + g (k < NQC*NG, else 0)
template <int NQC, int NG>
__device__ __forceinline__ double xc_at(const double *lc, const double *A, int k)
{
    return k < NQC * NG ? lc[k / NG] * A[k % NG] : 0.0;
}

// T = 16 * (waves per workgroup): one 16-element group per wave.
template <int D, int P, int NQM, int NQC, typename CT, int T>
__global__ __launch_bounds__(4 * T) void fused_mfma_kernel(FusedArgs a, int64_t n_tiles)
{
    using S = Shape<D, P>;
    using MF = Mfma<CT>;
    constexpr int NB = (S::NS + 15) / 16;
    constexpr int KSM = (NQM + 3) / 4;
    constexpr int KSC = (NQC * S::NG + 3) / 4;
    extern __shared__ __align__(16) unsigned char smem[];
    double *sVm = reinterpret_cast<double *>(smem);                                // [NS][T + 1]
    double *sVc = sVm + S::NS * (T + 1);                                           // [NS][T + 1]
    CT *sQ = reinterpret_cast<CT *>(smem + 2 * sizeof(double) * S::NS * (T + 1));  // [(KSM+KSC)][NB][64]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane >> 4, c16 = lane & 15;
    const int64_t ne = a.in.n_elem;

    {   // operand-ordered Q^T fragments, once per workgroup
        const CT *gq = reinterpret_cast<const CT *>(a.Qfrag);
        for (int k = tid; k < (KSM + KSC) * NB * 64; k += blockDim.x) sQ[k] = gq[k];
    }
    if (tid == 0) sVm[T] = sVc[T] = 0.0;  // zero kept in the (unused) padding column of row 0
    const bool need_eid = a.in.cm.kind == 2 || a.in.cc.kind == 2;
    TileWalk walk(n_tiles);
    int32_t v[S::NP];
    RawElem<D, P> raw;
    auto load_conn = [&](int64_t tt) {
        const int64_t pp = tt * T + 16 * wave + c16;
#pragma unroll
        for (int i = 0; i < S::NP; ++i) v[i] = pp < ne ? a.tconn[i * ne + pp] : 0;
    };
    if (walk.valid(walk.t)) {
        load_conn(walk.t);
        gather_raw<D, P>(a.in, v, raw);
    }
    for (int64_t tile = walk.t; walk.valid(tile); tile += walk.step) {
        const int64_t tnext = tile + walk.step;
        const int64_t p0 = tile * T;
        const int64_t p = p0 + 16 * wave + c16;  // this lane's element (4 lanes per element)
        uint4 pf[kPrefetch];
        prefetch_records(a.rec, a.rec_ptr[tile], a.rec_ptr[tile + 1], int(blockDim.x), pf);
        double A[S::NG], lm[NQM], lc[NQC];
        if (p < ne) {
            const int64_t eid = need_eid ? int64_t(a.elem_order[p]) : p;
            if (!setup_from_raw<D, P, NQM, NQC>(a.in, raw, v, eid, A, lm, lc) && j == 0) atomicOr(a.in.flags, 1);
        } else {
#pragma unroll
            for (int q = 0; q < S::NG; ++q) A[q] = 0.0;
#pragma unroll
            for (int q = 0; q < NQM; ++q) lm[q] = 0.0;
#pragma unroll
            for (int q = 0; q < NQC; ++q) lc[q] = 0.0;
        }
        if (walk.valid(tnext)) load_conn(tnext);  // in flight during the contraction
        lds_barrier();  // Q^T fragments ready (first tile) / staged V of the previous tile consumed
        typename MF::acc_t acc[NB];
        // V_m^T block: X_m^T (16 x 4 per step) times Q_m^T fragments
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = typename MF::acc_t{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
            const CT x = CT(sel4(j, xm_at<NQM>(lm, 4 * ks), xm_at<NQM>(lm, 4 * ks + 1), xm_at<NQM>(lm, 4 * ks + 2),
                                 xm_at<NQM>(lm, 4 * ks + 3)));
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb] = MF::step(x, sQ[(ks * NB + nb) * 64 + lane], acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int s = 16 * nb + c16;
            if (s < S::NS)
#pragma unroll
                for (int r = 0; r < 4; ++r) sVm[s * (T + 1) + 16 * wave + MF::row(lane, r)] = double(acc[nb][r]);
        }
        // V_c^T block: X_c^T = (Lambda_c (.) W)^T times Q_c^T fragments
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = typename MF::acc_t{0, 0, 0, 0};
        const CT *qc = sQ + KSM * NB * 64;
#pragma unroll
        for (int ks = 0; ks < KSC; ++ks) {
            const CT x = CT(sel4(j, xc_at<NQC, S::NG>(lc, A, 4 * ks), xc_at<NQC, S::NG>(lc, A, 4 * ks + 1),
                                 xc_at<NQC, S::NG>(lc, A, 4 * ks + 2), xc_at<NQC, S::NG>(lc, A, 4 * ks + 3)));
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb] = MF::step(x, qc[(ks * NB + nb) * 64 + lane], acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int s = 16 * nb + c16;
            if (s < S::NS)
#pragma unroll
                for (int r = 0; r < 4; ++r) sVc[s * (T + 1) + 16 * wave + MF::row(lane, r)] = double(acc[nb][r]);
        }
        if (walk.valid(tnext)) gather_raw<D, P>(a.in, v, raw);  // in flight during the reduction
        lds_barrier();
        tile_reduce(pf, a, tile, sVm, sVc, T, int(blockDim.x));
    }
}

// Shared slots: each output (upper or mirror entry, ascending CSR order) sums
// its partials in ascending tile order.
__global__ __launch_bounds__(256) void fixup_kernel(FixupArgs a)
{
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= a.n_fix) return;
    const int32_t lo = a.fix_ptr[f], hi = a.fix_ptr[f + 1];
    const int32_t t = a.fix_target[f];
    double m = 0.0, c = 0.0;
    for (int32_t k = lo; k < hi; ++k) {
        const int32_t pi = a.fix_idx[k];
        if (a.M) m += a.Mpart[pi];
        if (a.C) c += a.Cpart[pi];
    }
    if (a.M) a.M[t] = m;
    if (a.C) a.C[t] = c;
}

template <int D, int P>
constexpr bool use_mfma()
{
    return P >= 2 && !(D == 3 && P == 3);
}

bool fused_uses_mfma(int D, int P) { return P >= 2 && !(D == 3 && P == 3); }

// Resident workgroups for a persistent launch: CUs x workgroups per CU.
template <class K>
static unsigned persistent_grid(K kernel, int block, size_t lds, int64_t n_tiles)
{
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return unsigned(std::min<int64_t>(n_tiles, int64_t(cus) * per_cu));
}

hipError_t launch_fused(const FusedArgs &a, int64_t n_tiles, int D, int P, int nqm, int nqc, int precision,
                        hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
#define X(d, p, m, c)                                                                                          \
    if (D == d && P == p && nqm == m && nqc == c) {                                                            \
        constexpr int T = tile_size(d, p);                                                                     \
        if constexpr (use_mfma<d, p>()) {                                                                      \
            const size_t lds = 2 * size_t(T + 1) * Shape<d, p>::NS * sizeof(double) + qfrag_count(d, p, m, c) *    \
                                   (precision == 1 ? sizeof(float) : sizeof(double));                          \
            if (precision == 1) {                                                                              \
                auto k = fused_mfma_kernel<d, p, m, c, float, T>;                                              \
                k<<<persistent_grid(k, 4 * T, lds, n_tiles), 4 * T, lds, st>>>(a, n_tiles);                    \
            } else {                                                                                           \
                auto k = fused_mfma_kernel<d, p, m, c, double, T>;                                             \
                k<<<persistent_grid(k, 4 * T, lds, n_tiles), 4 * T, lds, st>>>(a, n_tiles);                    \
            }                                                                                                  \
        } else {                                                                                               \
            const size_t lds = 2 * size_t(T + 1) * Shape<d, p>::NS * sizeof(double);                            \
            if (precision == 1) fused_kernel<d, p, m, c, float, T><<<unsigned(n_tiles), T, lds, st>>>(a);      \
            else fused_kernel<d, p, m, c, double, T><<<unsigned(n_tiles), T, lds, st>>>(a);                    \
        }                                                                                                      \
        return hipGetLastError();                                                                              \
    }
    QXA_FORM_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_fixup(const FixupArgs &a, hipStream_t st)
{
    if (a.n_fix == 0) return hipSuccess;
    fixup_kernel<<<unsigned((a.n_fix + 255) / 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace qxa
