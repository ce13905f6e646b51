// Fused assembly kernel: all of Algorithm 2 after the reference tables, in one
// pass over the mesh.
//
// One workgroup per tile of T consecutive elements (plan order), one lane per
// element. Each lane computes its element's geometry and weighted coefficient
// columns (geometry, S, Lambda, W), then for each matrix in turn forms the element
// matrix V = Q X (symmetric-pair rows only) into LDS, and the
// workgroup reduces every CSR slot the tile touches over the tile's
// contributions in the plan's fixed order (the global assembly). Slots owned by the tile
// are written directly (upper entry and its mirror); slots shared with other
// tiles are written as partials and summed by the fix-up kernel in
// ascending tile order. No float atomics: results are bitwise reproducible.
#include <algorithm>

#include "../../include/qxa.h"
#include "kernels.hpp"
#include "kernels_common.hpp"

namespace qxa {

// Reduction of one record: sum the contributions (padded LDS indices) of both
// staged matrices in the plan's order and write the target slot or partial.
// Empty inline slots hold the index of a zero kept in LDS, so the six reads
// are issued unconditionally (adding +0.0 leaves every sum unchanged).
template <typename ST>
__device__ __forceinline__ void reduce_record(const uint4 R, const ST *sVm, const ST *sVc, uint32_t zero,
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
        vm[q] = double(sVm[c[q]]);
        vc[q] = double(sVc[c[q]]);
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
            am += double(sVm[o[q]]);
            ac += double(sVc[o[q]]);
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
template <typename ST>
__device__ __forceinline__ void tile_reduce(const uint4 (&pf)[kPrefetch], const FusedArgs &a, int64_t tile,
                                            const ST *sVm, const ST *sVc, uint32_t zero, int stride)
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

// Job of global tile g (uniform across the workgroup) and the tile's index in
// it; MULTI = false compiles the single-assembly launch (job carried by value).
template <bool MULTI>
__device__ __forceinline__ int job_of(const JobTable &jt, int64_t g, int64_t &local)
{
    if (!MULTI) {
        local = g;
        return -1;
    }
    int lo = 0, hi = jt.n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (jt.tile_end[mid] > g) hi = mid;
        else lo = mid + 1;
    }
    local = g - (lo > 0 ? jt.tile_end[lo - 1] : 0);
    return lo;
}
template <bool MULTI>
__device__ __forceinline__ FusedArgs args_of(const JobTable &jt, int j)
{
    if constexpr (MULTI) return jt.jobs[j];
    return jt.one;
}

template <int D, int P, int NQM, int NQC, typename CT, int T, bool MULTI>
__global__ __launch_bounds__(T) void fused_kernel(JobTable jt)
{
    using S = Shape<D, P>;
    extern __shared__ double sV[];  // [2][NS][T + 1] (row stride padded against bank conflicts)
    double *sVm = sV, *sVc = sV + S::NS * (T + 1);
    // the padding column of row 0 is never a contribution: keep a zero there
    if (threadIdx.x == 0) sVm[T] = sVc[T] = 0.0;
    int64_t tile;
    const FusedArgs a = args_of<MULTI>(jt, job_of<MULTI>(jt, xcd_tile(blockIdx.x, gridDim.x), tile));
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

// Split-precision operands of the 16 x 16 x 32 MFMA (gfx950): a value is
// carried as a sum of 16-bit terms (hi + lo, or hi + mid + lo) and the
// contraction keeps the products of total order < 2 (3 terms) or < 3 (6
// terms), accumulated in FP32.
typedef __bf16 qxa_bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 qxa_h8 __attribute__((ext_vector_type(8)));

template <int PF>
struct Split;
template <>
struct Split<QXA_BF16X2> {
    using vec = qxa_bf8;
    using elem = __bf16;
    static constexpr int NC = 2;  // components
    static constexpr int NT = 3;  // products: hh, hl, lh
    static constexpr int pa[3] = {0, 0, 1}, pb[3] = {0, 1, 0};
    static constexpr bool scaled = false;
    static __device__ __forceinline__ void split(float x, __bf16 *c)
    {
        c[0] = __bf16(x);
        c[1] = __bf16(x - float(c[0]));
    }
    static __device__ __forceinline__ qxa_f4 mfma(vec a, vec b, qxa_f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Split<QXA_BF16X3> {
    using vec = qxa_bf8;
    using elem = __bf16;
    static constexpr int NC = 3;
    static constexpr int NT = 6;  // hh, hm, mh, hl, mm, lh
    static constexpr int pa[6] = {0, 0, 1, 0, 1, 2}, pb[6] = {0, 1, 0, 2, 1, 0};
    static constexpr bool scaled = false;
    static __device__ __forceinline__ void split(float x, __bf16 *c)
    {
        c[0] = __bf16(x);
        const float r = x - float(c[0]);
        c[1] = __bf16(r);
        c[2] = __bf16(r - float(c[1]));
    }
    static __device__ __forceinline__ qxa_f4 mfma(vec a, vec b, qxa_f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Split<QXA_F16X2> {
    using vec = qxa_h8;
    using elem = _Float16;
    static constexpr int NC = 2;
    static constexpr int NT = 3;
    static constexpr int pa[3] = {0, 0, 1}, pb[3] = {0, 1, 0};
    static constexpr bool scaled = true;  // FP16 range: X is scaled per element by a power of two
    static __device__ __forceinline__ void split(float x, _Float16 *c)
    {
        c[0] = _Float16(x);
        c[1] = _Float16(x - float(c[0]));
    }
    static __device__ __forceinline__ qxa_f4 mfma(vec a, vec b, qxa_f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Contraction of one 16-element group, plain FP64/FP32 operands (16x16x4 MFMA).
// xat(k) is the k-th entry of this lane's element's X column (compile-time k).
template <typename CT, int K, int NB, int NS, int T, typename ST, class XAt>
__device__ __forceinline__ void contract_group_plain(const CT *sQ, XAt &&xat, ST *sV, int lane, int col0)
{
    using MF = Mfma<CT>;
    constexpr int KS = (K + 3) / 4;
    const int j = lane >> 4, c16 = lane & 15;
    typename MF::acc_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = typename MF::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const CT x = CT(sel4(j, xat(4 * ks), xat(4 * ks + 1), xat(4 * ks + 2), xat(4 * ks + 3)));
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = MF::step(x, sQ[(ks * NB + nb) * 64 + lane], acc[nb]);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int s = 16 * nb + c16;
        if (s < NS)
#pragma unroll
            for (int r = 0; r < 4; ++r) sV[s * (T + 1) + col0 + MF::row(lane, r)] = ST(acc[nb][r]);
    }
}

// Contraction of one 16-element group with split 16-bit operands
// (16x16x32 MFMA). Q^T fragments: [component][ks][nb][lane] x 8 values.
template <int PF, int K, int NB, int NS, int T, typename ST, class XAt>
__device__ __forceinline__ void contract_group_split(const uint4 *sQ, XAt &&xat, ST *sV, int lane, int col0,
                                                     double qinv)
{
    using SP = Split<PF>;
    using elem_t = typename SP::elem;
    constexpr int KS = (K + 31) / 32;
    const int j = lane >> 4, c16 = lane & 15;
    // this lane's X entries k = 32 ks + 8 j + t, t = 0..7
    double xv[KS][8];
    double amax = 0.0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            xv[ks][t] = sel4(j, xat(32 * ks + t), xat(32 * ks + 8 + t), xat(32 * ks + 16 + t), xat(32 * ks + 24 + t));
            amax = fmax(amax, fabs(xv[ks][t]));
        }
    double scale = 1.0, inv = 1.0;
    if constexpr (SP::scaled) {
        // element-wide max over the 4 lanes holding the element (lanes c16 + 16 j)
        amax = fmax(amax, __shfl_xor(amax, 16));
        amax = fmax(amax, __shfl_xor(amax, 32));
        if (amax > 0.0) {
            const int e = ilogb(amax);
            scale = ldexp(1.0, -e);
            inv = ldexp(1.0, e);
        }
    }
    typename SP::vec xc[KS][SP::NC];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            elem_t c[SP::NC];
            SP::split(float(xv[ks][t] * scale), c);
#pragma unroll
            for (int q = 0; q < SP::NC; ++q) xc[ks][q][t] = c[q];
        }
    qxa_f4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = qxa_f4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int tm = 0; tm < SP::NT; ++tm) {
                const uint4 qv = sQ[((SP::pb[tm] * KS + ks) * NB + nb) * 64 + lane];
                acc[nb] = SP::mfma(xc[ks][SP::pa[tm]], __builtin_bit_cast(typename SP::vec, qv), acc[nb]);
            }
    // undo the element scale and the table scale: row r of this lane is element 4 (lane/16) + r
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double ir = SP::scaled ? __shfl(inv, 4 * j + r) * qinv : 1.0;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int s = 16 * nb + c16;
            if (s < NS) sV[s * (T + 1) + col0 + 4 * j + r] = ST(double(acc[nb][r]) * ir);
        }
    }
}

template <int PF>
struct FormTraits {
    using stage_t = float;  // reduced forms stage V in FP32; CSR accumulation stays FP64
    using qplain_t = float;
};
template <>
struct FormTraits<QXA_FP64> {
    using stage_t = double;
    using qplain_t = double;
};

// T = 16 * (waves per workgroup): one 16-element group per wave.
template <int D, int P, int NQM, int NQC, int PF, int T, bool MULTI>
__global__ __launch_bounds__(4 * T) void fused_mfma_kernel(JobTable jt)
{
    using S = Shape<D, P>;
    using ST = typename FormTraits<PF>::stage_t;
    constexpr bool SPLIT = PF >= QXA_F16X2;
    constexpr int NB = (S::NS + 15) / 16;
    constexpr int KM = NQM, KC = NQC * S::NG;
    extern __shared__ __align__(16) unsigned char smem[];
    ST *sVm = reinterpret_cast<ST *>(smem);  // [NS][T + 1]
    ST *sVc = sVm + S::NS * (T + 1);         // [NS][T + 1]
    unsigned char *sQraw = smem + ((2 * sizeof(ST) * S::NS * (T + 1) + 15) / 16) * 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane >> 4, c16 = lane & 15;
    {   // operand-ordered Q^T fragments, once per workgroup (shared by every job of the launch)
        const FusedArgs a0 = args_of<MULTI>(jt, 0);
        const uint4 *gq = reinterpret_cast<const uint4 *>(a0.Qfrag);
        uint4 *dq = reinterpret_cast<uint4 *>(sQraw);
        for (int64_t k = tid; k < a0.qfrag_vec16; k += blockDim.x) dq[k] = gq[k];
    }
    if (tid == 0) sVm[T] = sVc[T] = ST(0);  // zero kept in the (unused) padding column of row 0
    TileWalk walk(jt.n_tiles);
    int32_t v[S::NP];
    RawElem<D, P> raw;
    // connectivity and gathers of (global) tile g, for the lane's element
    auto load_conn = [&](int64_t g) {
        int64_t lt;
        const FusedArgs b = args_of<MULTI>(jt, job_of<MULTI>(jt, g, lt));
        const int64_t pp = lt * T + 16 * wave + c16;
#pragma unroll
        for (int i = 0; i < S::NP; ++i) v[i] = pp < b.in.n_elem ? b.tconn[i * b.in.n_elem + pp] : 0;
    };
    auto gather = [&](int64_t g) {
        int64_t lt;
        const FusedArgs b = args_of<MULTI>(jt, job_of<MULTI>(jt, g, lt));
        gather_raw<D, P>(b.in, v, raw);
    };
    if (walk.valid(walk.t)) {
        load_conn(walk.t);
        gather(walk.t);
    }
    for (int64_t g = walk.t; walk.valid(g); g += walk.step) {
        const int64_t gnext = g + walk.step;
        int64_t tile;
        const FusedArgs a = args_of<MULTI>(jt, job_of<MULTI>(jt, g, tile));
        const int64_t ne = a.in.n_elem;
        const int64_t p = tile * T + 16 * wave + c16;  // this lane's element (4 lanes per element)
        uint4 pf[kPrefetch];
        prefetch_records(a.rec, a.rec_ptr[tile], a.rec_ptr[tile + 1], int(blockDim.x), pf);
        double A[S::NG], lm[NQM], lc[NQC];
        if (p < ne) {
            const int64_t eid = (a.in.cm.kind == 2 || a.in.cc.kind == 2) ? int64_t(a.elem_order[p]) : p;
            if (!setup_from_raw<D, P, NQM, NQC>(a.in, raw, v, eid, A, lm, lc) && j == 0) atomicOr(a.in.flags, 1);
        } else {
#pragma unroll
            for (int q = 0; q < S::NG; ++q) A[q] = 0.0;
#pragma unroll
            for (int q = 0; q < NQM; ++q) lm[q] = 0.0;
#pragma unroll
            for (int q = 0; q < NQC; ++q) lc[q] = 0.0;
        }
        if (walk.valid(gnext)) load_conn(gnext);  // in flight during the contraction
        lds_barrier();  // Q^T fragments ready (first tile) / staged V of the previous tile consumed
        // V_m^T = X_m^T Q_m^T with X_m = Lambda_m; V_c^T = X_c^T Q_c^T with X_c = Lambda_c (.) W
        auto xm = [&](int k) { return xm_at<NQM>(lm, k); };
        auto xc = [&](int k) { return xc_at<NQC, S::NG>(lc, A, k); };
        if constexpr (!SPLIT) {
            using CT = typename FormTraits<PF>::qplain_t;
            const CT *q = reinterpret_cast<const CT *>(sQraw);
            contract_group_plain<CT, KM, NB, S::NS, T, ST>(q, xm, sVm, lane, 16 * wave);
            contract_group_plain<CT, KC, NB, S::NS, T, ST>(q + ((KM + 3) / 4) * NB * 64, xc, sVc, lane, 16 * wave);
        } else {
            const uint4 *q = reinterpret_cast<const uint4 *>(sQraw);
            constexpr int NC = Split<PF>::NC;
            contract_group_split<PF, KM, NB, S::NS, T, ST>(q, xm, sVm, lane, 16 * wave, a.qinv_m);
            contract_group_split<PF, KC, NB, S::NS, T, ST>(q + NC * ((KM + 31) / 32) * NB * 64, xc, sVc, lane,
                                                          16 * wave, a.qinv_c);
        }
        if (walk.valid(gnext)) gather(gnext);  // in flight during the reduction
        lds_barrier();
        tile_reduce(pf, a, tile, sVm, sVc, T, int(blockDim.x));
    }
}

// Shared slots: each output (upper or mirror entry, ascending CSR order) sums
// its partials in ascending tile order.
__global__ __launch_bounds__(256) void fixup_kernel(FixupTable ft)
{
    int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= ft.n_fix) return;
    int jb = -1;
    if (ft.n_jobs > 0) {
        int lo = 0, hi = ft.n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ft.fix_end[mid] > f) hi = mid;
            else lo = mid + 1;
        }
        f -= lo > 0 ? ft.fix_end[lo - 1] : 0;
        jb = lo;
    }
    const FixupArgs a = jb < 0 ? ft.one : ft.jobs[jb];
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
    (void)hipGetLastError();  // a failed occupancy query must not be reported as a launch error
    return unsigned(std::min<int64_t>(n_tiles, int64_t(cus) * per_cu));
}

hipError_t launch_fused(const JobTable &jt, int D, int P, int nqm, int nqc, int precision, hipStream_t st)
{
    const int64_t n_tiles = jt.n_tiles;
    if (n_tiles == 0) return hipSuccess;
    const FusedArgs &a = jt.one;  // the first job (Q^T fragment size is shared by all jobs)
#define QXA_LAUNCH_MFMA(d, p, m, c, PF, MULTI)                                                            \
    {                                                                                                     \
        constexpr int T = tile_size(d, p);                                                                \
        using STg = typename FormTraits<PF>::stage_t;                                                     \
        const size_t lds = ((2 * sizeof(STg) * Shape<d, p>::NS * (T + 1) + 15) / 16) * 16 +               \
                           size_t(a.qfrag_vec16) * 16;                                                    \
        auto k = fused_mfma_kernel<d, p, m, c, PF, T, MULTI>;                                             \
        k<<<persistent_grid(k, 4 * T, lds, n_tiles), 4 * T, lds, st>>>(jt);                               \
    }
#define X(d, p, m, c)                                                                                      \
    if (D == d && P == p && nqm == m && nqc == c) {                                                        \
        constexpr int T = tile_size(d, p);                                                                 \
        const bool multi = jt.n_jobs > 0;                                                                  \
        if (multi && precision != QXA_FP64 && precision != QXA_FP32) return hipErrorInvalidValue;          \
        if constexpr (use_mfma<d, p>()) {                                                                  \
            switch (precision * 2 + int(multi)) {                                                          \
            case 2 * QXA_FP64: QXA_LAUNCH_MFMA(d, p, m, c, QXA_FP64, false) break;                         \
            case 2 * QXA_FP64 + 1: QXA_LAUNCH_MFMA(d, p, m, c, QXA_FP64, true) break;                      \
            case 2 * QXA_FP32: QXA_LAUNCH_MFMA(d, p, m, c, QXA_FP32, false) break;                         \
            case 2 * QXA_FP32 + 1: QXA_LAUNCH_MFMA(d, p, m, c, QXA_FP32, true) break;                      \
            case 2 * QXA_F16X2: QXA_LAUNCH_MFMA(d, p, m, c, QXA_F16X2, false) break;                       \
            case 2 * QXA_BF16X2: QXA_LAUNCH_MFMA(d, p, m, c, QXA_BF16X2, false) break;                     \
            case 2 * QXA_BF16X3: QXA_LAUNCH_MFMA(d, p, m, c, QXA_BF16X3, false) break;                     \
            default: return hipErrorInvalidValue;                                                          \
            }                                                                                              \
        } else {                                                                                           \
            if (precision != QXA_FP64 && precision != QXA_FP32) return hipErrorInvalidValue;               \
            const size_t lds = 2 * size_t(T + 1) * Shape<d, p>::NS * sizeof(double);                      \
            const unsigned grid = unsigned(n_tiles);                                                       \
            if (precision == QXA_FP32) {                                                                   \
                if (multi) fused_kernel<d, p, m, c, float, T, true><<<grid, T, lds, st>>>(jt);              \
                else fused_kernel<d, p, m, c, float, T, false><<<grid, T, lds, st>>>(jt);                  \
            } else {                                                                                       \
                if (multi) fused_kernel<d, p, m, c, double, T, true><<<grid, T, lds, st>>>(jt);             \
                else fused_kernel<d, p, m, c, double, T, false><<<grid, T, lds, st>>>(jt);                 \
            }                                                                                              \
        }                                                                                                  \
        return hipGetLastError();                                                                          \
    }
    QXA_FORM_CASES(X)
#undef X
#undef QXA_LAUNCH_MFMA
    return hipErrorInvalidValue;
}

hipError_t launch_fixup(const FixupTable &ft, hipStream_t st)
{
    if (ft.n_fix == 0) return hipSuccess;
    fixup_kernel<<<unsigned((ft.n_fix + 255) / 256), 256, 0, st>>>(ft);
    return hipGetLastError();
}

}  // namespace qxa
