// Fused assembly kernels: all of Algorithm 2 after the reference tables, in
// one pass over the mesh.
//
// A workgroup walks the tiles of its chains (plan order). For each tile it
// computes every element's geometry and weighted coefficient columns
// (geometry, S, Lambda, W), forms the element matrices V = Q X (symmetric-pair
// rows only) into LDS, and reduces the tile's outputs (the global assembly):
// for every CSR slot the tile touches, the tile's contributions in the
// plan's fixed order, added to a carry entry of an earlier tile of the chain
// when there is one, and stored as the CSR value (upper slot and mirror), as
// a carry entry for a later tile, or as a partial that the fix-up kernel sums
// in ascending tile order. No float atomics: results are bitwise
// reproducible.
#include <algorithm>
#include <type_traits>

#include "../../include/qxa.h"
#include "kernels.hpp"
#include "kernels_common.hpp"

// This file is built twice: on its own (the rule sizes of QXA_FORM_CASES_TUNED,
// the fix-up and the dispatch) and through kernels_fused_padded.hip (those of
// QXA_FORM_CASES_PADDED), so that the two sets of kernels compile in parallel.
#ifdef QXA_FUSED_PADDED
#define QXA_FUSED_CASES QXA_FORM_CASES_PADDED
#define QXA_PART(name) name##_padded
#else
#define QXA_FUSED_CASES QXA_FORM_CASES_TUNED
#define QXA_PART(name) name##_tuned
#endif

namespace qxa {

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
        if (uniform_table(jt.tile_end)[mid] > g) hi = mid;
        else lo = mid + 1;
    }
    local = g - (lo > 0 ? uniform_table(jt.tile_end)[lo - 1] : 0);
    return lo;
}
template <bool MULTI>
__device__ __forceinline__ FusedArgs args_of(const JobTable &jt, int j)
{
    if constexpr (MULTI) {
        // word by word through the scalar path (j is uniform)
        static_assert(sizeof(FusedArgs) % 8 == 0, "FusedArgs is copied in 8-byte words");
        FusedArgs r;
        const auto src = uniform_table(reinterpret_cast<const uint64_t *>(jt.jobs + j));
        uint64_t *dst = reinterpret_cast<uint64_t *>(&r);
#pragma unroll
        for (size_t i = 0; i < sizeof(FusedArgs) / 8; ++i) dst[i] = src[i];
        return r;
    }
    return jt.one;
}

typedef uint32_t qxa_u2 __attribute__((ext_vector_type(2)));

// Raw buffer resource over [base, base + bytes) for stores: stride 0, word 3
// as the gfx9 family takes it (32-bit data format, no swizzle, no index
// range). A store whose offset is at or past `bytes` is dropped by the
// hardware; bytes = 0 drops every store.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t store_rsrc(void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, int(bytes), 0x00020000);
}

// Tiles of a workgroup: the chains jt.chain_ptr assigns it, one range of
// global tiles. With one chain per workgroup the chains are spread
// XCD-aware (the workgroups of one XCD take consecutive chains, which are
// neighbouring regions of the mesh).
__device__ __forceinline__ TileWalk chain_walk(const JobTable &jt)
{
    const int64_t G = gridDim.x, b = blockIdx.x, nc = jt.n_chains;
    // chains of one tile (no carries): the XCDs each walk an eighth of the tile order with
    // their workgroups side by side, so that tiles sharing CSR lines run at the same time
    // on one XCD and their writes meet in its L2
    if (nc == jt.n_tiles) return TileWalk(jt.n_tiles);
    int64_t c0, c1;
    if (G == nc) {
        c0 = xcd_tile(b, nc);
        c1 = c0 + 1;
    } else {
        c0 = b * nc / G;
        c1 = (b + 1) * nc / G;
    }
    return TileWalk(uniform_table(jt.chain_ptr)[c0], uniform_table(jt.chain_ptr)[c1]);
}

// ---------------------------------------------------------------------------
// Outputs of a tile (plan_format.hpp): 16-byte units, read by the consumer
// threads in rounds (one unit per thread), CH rounds per chunk, the next
// chunk (or the next tile's first) loaded before the current one is stored.
// Each output sums its entries (a carry entry first, then the staged pairs
// (V_m, V_c)) in FP64 and stores the sum: CSR values through buffer stores
// that drop lanes without a CSR target (so every round issues the same two
// stores and a wait for the next units leaves them in flight), a carry entry
// (LDS) or a partial (global).

// Entries of an output: staged pairs (ST2: FP64 or FP32 pairs) and, as the
// first entry only, a carry entry (an FP64 pair).
template <typename ST>
struct Entries {
    using ST2 = typename std::conditional<sizeof(ST) == 8, double2, float2>::type;
    const ST2 *v2;
    const double2 *carry;
    uint32_t cb, zero;
    __device__ __forceinline__ double2 pair(uint32_t c) const
    {
        const ST2 x = v2[c];
        return make_double2(double(x.x), double(x.y));
    }
    // first entry: a staged pair or a carry entry; with FP64 staging one read
    // through a selected address, else both reads (each in bounds) and a select
    __device__ __forceinline__ double2 first(uint32_t c) const
    {
        if constexpr (sizeof(ST) == 8) {
            return *(c < cb ? reinterpret_cast<const double2 *>(v2) + c : carry + (c - cb));
        } else {
            const bool isc = c >= cb;
            const double2 xc = carry[isc ? c - cb : 0u];
            const double2 xv = pair(isc ? zero : c);
            return isc ? xc : xv;
        }
    }
};

// The sums of a single unit {t, c0|c1, c2|c3, c4|c5} (absent entries index the zero pair).
template <typename ST>
__device__ __forceinline__ void unit_sums(const uint4 U, const Entries<ST> &E, double &am, double &ac)
{
    const uint32_t c[6] = {U.y & 0xffffu, U.y >> 16, U.z & 0xffffu, U.z >> 16, U.w & 0xffffu, U.w >> 16};
    double2 v[6];
    v[0] = E.first(c[0]);
#pragma unroll
    for (int q = 1; q < 6; ++q) v[q] = E.pair(c[q]);
    am = v[0].x;
    ac = v[0].y;
#pragma unroll
    for (int q = 1; q < 6; ++q) {
        am += v[q].x;
        ac += v[q].y;
    }
}

// The two outputs of a pair unit {ta, a0|a1, tb, b0|b1}.
template <typename ST>
__device__ __forceinline__ void pair_sums(const uint4 U, const Entries<ST> &E, double &ama, double &aca, double &amb,
                                          double &acb)
{
    const double2 a0 = E.first(U.y & 0xffffu), a1 = E.pair(U.y >> 16);
    const double2 b0 = E.first(U.w & 0xffffu), b1 = E.pair(U.w >> 16);
    ama = a0.x + a1.x;
    aca = a0.y + a1.y;
    amb = b0.x + b1.x;
    acb = b0.y + b1.y;
}

// Outputs of several units (plan_format.hpp): lane l of the wave adds the sum
// of lane l - d when lanes l - d .. l - 1 all continue into the next one
// (their bits in `ext`), for d = 1, 2, ..., 32; each segment's last lane then
// holds the segment's sum. Called by all lanes of a wave with ext != 0.
__device__ __forceinline__ void ext_segment_sums(uint64_t ext, double &am, double &ac)
{
    const int l = __lane_id();
#pragma unroll
    for (int d = 1; d < kSegLanes; d <<= 1) {
        const double tm = __shfl_up(am, d), tc = __shfl_up(ac, d);
        const uint64_t run = (uint64_t(1) << d) - 1;
        if (l >= d && ((ext >> (l - d)) & run) == run) {
            am += tm;
            ac += tc;
        }
    }
}

// Consumer threads (NCT of them, ct = 0 .. NCT - 1) of a workgroup: the units
// of every tile of the walk. on_tile(k) is called before tile k of the walk is
// reduced: it waits for (or stages) the tile's element matrices and returns
// their LDS pairs.
template <typename ST, bool MULTI, bool BUF, int CH, int NCT, class OnTile>
__device__ __forceinline__ void consume_units(const JobTable &jt, const TileWalk &walk, int ct, double2 *carry,
                                              uint32_t cb, uint32_t zero, OnTile &&on_tile)
{
    const int cw = 64 * __builtin_amdgcn_readfirstlane(ct >> 6);  // this wave's first lane (uniform)
    uint4 R[CH], Rn[CH];
    // unit of round q of chunk c: r0 + (c * CH + q) * NCT + ct, clamped to the tile
    auto load_chunk = [&](const uint4 *rec, int64_t r0, int64_t r1, int64_t c, uint4(&dst)[CH]) {
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int64_t k = r0 + (c * CH + q) * NCT + ct;
            dst[q] = rec[k < r1 ? k : r1 - 1];
        }
    };
    // tile ranges are uniform: read them through the scalar path, so that
    // waiting for them never waits for this wave's outstanding stores
    auto tile_range = [&](const FusedArgs &b, int64_t t, int64_t &r0, int64_t &r1) {
        r0 = uniform_table(b.rec_ptr)[t];
        r1 = uniform_table(b.rec_ptr)[t + 1];
    };
    static_assert(NCT % kSegLanes == 0, "rounds of whole waves");
    int64_t g = walk.t;
    {
        int64_t tile, r0, r1;
        const FusedArgs a = args_of<MULTI>(jt, job_of<MULTI>(jt, g, tile));
        tile_range(a, tile, r0, r1);
        load_chunk(reinterpret_cast<const uint4 *>(a.rec), r0, r1, 0, R);
    }
    for (int64_t k = 0;; ++k, g += walk.step) {
        const ST *bV = on_tile(k);
        const Entries<ST> E{reinterpret_cast<const typename Entries<ST>::ST2 *>(bV), carry, cb, zero};
        int64_t tile, r0, r1;
        const FusedArgs a = args_of<MULTI>(jt, job_of<MULTI>(jt, g, tile));
        tile_range(a, tile, r0, r1);
        const int64_t rm = uniform_table(a.rec_mid)[tile];  // pair units end here
        const int64_t nch = (r1 - r0 + int64_t(CH) * NCT - 1) / (int64_t(CH) * NCT);
        const int64_t gn = g + walk.step;
        const bool more = walk.valid(gn);
        const uint4 *rec = reinterpret_cast<const uint4 *>(a.rec), *rec_n = rec;
        int64_t r0n = r0, r1n = r1;
        if (more) {
            int64_t tn;
            const FusedArgs an = args_of<MULTI>(jt, job_of<MULTI>(jt, gn, tn));
            rec_n = reinterpret_cast<const uint4 *>(an.rec);
            tile_range(an, tn, r0n, r1n);
        }
        const __amdgpu_buffer_rsrc_t rM = store_rsrc(a.M ? a.M : a.sink, a.M ? a.bytes_vals : 0u);
        const __amdgpu_buffer_rsrc_t rC = store_rsrc(a.C ? a.C : a.sink, a.C ? a.bytes_vals : 0u);
        double2 *part = reinterpret_cast<double2 *>(a.part);
        for (int64_t c = 0; c < nch; ++c) {
            // next chunk: the following one of this tile, else the next tile's first
            const bool inner = c + 1 < nch;
            load_chunk(inner ? rec : rec_n, inner ? r0 : r0n, inner ? r1 : r1n, inner ? c + 1 : 0, Rn);
            const uint32_t none = zero | (zero << 16);  // no entries
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int64_t k0 = r0 + (c * CH + q) * NCT;
                if (!BUF && k0 >= r1) continue;  // the whole round is past the tile's units (uniform)
                const int64_t ku = k0 + ct, kw = k0 + cw;
                const bool active = ku < r1, pair = ku < rm;  // rm <= r1: a pair unit is active
                const uint4 U = R[q];
                const int32_t ta = int32_t(U.x), tb = int32_t(U.z);
                double ama = 0.0, aca = 0.0, amb = 0.0, acb = 0.0;
                if (k0 < r1) {  // (uniform) no LDS reads for a round past the tile's units
                    if (kw + 63 < rm) {  // the wave's units are all pairs
                        pair_sums(U, E, ama, aca, amb, acb);
                    } else if (kw >= rm) {  // all singles; idle lanes read the zero pair
                        unit_sums(active ? U : make_uint4(0u, none, none, none), E, ama, aca);
                    } else if (pair) {  // the wave that holds the boundary
                        pair_sums(U, E, ama, aca, amb, acb);
                    } else {
                        unit_sums(active ? U : make_uint4(0u, none, none, none), E, ama, aca);
                    }
                }
                const uint64_t ext = __builtin_amdgcn_ballot_w64(active && !pair && ta == kCodeExt);
                if (ext) ext_segment_sums(ext, ama, aca);  // (uniform)
                const bool csra = active && ta >= 0 && ta < kCodeCarry, csrb = pair && tb >= 0 && tb < kCodeCarry;
                if constexpr (BUF) {
                    const uint32_t drop = 0x80000000u;
                    const uint32_t oa = csra ? uint32_t(ta) * 8u : drop;
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(qxa_u2, ama), rM, oa, 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(qxa_u2, aca), rC, oa, 0, 0);
                    if (kw < rm) {  // (uniform) second outputs of the wave's pair units
                        const uint32_t ob = csrb ? uint32_t(tb) * 8u : drop;
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(qxa_u2, amb), rM, ob, 0, 0);
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(qxa_u2, acb), rC, ob, 0, 0);
                    }
                } else {
                    if (csra) {
                        if (a.M) a.M[ta] = ama;
                        if (a.C) a.C[ta] = aca;
                    }
                    if (csrb) {
                        if (a.M) a.M[tb] = amb;
                        if (a.C) a.C[tb] = acb;
                    }
                }
                // carries and partials sit at the end of each group: branches (skipped by
                // waves without one) add stores but never remove the ones above
                if (active && ta >= kCodeCarry && ta < kCodeCarryEnd) carry[ta - kCodeCarry] = make_double2(ama, aca);
                if (active && ta < 0) part[-int64_t(ta) - 1] = make_double2(ama, aca);
                if (pair && tb >= kCodeCarry && tb < kCodeCarryEnd) carry[tb - kCodeCarry] = make_double2(amb, acb);
                if (pair && tb < 0) part[-int64_t(tb) - 1] = make_double2(amb, acb);
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) R[q] = Rn[q];
        }
        if (!more) break;
    }
}

// ---------------------------------------------------------------------------
// Vector-ALU variant (P1): one workgroup per tile, one lane per element. The
// lanes load their first output units, form their element's matrices into LDS
// as (V_m, V_c) pairs, then reduce the tile's units. Every tile is a chain of
// its own (no carries): the elements are cheap to form and many small
// workgroups per CU hide the memory latency better than a pipeline.
constexpr int kP1Prefetch = 4;  // units per thread loaded before the contraction

template <int D, int P, int NQM, int NQC, typename CT, int T, bool MULTI>
__global__ __launch_bounds__(T) void fused_kernel(JobTable jt)
{
    using S = Shape<D, P>;
    extern __shared__ __align__(16) double2 sP[];  // [NS][T + 1] pairs
    double *sV = reinterpret_cast<double *>(sP);
    if (threadIdx.x == 0) sP[T] = make_double2(0.0, 0.0);  // the zero pair: column T of pair 0
    int64_t tile;
    const FusedArgs a = args_of<MULTI>(jt, job_of<MULTI>(jt, xcd_tile(blockIdx.x, gridDim.x), tile));
    const int64_t ne = a.in.n_elem;
    const int64_t r0 = a.rec_ptr[tile], r1 = a.rec_ptr[tile + 1], rm = a.rec_mid[tile];
    const uint4 *rec = reinterpret_cast<const uint4 *>(a.rec);
    uint4 pf[kP1Prefetch];
#pragma unroll
    for (int i = 0; i < kP1Prefetch; ++i) {
        const int64_t k = r0 + threadIdx.x + int64_t(i) * T;
        pf[i] = k < r1 ? rec[k] : make_uint4(0u, 0u, 0u, 0u);
    }
    const int64_t p = tile * T + threadIdx.x;
    if (p < ne) {
        double A[S::NG], lm[NQM], lc[NQC];
        int32_t v[S::NP];
#pragma unroll
        for (int i = 0; i < S::NP; ++i) v[i] = a.tconn[i * ne + p];
        const int64_t eid = (a.in.cm.kind == 2 || a.in.cc.kind == 2) ? int64_t(a.elem_order[p]) : p;
        if (!element_setup<D, P, NQM, NQC>(a.in, v, eid, A, lm, lc)) atomicOr(a.in.flags, 1);
        // a matrix that is not requested is not formed (its sums are never stored)
        if (a.M)
            contract_mass<S::NS, NQM>(reinterpret_cast<const CT *>(a.Qm), lm,
                                      [&](int s, double x) { sV[2 * (s * (T + 1) + threadIdx.x)] = x; });
        if (a.C)
            contract_stiff<P, S::NS, NQC, S::NG>(reinterpret_cast<const CT *>(a.Qc), lc, A, [&](int s, double x) {
                sV[2 * (s * (T + 1) + threadIdx.x) + 1] = x;
            });
    }
    lds_barrier();
    // no carry entries: every entry is a staged pair
    const Entries<double> E{reinterpret_cast<const double2 *>(sP), nullptr, 0xffffu, uint32_t(T)};
    double2 *part = reinterpret_cast<double2 *>(a.part);
    auto put = [&](int32_t t, double am, double ac) {
        if (t >= 0 && t < kCodeCarry) {
            if (a.M) a.M[t] = am;
            if (a.C) a.C[t] = ac;
        } else if (t < 0) {
            part[-int64_t(t) - 1] = make_double2(am, ac);
        }
    };
    // unit k of this lane (k >= r1: none); called by whole waves, since an
    // output of several units is summed across lanes
    auto reduce = [&](int64_t k, const uint4 U) {
        const bool act = k < r1, pr = act && k < rm;
        double ama = 0.0, aca = 0.0, amb = 0.0, acb = 0.0;
        if (pr)
            pair_sums(U, E, ama, aca, amb, acb);
        else if (act)
            unit_sums(U, E, ama, aca);
        const uint64_t ext = __builtin_amdgcn_ballot_w64(act && !pr && int32_t(U.x) == kCodeExt);
        if (ext) ext_segment_sums(ext, ama, aca);
        if (act) {
            put(int32_t(U.x), ama, aca);
            if (pr) put(int32_t(U.z), amb, acb);
        }
    };
    static_assert(T % kSegLanes == 0, "rounds of whole waves");
    const int64_t wb = r0 + (threadIdx.x & ~(kSegLanes - 1));  // this wave's first unit (uniform)
#pragma unroll
    for (int i = 0; i < kP1Prefetch; ++i)
        if (wb + int64_t(i) * T < r1) reduce(r0 + threadIdx.x + int64_t(i) * T, pf[i]);
    for (int64_t w0 = wb + int64_t(kP1Prefetch) * T; w0 < r1; w0 += int64_t(kP1Prefetch) * T) {
        const int64_t k0 = w0 + (threadIdx.x & (kSegLanes - 1));
        uint4 U[kP1Prefetch];
#pragma unroll
        for (int i = 0; i < kP1Prefetch; ++i) {
            const int64_t k = k0 + int64_t(i) * T;
            U[i] = k < r1 ? rec[k] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < kP1Prefetch; ++i)
            if (w0 + int64_t(i) * T < r1) reduce(k0 + int64_t(i) * T, U[i]);
    }
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
// xk(ks) is this lane's A-operand entry of k-step ks: X[k = 4 ks + lane / 16]
// of the lane's element (compile-time ks).
// NBW row blocks starting at nb0 (of NB) are computed; sQ may be LDS or global.
template <typename CT, int K, int NB, int NS, int T, typename ST, int STRIDE, int NBW = NB, class XK>
__device__ __forceinline__ void contract_group_plain(const CT *sQ, XK &&xk, ST *sV, int lane, int col0, int nb0 = 0)
{
    using MF = Mfma<CT>;
    constexpr int KS = (K + 3) / 4;
    const int c16 = lane & 15;
    typename MF::acc_t acc[NBW];
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) acc[nb] = typename MF::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const CT x = CT(xk(ks));
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
            if (NBW == NB || nb0 + nb < NB)
                acc[nb] = MF::step(x, sQ[(ks * NB + nb0 + nb) * 64 + lane], acc[nb]);
    }
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
        const int s = 16 * (nb0 + nb) + c16;
        if (s < NS)
#pragma unroll
            for (int r = 0; r < 4; ++r) sV[STRIDE * (s * (T + 1) + col0 + MF::row(lane, r))] = ST(acc[nb][r]);
    }
}

// Contraction of one 16-element group with split 16-bit operands
// (16x16x32 MFMA). Q^T fragments: [component][ks][nb][lane] x 8 values.
// xv(ks, t) is this lane's entry X[k = 32 ks + 8 (lane / 16) + t] (compile-time ks, t).
template <int PF, int K, int NB, int NS, int T, typename ST, int STRIDE, class XV>
__device__ __forceinline__ void contract_group_split(const uint4 *sQ, XV &&xvf, ST *sV, int lane, int col0,
                                                     double qinv)
{
    using SP = Split<PF>;
    using elem_t = typename SP::elem;
    constexpr int KS = (K + 31) / 32;
    const int j = lane >> 4, c16 = lane & 15;
    double scale = 1.0, inv = 1.0;
    if constexpr (SP::scaled) {
        // element-wide max over the 4 lanes holding the element (lanes c16 + 16 j);
        // the X entries are recomputed below rather than held
        double amax = 0.0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int t = 0; t < 8; ++t) amax = fmax(amax, fabs(xvf(ks, t)));
        amax = fmax(amax, __shfl_xor(amax, 16));
        amax = fmax(amax, __shfl_xor(amax, 32));
        if (amax > 0.0) {
            const int e = ilogb(amax);
            scale = ldexp(1.0, -e);
            inv = ldexp(1.0, e);
        }
    }
    qxa_f4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = qxa_f4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {  // one 32-wide K block at a time: split, then multiply
        typename SP::vec xc[SP::NC];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            elem_t c[SP::NC];
            SP::split(float(xvf(ks, t) * scale), c);
#pragma unroll
            for (int q = 0; q < SP::NC; ++q) xc[q][t] = c[q];
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int tm = 0; tm < SP::NT; ++tm) {
                const uint4 qv = sQ[((SP::pb[tm] * KS + ks) * NB + nb) * 64 + lane];
                acc[nb] = SP::mfma(xc[SP::pa[tm]], __builtin_bit_cast(typename SP::vec, qv), acc[nb]);
            }
    }
    // undo the element scale and the table scale: row r of this lane is element 4 (lane/16) + r
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double ir = SP::scaled ? __shfl(inv, 4 * j + r) * qinv : 1.0;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int s = 16 * nb + c16;
            if (s < NS) sV[STRIDE * (s * (T + 1) + col0 + 4 * j + r)] = ST(double(acc[nb][r]) * ir);
        }
    }
}

// Quadrature nodes whose weighted coefficients a lane of an element needs on
// the matrix cores: lane group j = lane / 16 holds the nodes q = 4 m + j. The K
// order of the Q^T fragments makes this so:
//   16x16x4 forms (lane holds k = 4 ks + j): mass k = q; conductivity
//     k = g * NQP + q with NQP = n_q rounded up to 4;
//   split forms (lane holds k = 32 ks + 8 j + t, t < 8): each 8-slot segment
//     holds QPS = 8 / G whole (node, component) groups of G slots, node
//     q = 4 (QPS ks + t / G) + j, component t % G (G = 1 for the mass,
//     d(d+1)/2 for the conductivity); the remaining slots are zero.
template <int NQM, int NQC, int NG>
struct LaneQ {
    static constexpr int NQP = (NQC + 3) / 4 * 4;
    static constexpr int MM = (NQM + 3) / 4;  // mass nodes per lane
    static constexpr int MC = NQP / 4;        // conductivity nodes per lane
    static constexpr int QPSM = 8, QPSC = 8 / NG;
    static constexpr int KSM = (MM + QPSM - 1) / QPSM, KSC = (MC + QPSC - 1) / QPSC;  // split K blocks
    static __device__ __forceinline__ int q(int j, int m) { return 4 * m + j; }
};

// Per-lane setup on the matrix-core path: geometry (all lanes) and the
// weighted coefficients Lambda of this lane's quadrature nodes only (zero for
// nodes past n_q). Basis values and weights come from LDS, q-major
// (sPhi[q * NP + i]). Returns false when a coefficient value is not finite.
template <int D, int P, int NQM, int NQC>
__device__ __forceinline__ bool lane_setup(const FormInputs &in, const RawElem<D, P> &r, const int32_t *tconn,
                                           int64_t pos, int64_t eid, int j, const double *sPhiM,
                                           const double *sPhiC, const double *sWM, const double *sWC, double *A,
                                           double *lm, double *lc)
{
    using L = LaneQ<NQM, NQC, Shape<D, P>::NG>;
    constexpr int NP = Shape<D, P>::NP;
    double babs;
    geometry_from<D>(r.x, babs, A, in.aniso, in.K);
    bool ok = true;
#pragma unroll
    for (int m = 0; m < L::MM; ++m) {
        const int q = L::q(j, m);
        double v = 0.0;
        if (q < NQM) {
            double s;
            if (in.cm.kind == 0) {
                s = in.cm.value;
            } else if (in.cm.kind == 1) {
                double uh = 0.0;
#pragma unroll
                for (int i = 0; i < NP; ++i) uh = fma(sPhiM[q * NP + i], r.u[i], uh);
                s = apply_law(in.cm, uh);
            } else {
                s = apply_law(in.cm, qe_value(in.cm, q, in.n_elem, eid));
            }
            v = sWM[q] * s * babs;
        }
        lm[m] = v;
        ok &= isfinite(v);
    }
    const bool other = in.cc.kind == 1 && in.cm.kind == 1 && in.cc.field != in.cm.field;
#pragma unroll
    for (int m = 0; m < L::MC; ++m) {
        const int q = L::q(j, m);
        double v = 0.0;
        if (q < NQC) {
            double s;
            if (in.cc.kind == 0) {
                s = in.cc.value;
            } else if (in.cc.kind == 1) {
                double uh = 0.0;
                if (!other) {
#pragma unroll
                    for (int i = 0; i < NP; ++i) uh = fma(sPhiC[q * NP + i], r.u[i], uh);
                } else {  // a second nodal field, read through the element's connectivity
#pragma unroll
                    for (int i = 0; i < NP; ++i)
                        uh = fma(sPhiC[q * NP + i], in.cc.field[tconn[i * in.n_elem + pos]], uh);
                }
                s = apply_law(in.cc, uh);
            } else {
                s = apply_law(in.cc, qe_value(in.cc, q, in.n_elem, eid));
            }
            v = sWC[q] * s * babs;
        }
        lc[m] = v;
        ok &= isfinite(v);
    }
    return ok;
}

// Isoparametric elements on the matrix-core path: the four lanes of an element
// (j = lane / 16) each gather a quarter of its node positions (items
// it = 4 t + j of the node-major list, it = node * D + component) and of its
// first nodal field (node 4 t + j), one tile ahead; iso_expand rebuilds the
// whole element on every lane with cross-lane reads (the lanes of one element
// are active together), so that no lane keeps all positions in registers
// while the previous tile is contracted.
template <int D, int P>
struct IsoRaw {
    // whole groups of four nodes (D items per lane each); items past the last node repeat a valid position
    static constexpr int NP = Shape<D, P>::NP, NU = (NP + 3) / 4, NX = D * NU;
    double x[NX];
    double u[NU];
};

template <int D, int P>
__device__ __forceinline__ void gather_iso(const FormInputs &in, const int32_t *v, int j, IsoRaw<D, P> &r)
{
    using R = IsoRaw<D, P>;
    constexpr int NP = R::NP;
    auto node = [&](int it) { return it < NP ? v[it] : v[0]; };
#pragma unroll
    for (int t = 0; t < R::NX; ++t) {
        // item 4 t + j: node and component picked among the four candidates (static indices)
        const int it0 = 4 * t;
        const int32_t nd = sel4(j, node((it0 + 0) / D), node((it0 + 1) / D), node((it0 + 2) / D), node((it0 + 3) / D));
        const int cp = sel4(j, (it0 + 0) % D, (it0 + 1) % D, (it0 + 2) % D, (it0 + 3) % D);
        r.x[t] = in.coords[int64_t(cp) * in.n_nodes + nd];  // past the last item: a valid position, unused
    }
    if (in.cm.kind == 1 || in.cc.kind == 1) {
        const double *f = in.cm.kind == 1 ? in.cm.field : in.cc.field;
#pragma unroll
        for (int t = 0; t < R::NU; ++t) r.u[t] = f[sel4(j, node(4 * t), node(4 * t + 1), node(4 * t + 2), node(4 * t + 3))];
    }
}

// Per-lane setup of the isoparametric kernel (curved elements, Section 7:
// the geometry is evaluated at every quadrature node from all the element's
// node positions). For each node q = 4 m + j of this lane: B_q = sum_i
// (x_i - x_0) grad phi_i(q)^T (the gradients sum to zero, so this is B_q
// without the cancellation of absolute coordinates), its inverse and
// |det B_q|; then X_m[q] = w_q m_q |det B_q| and X_c[(q, g)] = w_q c_q
// |det B_q| A_q[g] with A_q = B_q^{-1} K_q B_q^{-T}. One rule serves both
// matrices (sDphi: [q][i][d] in LDS); a matrix that is not requested is not
// formed. The nodes are visited once, each node's position and field value
// read from the lane that gathered it and added into every B_q and u_h(q) of
// the lane. All 64 lanes must call this (cross-lane reads); live = false
// (past the last element) gives zeros. Returns false when a value is not
// finite or |det B_q| is not positive.
template <int D, int P, int NQ>
__device__ __forceinline__ bool lane_setup_iso(const FusedArgs &a, const IsoRaw<D, P> &r, bool live, int64_t pos,
                                               int64_t eid, int j, int c16, const double *sPhi, const double *sW,
                                               const double *sDphi, double *lm, double (*xc)[Shape<D, P>::NG])
{
    constexpr int NP = Shape<D, P>::NP, NG = Shape<D, P>::NG;
    using L = LaneQ<NQ, NQ, NG>;
    constexpr int MM = L::MM;
    static_assert(L::MM == L::MC, "one rule for both matrices");
    const FormInputs &in = a.in;
    const bool field = in.cm.kind == 1 || in.cc.kind == 1;
    const bool other = in.cc.kind == 1 && in.cm.kind == 1 && in.cc.field != in.cm.field;
    // group k of four nodes (k = 0, 1, ...) sits in registers [D k, D k + D) of x and k of u;
    // each pass reads group 0 and shifts the next one down, so every index is static
    using R = IsoRaw<D, P>;
    double rx[R::NX], ru[R::NU];
#pragma unroll
    for (int t = 0; t < R::NX; ++t) rx[t] = r.x[t];
#pragma unroll
    for (int t = 0; t < R::NU; ++t) ru[t] = r.u[t];
    double x0[D];
#pragma unroll
    for (int c = 0; c < D; ++c) x0[c] = __shfl(rx[c / 4], c16 + 16 * (c % 4), 64);
    double B[MM][D][D], uh[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        uh[m] = 0.0;
#pragma unroll
        for (int rr = 0; rr < D; ++rr)
#pragma unroll
            for (int c = 0; c < D; ++c) B[m][rr][c] = 0.0;
    }
    // q past the rule (lanes of the last node group): the last node's tables, results unused.
    // The loop over the groups stays rolled: one group's values are live at a time.
#pragma unroll 1
    for (int k = 0; k < R::NU; ++k) {
#pragma unroll
        for (int ip = 0; ip < 4; ++ip) {
            const int i = 4 * k + ip;
            if (i >= NP) break;  // wave-uniform
            double xr[D];
#pragma unroll
            for (int rr = 0; rr < D; ++rr) {
                const int it = ip * D + rr;  // item within the group
                xr[rr] = __shfl(rx[it / 4], c16 + 16 * (it % 4), 64) - x0[rr];
            }
            const double ui = field ? __shfl(ru[0], c16 + 16 * ip, 64) : 0.0;
#pragma unroll
            for (int m = 0; m < MM; ++m) {
                const int q = min(L::q(j, m), NQ - 1);
#pragma unroll
                for (int rr = 0; rr < D; ++rr)
#pragma unroll
                    for (int c = 0; c < D; ++c) B[m][rr][c] = fma(xr[rr], sDphi[(q * NP + i) * D + c], B[m][rr][c]);
                uh[m] = fma(sPhi[q * NP + i], ui, uh[m]);  // u_h(xhat_q) = phi_q^T u_e
            }
        }
#pragma unroll
        for (int t = 0; t + D < R::NX; ++t) rx[t] = rx[t + D];
#pragma unroll
        for (int t = 0; t + 1 < R::NU; ++t) ru[t] = ru[t + 1];
    }
    bool ok = true;
    auto coeff = [&](const CoeffDev &cf, int q, int m, bool second) -> double {
        if (cf.kind == 0) return cf.value;
        if (cf.kind == 2) return apply_law(cf, qe_value(cf, q, in.n_elem, eid));
        if (!second) return apply_law(cf, uh[m]);
        double u2 = 0.0;  // a second nodal field, read through the element's connectivity
#pragma unroll
        for (int i = 0; i < NP; ++i) u2 = fma(sPhi[q * NP + i], cf.field[a.tconn[i * in.n_elem + pos]], u2);
        return apply_law(cf, u2);
    };
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        const int q = L::q(j, m);
        lm[m] = 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) xc[m][g] = 0.0;
        if (!live || q >= NQ) continue;
        double I[D][D], adet;
        inverse_abs_det<D>(B[m], I, adet);
        if (a.M) {
            const double lam = sW[q] * coeff(in.cm, q, m, false) * adet;
            lm[m] = lam;
            ok &= isfinite(lam) && adet > 0.0;
        }
        if (a.C) {
            const double lam = sW[q] * coeff(in.cc, q, m, other) * adet;
            double Au[NG];
            if (a.Kq) {  // K_qe: a tensor per quadrature node
                double Kl[NG];
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    Kl[g] = a.Kq[(int64_t(q < a.nq_kq ? q : 0) * NG + g) * in.n_elem + eid];
                    ok &= isfinite(Kl[g]);
                }
                metric_from_inverse<D>(I, 1, Kl, Au);
            } else {
                metric_from_inverse<D>(I, in.aniso, in.K, Au);
            }
            ok &= isfinite(lam) && adet > 0.0;
#pragma unroll
            for (int g = 0; g < NG; ++g) xc[m][g] = lam * Au[g];
        }
    }
    return ok;
}

template <int PF>
struct FormTraits {
    using stage_t = float;  // reduced forms stage V in FP32; carries and the CSR accumulation stay FP64
    using qplain_t = float;
};
template <>
struct FormTraits<QXA_FP64> {
    using stage_t = double;
    using qplain_t = double;
};

// Warp-specialised matrix-core kernel (persistent). The workgroup walks its
// tiles with a two-buffer pipeline: waves 0-3 (producers, 16 elements each,
// T = 64; waves 0-7 for T = 16, see WideProducer) gather, set up and contract
// tile i into LDS buffer i % 2 while the other waves (consumers) reduce tile
// i-1 from the other buffer; one LDS-only barrier per tile separates the two.
// Producers issue only loads (the next tile's gathers and connectivity),
// consumers only output-unit loads and stores, so neither role waits on the
// other's memory traffic. Consumers walk a tile's units in chunks of CH
// rounds, loading chunk c+1 (or the next tile's first chunk) before storing
// chunk c; every round issues at least two stores (buffer stores that drop the
// lanes with nothing to write), so each wait for units leaves the stores
// behind them in flight.
// producer threads: 4 waves of one 16-element group each, or 8 waves for T = 16
constexpr int ws_producers(int T) { return T == 16 ? 512 : 256; }
// unit rounds per consumer chunk, sized so that one chunk holds all of a
// tile's output units on Kuhn meshes (the next tile's are then loaded a whole
// tile ahead): 2D P2 up to ~790 units per 64-element tile on 512 consumer
// threads, 2D P3 ~2,520, 3D P2 ~1,700, 3D P3 ~2,100 per 16-element tile
constexpr int ws_chunk(int D, int P) { return D == 2 ? (P == 3 ? 5 : 2) : 4; }
// consumer threads: 8 waves; 4 for the isoparametric kernel, whose producers
// need more than the 168 registers a lane has at three waves per SIMD
constexpr int ws_consumers(int T, bool iso = false) { return iso ? 256 : 512; }
constexpr int ws_threads(int T, bool iso = false) { return ws_producers(T) + ws_consumers(T, iso); }

// Producers of the T = 16 shape (3D P3: 210 symmetric rows, Q^T of 282 KB in
// FP64, read from global memory where it stays cached), eight waves:
// - the connectivity, vertex coordinates and nodal field of a tile are
//   gathered by all producer lanes together, one value per lane (tile g + 2),
//   and staged in LDS;
// - the weighted coefficients Lambda (one (element, node) per lane and pass)
//   and the metric W of each element are formed from the staged values
//   (tile g + 1) and staged in LDS, so no coefficient is evaluated twice;
// - each wave multiplies X^T (16 elements, read back from LDS) by the
//   Q^T fragments of its row blocks nb = wave and wave + 8 (tile g), the
//   fragments of the next chunk of k-steps being loaded during the current one.
// Every stage works on a different tile, so one barrier per tile orders them;
// two barriers before the loop fill the pipeline.
template <int D, int P, int NQM, int NQC, int PF, int T, bool MULTI>
struct WideProducer {
    using S = Shape<D, P>;
    using ST = typename FormTraits<PF>::stage_t;
    using CT = typename FormTraits<PF>::qplain_t;
    using MF = Mfma<CT>;
    static constexpr int NPT = 512;                    // producer threads
    static constexpr int NP = S::NP, NG = S::NG, NS = S::NS;
    static constexpr int DC = (D + 1) * D;             // staged vertex coordinates per element
    static constexpr int RAWN = DC + 2 * NP;           // + first and second nodal field
    static constexpr int NITEM = DC + NP;              // gather items per element
    static constexpr int NQL = NQM + NQC;              // staged Lambda per element
    static constexpr int NQP = (NQC + 3) / 4 * 4;
    static constexpr int KSM = (NQM + 3) / 4, MSC = NQP / 4;
    static constexpr int NSTEP = KSM + NG * MSC;       // k-steps: mass, then conductivity (k = g NQP + q)
    static constexpr int NB = (NS + 15) / 16;
    static constexpr int CHS = 6;                      // k-steps per chunk
    static constexpr int NCHK = (NSTEP + CHS - 1) / CHS;
    static constexpr int BUF_ELEMS = 2 * NS * (T + 1);
    static constexpr size_t lds_doubles = size_t(2) * T * (RAWN + NQL + NG);
    static_assert(T == 16 && NITEM <= NPT / T, "one gather item per producer lane");
    static_assert(NB <= 16, "two row blocks per producer wave");

    const JobTable &jt;
    const TileWalk &walk;
    ST *sV;
    const double *sPhiM, *sPhiC, *sWM, *sWC;
    double *sRaw, *sLam, *sA;  // [2][T][RAWN], [2][T][NQL], [2][T][NG]
    int tid, lane, wave, ge, gk;  // gather item of this lane: element ge, item gk

    __device__ WideProducer(const JobTable &jt_, const TileWalk &w, ST *sV_, const double *pm, const double *pc,
                            const double *wm, const double *wc, double *wide, int tid_)
        : jt(jt_), walk(w), sV(sV_), sPhiM(pm), sPhiC(pc), sWM(wm), sWC(wc), sRaw(wide),
          sLam(wide + 2 * T * RAWN), sA(wide + 2 * T * (RAWN + NQL)), tid(tid_), lane(tid_ & 63), wave(tid_ >> 6),
          ge(tid_ % T), gk(tid_ / T)
    {
    }

    // this lane's connectivity entry of tile g (node gk, or the vertex of coordinate item gk)
    __device__ int32_t conn_of(int64_t g) const
    {
        int64_t lt;
        const FusedArgs b = args_of<MULTI>(jt, job_of<MULTI>(jt, g, lt));
        const int64_t p = min(lt * T + ge, b.in.n_elem - 1);
        const int ci = gk < NP ? gk : (gk < NITEM ? (gk - NP) / D : 0);
        return b.tconn[ci * b.in.n_elem + p];
    }
    __device__ void gather(int64_t g, int32_t node, double &d0, double &d1) const
    {
        int64_t lt;
        const FusedArgs b = args_of<MULTI>(jt, job_of<MULTI>(jt, g, lt));
        const CoeffDev &cm = b.in.cm, &cc = b.in.cc;
        if (gk < NP) {
            if (cm.kind == 1 || cc.kind == 1) d0 = (cm.kind == 1 ? cm.field : cc.field)[node];
            if (cm.kind == 1 && cc.kind == 1 && cc.field != cm.field) d1 = cc.field[node];
        } else if (gk < NITEM) {
            d0 = b.in.coords[((gk - NP) % D) * b.in.n_nodes + node];
        }
    }
    __device__ void put_raw(int buf, double d0, double d1) const
    {
        double *r = sRaw + (buf * T + ge) * RAWN;
        if (gk < NP) {
            r[DC + gk] = d0;
            r[DC + NP + gk] = d1;
        } else if (gk < NITEM) {
            r[gk - NP] = d0;
        }
    }

    // Lambda (and W) of tile g from its staged raw values, into buffer buf
    __device__ void lambda(int64_t g, int buf) const
    {
        int64_t lt;
        const FusedArgs b = args_of<MULTI>(jt, job_of<MULTI>(jt, g, lt));
        const FormInputs &in = b.in;
        const bool other = in.cc.kind == 1 && in.cm.kind == 1 && in.cc.field != in.cm.field;
        bool ok = true;
        for (int id = tid; id < T * (NQL + 1); id += NPT) {
            const int e = id % T, which = id / T;
            const int64_t p = lt * T + e;
            const double *r = sRaw + (buf * T + e) * RAWN;
            double x[D + 1][D];
#pragma unroll
            for (int v = 0; v <= D; ++v)
#pragma unroll
                for (int c = 0; c < D; ++c) x[v][c] = r[v * D + c];
            double babs, A[NG];
            geometry_from<D>(x, babs, A, in.aniso, in.K);
            const bool live = p < in.n_elem;
            if (which == NQL) {
#pragma unroll
                for (int gg = 0; gg < NG; ++gg) sA[(buf * T + e) * NG + gg] = live ? A[gg] : 0.0;
                continue;
            }
            const bool mass = which < NQM;
            const int q = mass ? which : which - NQM;
            const CoeffDev &cf = mass ? in.cm : in.cc;
            double v = 0.0;
            if (live) {
                double s;
                if (cf.kind == 0) {
                    s = cf.value;
                } else if (cf.kind == 1) {
                    const double *phi = mass ? sPhiM : sPhiC;
                    const double *u = r + DC + (!mass && other ? NP : 0);
                    double uh = 0.0;  // u_h(xhat_q) = phi_q^T u_e
#pragma unroll
                    for (int i = 0; i < NP; ++i) uh = fma(phi[q * NP + i], u[i], uh);
                    s = apply_law(cf, uh);
                } else {
                    const int64_t eid = b.elem_order[p];
                    s = apply_law(cf, qe_value(cf, q, in.n_elem, eid));
                }
                v = (mass ? sWM : sWC)[q] * s * babs;
                ok &= isfinite(v);
            }
            sLam[(buf * T + e) * NQL + which] = v;
        }
        if (!ok) atomicOr(in.flags, 1);
    }

    // V_m^T = X_m^T Q_m^T and V_c^T = X_c^T Q_c^T of tile g (Lambda, W in buffer
    // buf) for row blocks wave and wave + 8, into V buffer buf
    __device__ void contract(const CT *gQ, int buf) const
    {
        const int j = lane >> 4, c16 = lane & 15;
        const double *lam = sLam + (buf * T + c16) * NQL;
        double lm[KSM], lc[MSC], A[NG];
#pragma unroll
        for (int m = 0; m < KSM; ++m) lm[m] = 4 * m + j < NQM ? lam[4 * m + j] : 0.0;
#pragma unroll
        for (int m = 0; m < MSC; ++m) lc[m] = 4 * m + j < NQC ? lam[NQM + 4 * m + j] : 0.0;
#pragma unroll
        for (int gg = 0; gg < NG; ++gg) A[gg] = sA[(buf * T + c16) * NG + gg];
        // row blocks wave and wave + 8; a second block past the last one (waves 6
        // and 7 of 14 blocks) repeats the last block and is not stored, which
        // keeps the code free of branches and gives every SIMD four blocks
        const int w = __builtin_amdgcn_readfirstlane(wave);
        const int nb0 = w, nb1 = w + 8 < NB ? w + 8 : NB - 1;
        typename MF::acc_t am[2], ac[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) am[u] = ac[u] = typename MF::acc_t{0, 0, 0, 0};
        // fragments through a buffer resource: one lane offset per block, the
        // k-step in the scalar offset
        const __amdgpu_buffer_rsrc_t rq =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<CT *>(gQ), 0, int(sizeof(CT) * NSTEP * NB * 64), 0x00020000);
        const int o0 = int(sizeof(CT)) * (nb0 * 64 + lane), o1 = int(sizeof(CT)) * (nb1 * 64 + lane);
        auto ldq = [&](int off, int t) -> CT {
            const int so = int(sizeof(CT)) * t * NB * 64;
            if constexpr (sizeof(CT) == 8)
                return __builtin_bit_cast(CT, __builtin_amdgcn_raw_buffer_load_b64(rq, off, so, 0));
            else
                return __builtin_bit_cast(CT, __builtin_amdgcn_raw_buffer_load_b32(rq, off, so, 0));
        };
        CT cur[CHS][2], nxt[CHS][2];
        auto load = [&](int c, CT (&f)[CHS][2]) {
#pragma unroll
            for (int tt = 0; tt < CHS; ++tt) {
                const int t = c * CHS + tt;
                f[tt][0] = t < NSTEP ? ldq(o0, t) : CT(0);
                f[tt][1] = t < NSTEP ? ldq(o1, t) : CT(0);
            }
        };
        load(0, cur);
#pragma unroll
        for (int c = 0; c < NCHK; ++c) {
            if (c + 1 < NCHK) load(c + 1, nxt);
#pragma unroll
            for (int tt = 0; tt < CHS; ++tt) {
                const int t = c * CHS + tt;
                if (t >= NSTEP) continue;
                if (t < KSM) {  // mass: k = q
                    const CT x = CT(lm[t]);
                    am[0] = MF::step(x, cur[tt][0], am[0]);
                    am[1] = MF::step(x, cur[tt][1], am[1]);
                } else {  // conductivity: k = g NQP + q
                    const int tc = t - KSM;
                    const CT x = CT(lc[tc % MSC] * A[tc / MSC]);
                    ac[0] = MF::step(x, cur[tt][0], ac[0]);
                    ac[1] = MF::step(x, cur[tt][1], ac[1]);
                }
            }
            if (c + 1 < NCHK) {
#pragma unroll
                for (int tt = 0; tt < CHS; ++tt) {
                    cur[tt][0] = nxt[tt][0];
                    cur[tt][1] = nxt[tt][1];
                }
            }
        }
        ST *bV = sV + buf * BUF_ELEMS;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int s = 16 * (u ? nb1 : nb0) + c16;
            if (s < NS && (u == 0 || w + 8 < NB))
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int o = 2 * (s * (T + 1) + MF::row(lane, r));
                    bV[o] = ST(am[u][r]);
                    bV[o + 1] = ST(ac[u][r]);
                }
        }
    }

    __device__ void run(const CT *gQ) const
    {
        const int64_t step = walk.step;
        int64_t g = walk.t;  // every workgroup of a persistent launch has at least one tile
        int32_t cn;
        {
            const int32_t c0 = conn_of(g);
            const int32_t c1 = walk.valid(g + step) ? conn_of(g + step) : 0;
            double d0 = 0.0, d1 = 0.0, e0 = 0.0, e1 = 0.0;
            gather(g, c0, d0, d1);
            if (walk.valid(g + step)) gather(g + step, c1, e0, e1);
            cn = walk.valid(g + 2 * step) ? conn_of(g + 2 * step) : 0;
            put_raw(0, d0, d1);
            lds_barrier();  // raw values of the first tile staged
            lambda(g, 0);
            if (walk.valid(g + step)) put_raw(1, e0, e1);
            lds_barrier();  // Lambda of the first tile, raw values of the second staged
        }
        for (int it = 0; walk.valid(g); g += step, ++it) {
            const int64_t g1 = g + step, g2 = g + 2 * step, g3 = g + 3 * step;
            double r0 = 0.0, r1 = 0.0;
            if (walk.valid(g2)) gather(g2, cn, r0, r1);  // its connectivity was loaded one tile ago
            if (walk.valid(g3)) cn = conn_of(g3);
            contract(gQ, it & 1);
            if (walk.valid(g1)) lambda(g1, (it + 1) & 1);
            if (walk.valid(g2)) put_raw(it & 1, r0, r1);
            lds_barrier();  // tile g staged; buffers of tile g - 1 free
        }
    }
};
constexpr int kWidePrologueBarriers = 2;

// LDS of the kernel: staged V (two buffers, both matrices), Q^T fragments,
// basis values and weights of both rules (q-major). With T = 16 (wide shapes:
// 3D P3) Q^T (too large for LDS) is read from global memory, where it stays
// cached, and the producers' staged raw values, Lambda and W follow.
template <int D, int P, int NQM, int NQC, int PF, int T, bool ISO = false>
struct WsLds {
    using ST = typename FormTraits<PF>::stage_t;
    static constexpr bool QLDS = T != 16;
    static constexpr int NP = Shape<D, P>::NP, NS = Shape<D, P>::NS;
    static constexpr size_t v_bytes = ((4 * sizeof(ST) * NS * (T + 1) + 15) / 16) * 16;
    static constexpr size_t tab_doubles = size_t(NQM + NQC) * NP + NQM + NQC;
    static constexpr size_t wide_doubles =
        QLDS ? 0 : size_t(2) * T * ((D + 1) * D + 2 * NP + NQM + NQC + Shape<D, P>::NG);
    static constexpr size_t iso_doubles = ISO ? size_t(NQC) * NP * D : 0;  // reference gradients [q][i][d]
    static __host__ __device__ size_t bytes(int64_t qfrag_vec16)
    {
        return v_bytes + (QLDS ? size_t(qfrag_vec16) * 16 : 0) + (tab_doubles + wide_doubles + iso_doubles) * 8;
    }
};

// ISO: the isoparametric assembly (X per quadrature node, lane_setup_iso) with
// the same contraction and reduction; single assemblies in FP64 only.
template <int D, int P, int NQM, int NQC, int PF, int T, bool MULTI, bool ISO = false>
__global__ __launch_bounds__(ws_threads(T, ISO)) void fused_ws_kernel(JobTable jt)
{
    constexpr int NPT = ws_producers(T);
    static_assert(T == 16 * (NPT / 64) || T == 16, "one 16-element group per producer wave, or T = 16");
    using S = Shape<D, P>;
    using ST = typename FormTraits<PF>::stage_t;
    using L = LaneQ<NQM, NQC, S::NG>;
    using LDS = WsLds<D, P, NQM, NQC, PF, T, ISO>;
    constexpr bool SPLIT = PF >= QXA_F16X2;
    constexpr bool QLDS = LDS::QLDS;  // else: T = 16, WideProducer, Q^T from global memory
    static_assert(QLDS || !SPLIT, "split forms need Q^T in LDS");
    static_assert(!ISO || (QLDS && PF == QXA_FP64 && !MULTI && NQM == NQC), "isoparametric kernel: one rule, FP64");
    constexpr int NB = (S::NS + 15) / 16;
    constexpr int KM = NQM, KC = L::NQP * S::NG;  // conductivity K order: k = g * NQP + q
    constexpr int BUF_ELEMS = 2 * S::NS * (T + 1);  // one buffer: [NS][T + 1] pairs (V_m, V_c)
    constexpr int NCT = ws_consumers(T, ISO);
    constexpr int CH = ws_chunk(D, P) * (512 / NCT);  // a tile's units in one chunk either way
    constexpr int NTH = ws_threads(T, ISO);
    extern __shared__ __align__(16) unsigned char smem[];
    ST *sV = reinterpret_cast<ST *>(smem);  // [2 buffers][NS][T + 1][V_m, V_c]
    unsigned char *sQraw = smem + LDS::v_bytes;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const FusedArgs a0 = args_of<MULTI>(jt, 0);  // tables are shared by every job of the launch
    double *sPhiM = reinterpret_cast<double *>(sQraw + (QLDS ? size_t(a0.qfrag_vec16) * 16 : 0));
    double *sPhiC = sPhiM + NQM * S::NP, *sWM = sPhiC + NQC * S::NP, *sWC = sWM + NQM;
    {
        const uint4 *gq = reinterpret_cast<const uint4 *>(a0.Qfrag);
        uint4 *dq = reinterpret_cast<uint4 *>(sQraw);
        if (QLDS)
            for (int64_t k = tid; k < a0.qfrag_vec16; k += NTH) dq[k] = gq[k];
        for (int k = tid; k < NQM * S::NP; k += NTH) {
            const int q = k / S::NP, i = k % S::NP;
            sPhiM[k] = a0.in.phi_m[i * NQM + q];
        }
        for (int k = tid; k < NQC * S::NP; k += NTH) {
            const int q = k / S::NP, i = k % S::NP;
            sPhiC[k] = a0.in.phi_c[i * NQC + q];
        }
        for (int k = tid; k < NQM; k += NTH) sWM[k] = a0.in.w_m[k];
        for (int k = tid; k < NQC; k += NTH) sWC[k] = a0.in.w_c[k];
        if constexpr (ISO)
            for (int k = tid; k < NQC * S::NP * D; k += NTH) sWC[NQC + k] = a0.dphi[k];
    }
    // a zero pair in the (never written) padding column of row 0 of each buffer
    if (tid < 4) sV[(tid >> 1) * BUF_ELEMS + 2 * T + (tid & 1)] = ST(0);
    const TileWalk walk = chain_walk(jt);
    lds_barrier();
    if (tid < NPT) {
      if constexpr (!QLDS) {
        static_assert(WideProducer<D, P, NQM, NQC, PF, T, MULTI>::lds_doubles == LDS::wide_doubles, "LDS layout");
        const WideProducer<D, P, NQM, NQC, PF, T, MULTI> wp(jt, walk, sV, sPhiM, sPhiC, sWM, sWC, sWC + NQC, tid);
        wp.run(reinterpret_cast<const typename FormTraits<PF>::qplain_t *>(a0.Qfrag));
      } else {
        const int j = lane >> 4, c16 = lane & 15;
        int32_t v[S::NP];
        std::conditional_t<ISO, IsoRaw<D, P>, RawElem<D, P>> raw;
        auto load_conn = [&](int64_t g) {
            int64_t lt;
            const FusedArgs b = args_of<MULTI>(jt, job_of<MULTI>(jt, g, lt));
            // lanes past the last element read the last element (unconditional loads keep
            // the loads of one call in flight together)
            const int64_t pp = min(lt * T + 16 * wave + c16, b.in.n_elem - 1);
#pragma unroll
            for (int i = 0; i < S::NP; ++i) v[i] = b.tconn[i * b.in.n_elem + pp];
        };
        auto gather = [&](int64_t g) {
            int64_t lt;
            const FusedArgs b = args_of<MULTI>(jt, job_of<MULTI>(jt, g, lt));
            if constexpr (ISO)
                gather_iso<D, P>(b.in, v, j, raw);
            else
                gather_raw<D, P>(b.in, v, raw);
        };
        int64_t g = walk.t;  // every workgroup of a persistent launch has at least one tile
        load_conn(g);
        gather(g);
        if (walk.valid(g + walk.step)) load_conn(g + walk.step);
        for (int it = 0; walk.valid(g); g += walk.step, ++it) {
            int64_t tile;
            const FusedArgs a = args_of<MULTI>(jt, job_of<MULTI>(jt, g, tile));
            const int64_t ne = a.in.n_elem;
            const int64_t p = tile * T + 16 * wave + c16;  // this lane's element (4 lanes each)
            double A[S::NG], lm[L::MM], lc[L::MC];
            double xiso[ISO ? L::MC : 1][S::NG];  // X_c of the isoparametric kernel
            if constexpr (ISO) {
                const bool live = p < ne;
                const bool by_id = live && (a.in.cm.kind == 2 || a.in.cc.kind == 2 || a.Kq);
                const int64_t eid = by_id ? int64_t(a.elem_order[p]) : p;
                if (!lane_setup_iso<D, P, NQM>(a, raw, live, p, eid, j, c16, sPhiM, sWM, sWC + NQC, lm, xiso))
                    atomicOr(a.in.flags, 1);
            } else if (p < ne) {
                const int64_t eid = (a.in.cm.kind == 2 || a.in.cc.kind == 2) ? int64_t(a.elem_order[p]) : p;
                if (!lane_setup<D, P, NQM, NQC>(a.in, raw, a.tconn, p, eid, j, sPhiM, sPhiC, sWM, sWC, A, lm, lc))
                    atomicOr(a.in.flags, 1);
            } else {
#pragma unroll
                for (int q = 0; q < S::NG; ++q) A[q] = 0.0;
#pragma unroll
                for (int m = 0; m < L::MM; ++m) lm[m] = 0.0;
#pragma unroll
                for (int m = 0; m < L::MC; ++m) lc[m] = 0.0;
            }
            const int64_t gn = g + walk.step;
            if (walk.valid(gn)) {
                gather(gn);  // its connectivity was loaded one tile ago
                if (walk.valid(gn + walk.step)) load_conn(gn + walk.step);
            }
            ST *bVm = sV + (it & 1) * BUF_ELEMS, *bVc = bVm + 1;
            // V_m^T = X_m^T Q_m^T with X_m = Lambda_m; V_c^T = X_c^T Q_c^T with X_c = Lambda_c (.) W
            if constexpr (!SPLIT) {
                using CT = typename FormTraits<PF>::qplain_t;
                const CT *q = reinterpret_cast<const CT *>(sQraw);
                // k = 4 ks + j: mass node q = k, conductivity (g, q) = divmod(4 ks, NQP) + (0, j)
                auto xm = [&](int ks) { return lm[ks]; };
                auto xc = [&](int ks) {
                    if constexpr (ISO)
                        return xiso[((4 * ks) % L::NQP) / 4][(4 * ks) / L::NQP];
                    else
                        return lc[((4 * ks) % L::NQP) / 4] * A[(4 * ks) / L::NQP];
                };
                // a matrix that is not requested is not formed (its staged values are never stored)
                if (a.M) contract_group_plain<CT, KM, NB, S::NS, T, ST, 2>(q, xm, bVm, lane, 16 * wave);
                if (a.C)
                    contract_group_plain<CT, KC, NB, S::NS, T, ST, 2>(q + ((KM + 3) / 4) * NB * 64, xc, bVc, lane,
                                                                     16 * wave);
            } else {
                const uint4 *q = reinterpret_cast<const uint4 *>(sQraw);
                constexpr int NC = Split<PF>::NC;
                // k = 32 ks + 8 j + t holds node q = 4 m + j, m = QPS ks + t / G, component t % G
                auto xm = [&](int ks, int t) {
                    const int m = L::QPSM * ks + t;
                    return m < L::MM ? lm[m] : 0.0;
                };
                auto xc = [&](int ks, int t) {
                    const int u = t / S::NG, g = t % S::NG, m = L::QPSC * ks + u;
                    return u < L::QPSC && m < L::MC ? lc[m] * A[g] : 0.0;
                };
                if (a.M)
                    contract_group_split<PF, 32 * L::KSM, NB, S::NS, T, ST, 2>(q, xm, bVm, lane, 16 * wave, a.qinv_m);
                if (a.C)
                    contract_group_split<PF, 32 * L::KSC, NB, S::NS, T, ST, 2>(q + NC * L::KSM * NB * 64, xc, bVc,
                                                                              lane, 16 * wave, a.qinv_c);
            }
            lds_barrier();  // tile i staged; the consumers are done with buffer (i + 1) % 2
        }
      }
    } else {
        double2 *carry = reinterpret_cast<double2 *>(smem + ((LDS::bytes(a0.qfrag_vec16) + 15) & ~size_t(15)));
        // one barrier per tile: the producers have staged tile k, and the
        // consumers are done with the buffer of tile k - 1 (and its carries)
        auto on_tile = [&](int64_t k) -> const ST * {
            if constexpr (!QLDS)  // the wide producers' pipeline fill
                if (k == 0)
                    for (int b = 0; b < kWidePrologueBarriers; ++b) lds_barrier();
            lds_barrier();
            return sV + (k & 1) * BUF_ELEMS;
        };
        const uint32_t cb = uint32_t(carry_base(S::NS, T));
        if (jt.buf_stores)
            consume_units<ST, MULTI, true, CH, NCT>(jt, walk, tid - NPT, carry, cb, uint32_t(T), on_tile);
        else
            consume_units<ST, MULTI, false, CH, NCT>(jt, walk, tid - NPT, carry, cb, uint32_t(T), on_tile);
    }
}

#ifndef QXA_FUSED_PADDED

// Shared slots: one thread per shared upper slot sums its partials (stored
// contiguously, ascending tile order) and writes the slot and its mirror.
__global__ __launch_bounds__(256) void fixup_kernel(FixupTable ft)
{
    // XCD-aware: the blocks of one XCD take a contiguous range of shared slots,
    // so that stores into the same CSR rows meet in the same L2
    int64_t f = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
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
    const int64_t lo = a.part_ptr[f], hi = a.part_ptr[f + 1];
    const int32_t t = a.fix_target[f], tm = a.fix_mirror[f];
    const double2 *pp = reinterpret_cast<const double2 *>(a.part);
    const double2 first = pp[lo];
    double m = first.x, c = first.y;
    for (int64_t q = lo + 1; q < hi; ++q) {
        const double2 v = pp[q];
        m += v.x;
        c += v.y;
    }
    if (a.M) {
        a.M[t] = m;
        a.M[tm] = m;
    }
    if (a.C) {
        a.C[t] = c;
        a.C[tm] = c;
    }
}
#endif

#ifndef QXA_FUSED_PADDED
bool fused_uses_mfma(int D, int P, int nqm, int nqc) { return mfma_variant(D, P, nqm, nqc); }
#endif

// Resident workgroups for a persistent launch: CUs x workgroups per CU.
template <class K>
static unsigned persistent_grid(K kernel, int block, size_t lds, int64_t n_chains)
{
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    (void)hipGetLastError();  // a failed occupancy query must not be reported as a launch error
    return unsigned(std::min<int64_t>(n_chains, int64_t(cus) * per_cu));
}

// LDS bytes of a launch: the kernel's layout, then the carry entries (16 bytes each).
static size_t with_carries(size_t bytes, int carry_cap) { return ((bytes + 15) & ~size_t(15)) + 16 * size_t(carry_cap); }

constexpr int kMaxCarries = 4096;
constexpr int kMinCarries = 1024;
constexpr int kMinRunCarries = 128;

template <int D, int P>
static size_t p1_lds_bytes()
{
    return size_t(tile_size(D, P) + 1) * Shape<D, P>::NS * 16;
}

// LDS bytes of the matrix-core kernel of a shape (its largest precision form);
// false if the rule sizes are not among this file's.
bool QXA_PART(fused_base_lds)(int D, int P, int nqm, int nqc, const int64_t (&qv16)[5], size_t &base)
{
    base = 0;
#define X(d, p, m, c)                                                                                              \
    if (D == d && P == p && nqm == m && nqc == c) {                                                               \
        constexpr int T = tile_size(d, p);                                                                        \
        if constexpr (mfma_variant(d, p, m, c)) {                                                                         \
            base = std::max(WsLds<d, p, m, c, QXA_FP64, T>::bytes(qv16[QXA_FP64]),                                \
                            WsLds<d, p, m, c, QXA_FP32, T>::bytes(qv16[QXA_FP32]));                               \
            if constexpr (split_ok(d, p, m, c)) {                                                                 \
                base = std::max(base, WsLds<d, p, m, c, QXA_F16X2, T>::bytes(qv16[QXA_F16X2]));                   \
                base = std::max(base, WsLds<d, p, m, c, QXA_BF16X2, T>::bytes(qv16[QXA_BF16X2]));                 \
                base = std::max(base, WsLds<d, p, m, c, QXA_BF16X3, T>::bytes(qv16[QXA_BF16X3]));                 \
            }                                                                                                     \
        }                                                                                                         \
        return true;                                                                                              \
    }
    QXA_FUSED_CASES(X)
#undef X
    return false;
}

#ifndef QXA_FUSED_PADDED
// Shapes of the one-pass isoparametric kernel: Q^T staged in LDS, one rule for
// both matrices (the rule sizes of the default rules).
#define QXA_ISO_CASES(X) X(2, 2, 6, 6) X(2, 3, 12, 12) X(3, 2, 11, 11)

// LDS bytes of the isoparametric kernel of a shape (0 if it has none)
static size_t fused_iso_lds(int D, int P, int nqm, int nqc, int64_t qfrag_vec16)
{
#define X(d, p, m, c)                                                                                  \
    if (D == d && P == p && nqm == m && nqc == c) {                                                   \
        static_assert(mfma_variant(d, p, m, c) && tile_size(d, p) != 16, "Q^T staged in LDS");        \
        return WsLds<d, p, m, c, QXA_FP64, tile_size(d, p), true>::bytes(qfrag_vec16);                \
    }
    QXA_ISO_CASES(X)
#undef X
    return 0;
}

bool fused_base_lds_padded(int D, int P, int nqm, int nqc, const int64_t (&qv16)[5], size_t &base);
hipError_t launch_fused_padded(const JobTable &jt, int D, int P, int nqm, int nqc, int precision, hipStream_t st,
                               bool &found);

TileParams fused_tile_params(int D, int P, int nqm, int nqc, int cus, size_t lds_max, const int64_t (&qv16)[5])
{
    TileParams tp;
    tp.T = tile_size(D, P);
    tp.pair_units = true;
    if (!mfma_variant(D, P, nqm, nqc)) {  // the vector-ALU variant: a chain per tile, no carries
        tp.chains = int64_t(1) << 40;
        tp.carry_cap = 0;
        return tp;
    }
    size_t base = 0;
    if (!fused_base_lds_tuned(D, P, nqm, nqc, qv16, base)) fused_base_lds_padded(D, P, nqm, nqc, qv16, base);
    // the carry entries leave room for the isoparametric kernel's reference gradients, so
    // that a plan serves both assemblies (2D P3: 1,296 entries instead of 1,408; its plans
    // use at most about 900)
    base = std::max(base, fused_iso_lds(D, P, nqm, nqc, qv16[QXA_FP64]));
    const size_t room = lds_max > with_carries(base, 0) ? lds_max - with_carries(base, 0) : 0;
    tp.carry_cap = int(std::min<size_t>(kMaxCarries, room / 16) / 16 * 16);
    tp.chains = int64_t(std::max(1, cus));  // one workgroup per CU
    if (tp.carry_cap < kMinCarries) {
        // too few carry entries for long chains (3D P2: 272, 3D P3: 896): chains of short
        // runs, the workgroups of one XCD on neighbouring runs at the same time
        // (build_tile_plan), the slots a run's tiles share through carry entries
        if (tp.carry_cap >= kMinRunCarries) {
            tp.run_len = tp.carry_cap >= 512 ? 4 : 2;
        } else {  // tiles side by side, every shared slot through a partial
            tp.carry_cap = 0;
            tp.chains = int64_t(1) << 40;
        }
    }
    return tp;
}
#endif

// The launch of this file's rule sizes (found = false for others).
hipError_t QXA_PART(launch_fused)(const JobTable &jt, int D, int P, int nqm, int nqc, int precision, hipStream_t st,
                                  bool &found)
{
    const int64_t n_tiles = jt.n_tiles;
    found = true;
    const FusedArgs &a = jt.one;  // the first job (Q^T fragment size and carry entries are shared by all jobs)
#define QXA_LAUNCH_MFMA(d, p, m, c, PF, MULTI)                                                            \
    {                                                                                                     \
        constexpr int T = tile_size(d, p);                                                                \
        const size_t lds = with_carries(WsLds<d, p, m, c, PF, T>::bytes(a.qfrag_vec16), a.carry_cap);    \
        auto k = fused_ws_kernel<d, p, m, c, PF, T, MULTI>;                                               \
        k<<<persistent_grid(k, ws_threads(T), lds, jt.n_chains), ws_threads(T), lds, st>>>(jt);           \
    }
#define X(d, p, m, c)                                                                                      \
    if (D == d && P == p && nqm == m && nqc == c) {                                                        \
        constexpr int T = tile_size(d, p);                                                                 \
        const bool multi = jt.n_jobs > 0;                                                                  \
        if (multi && precision != QXA_FP64 && precision != QXA_FP32) return hipErrorInvalidValue;          \
        if constexpr (mfma_variant(d, p, m, c)) {                                                                  \
            switch (precision * 2 + int(multi)) {                                                          \
            case 2 * QXA_FP64: QXA_LAUNCH_MFMA(d, p, m, c, QXA_FP64, false) break;                         \
            case 2 * QXA_FP64 + 1: QXA_LAUNCH_MFMA(d, p, m, c, QXA_FP64, true) break;                      \
            case 2 * QXA_FP32: QXA_LAUNCH_MFMA(d, p, m, c, QXA_FP32, false) break;                         \
            case 2 * QXA_FP32 + 1: QXA_LAUNCH_MFMA(d, p, m, c, QXA_FP32, true) break;                      \
            case 2 * QXA_F16X2:                                                                                \
                if constexpr (split_ok(d, p, m, c)) QXA_LAUNCH_MFMA(d, p, m, c, QXA_F16X2, false)              \
                else return hipErrorInvalidValue;                                                              \
                break;                                                                                         \
            case 2 * QXA_BF16X2:                                                                               \
                if constexpr (split_ok(d, p, m, c)) QXA_LAUNCH_MFMA(d, p, m, c, QXA_BF16X2, false)             \
                else return hipErrorInvalidValue;                                                              \
                break;                                                                                         \
            case 2 * QXA_BF16X3:                                                                               \
                if constexpr (split_ok(d, p, m, c)) QXA_LAUNCH_MFMA(d, p, m, c, QXA_BF16X3, false)             \
                else return hipErrorInvalidValue;                                                              \
                break;                                                                                         \
            default: return hipErrorInvalidValue;                                                          \
            }                                                                                              \
        } else {                                                                                           \
            if (precision != QXA_FP64 && precision != QXA_FP32) return hipErrorInvalidValue;               \
            const size_t lds = p1_lds_bytes<d, p>();                                                       \
            if (precision == QXA_FP32) {                                                                   \
                if (multi) {                                                                               \
                    auto k = fused_kernel<d, p, m, c, float, T, true>;                                     \
                    k<<<unsigned(n_tiles), T, lds, st>>>(jt);                        \
                } else {                                                                                   \
                    auto k = fused_kernel<d, p, m, c, float, T, false>;                                    \
                    k<<<unsigned(n_tiles), T, lds, st>>>(jt);                        \
                }                                                                                          \
            } else {                                                                                       \
                if (multi) {                                                                               \
                    auto k = fused_kernel<d, p, m, c, double, T, true>;                                    \
                    k<<<unsigned(n_tiles), T, lds, st>>>(jt);                        \
                } else {                                                                                   \
                    auto k = fused_kernel<d, p, m, c, double, T, false>;                                   \
                    k<<<unsigned(n_tiles), T, lds, st>>>(jt);                        \
                }                                                                                          \
            }                                                                                              \
        }                                                                                                  \
        return hipGetLastError();                                                                          \
    }
    QXA_FUSED_CASES(X)
#undef X
#undef QXA_LAUNCH_MFMA
    found = false;
    return hipErrorInvalidValue;
}

#ifndef QXA_FUSED_PADDED
hipError_t launch_fused(const JobTable &jt, int D, int P, int nqm, int nqc, int precision, hipStream_t st)
{
    if (jt.n_tiles == 0 || jt.n_chains == 0) return hipSuccess;
    bool found = false;
    const hipError_t e = launch_fused_tuned(jt, D, P, nqm, nqc, precision, st, found);
    if (found) return e;
    return launch_fused_padded(jt, D, P, nqm, nqc, precision, st, found);
}
#endif

#ifndef QXA_FUSED_PADDED
// Reduction of local matrices formed elsewhere (the isoparametric path): the
// pair-major blocks of 64 tile positions [block][pair][64] of V_m and V_c are
// staged per tile into the LDS layout of the fused kernels ([NS][T + 1] pairs,
// two buffers) and reduced by the same consumer code with the plan's units,
// chains and carry entries. Every thread loads its share of the next tile into
// registers while the current one is reduced.
constexpr int kStageThreads = 512;

template <int D, int P>
__global__ __launch_bounds__(kStageThreads) void staged_reduce_kernel(JobTable jt, const double *Tm, const double *Tc)
{
    constexpr int NS = Shape<D, P>::NS, T = tile_size(D, P), BUF = NS * (T + 1);
    constexpr int CH = P == 1 ? 2 : ws_chunk(D, P);
    constexpr int PER = (NS * T + kStageThreads - 1) / kStageThreads;  // values per thread and tile
    extern __shared__ __align__(16) double2 sStage[];                  // [2][NS][T + 1], then the carries
    double2 *carry = sStage + 2 * BUF;
    const int tid = threadIdx.x;
    const int64_t ne = jt.one.in.n_elem;
    if (tid == 0) {
        sStage[T] = make_double2(0.0, 0.0);  // the zero pair of each buffer
        sStage[BUF + T] = make_double2(0.0, 0.0);
    }
    const TileWalk walk = chain_walk(jt);
    double2 reg[PER];
    auto load = [&](int64_t tile) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int idx = tid + k * kStageThreads, s = idx / T, i = idx % T;
            const int64_t p = tile * T + i;
            double2 v = make_double2(0.0, 0.0);
            if (idx < NS * T && p < ne) {
                const size_t o = (size_t(p / 64) * NS + s) * 64 + size_t(p % 64);
                v = make_double2(Tm ? Tm[o] : 0.0, Tc ? Tc[o] : 0.0);
            }
            reg[k] = v;
        }
    };
    if (walk.valid(walk.t)) load(walk.t);
    // tile k of the walk: stage it (its values arrived during tile k - 1), one barrier,
    // then ask for tile k + 1's
    auto on_tile = [&](int64_t k) -> const double * {
        double2 *b = sStage + (k & 1) * BUF;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int idx = tid + j * kStageThreads;
            if (idx < NS * T) b[(idx / T) * (T + 1) + idx % T] = reg[j];
        }
        lds_barrier();
        const int64_t gn = walk.t + (k + 1) * walk.step;
        if (walk.valid(gn)) load(gn);
        return reinterpret_cast<const double *>(b);
    };
    const uint32_t cb = uint32_t(carry_base(NS, T));
    if (jt.buf_stores)
        consume_units<double, false, true, CH, kStageThreads>(jt, walk, tid, carry, cb, uint32_t(T), on_tile);
    else
        consume_units<double, false, false, CH, kStageThreads>(jt, walk, tid, carry, cb, uint32_t(T), on_tile);
}

hipError_t launch_staged_reduce(const JobTable &jt, int D, int P, const double *Tm, const double *Tc, hipStream_t st)
{
    if (jt.n_tiles == 0 || jt.n_chains == 0) return hipSuccess;
#define QXA_STAGED(d, p)                                                                                \
    if (D == d && P == p) {                                                                             \
        constexpr int NS = Shape<d, p>::NS, T = tile_size(d, p);                                        \
        const size_t lds = with_carries(size_t(2) * NS * (T + 1) * 16, jt.one.carry_cap);              \
        auto k = staged_reduce_kernel<d, p>;                                                            \
        k<<<persistent_grid(k, kStageThreads, lds, jt.n_chains), kStageThreads, lds, st>>>(jt, Tm, Tc); \
        return hipGetLastError();                                                                       \
    }
    QXA_STAGED(2, 1) QXA_STAGED(2, 2) QXA_STAGED(2, 3) QXA_STAGED(3, 1) QXA_STAGED(3, 2) QXA_STAGED(3, 3)
#undef QXA_STAGED
    return hipErrorInvalidValue;
}

#endif

#ifndef QXA_FUSED_PADDED
hipError_t launch_fixup(const FixupTable &ft, hipStream_t st)
{
    if (ft.n_fix == 0) return hipSuccess;
    fixup_kernel<<<unsigned((ft.n_fix + 255) / 256), 256, 0, st>>>(ft);
    return hipGetLastError();
}

bool fused_iso_fits(int D, int P, int nqm, int nqc, int64_t qfrag_vec16, int carry_cap)
{
    const size_t bytes = fused_iso_lds(D, P, nqm, nqc, qfrag_vec16);
    return bytes > 0 && with_carries(bytes, carry_cap) <= kLdsBytes;
}

hipError_t launch_fused_iso(const JobTable &jt, int D, int P, int nqm, int nqc, hipStream_t st)
{
    const FusedArgs &a = jt.one;
    if (jt.n_jobs != 0 || !a.dphi) return hipErrorInvalidValue;
#define X(d, p, m, c)                                                                                  \
    if (D == d && P == p && nqm == m && nqc == c) {                                                   \
        constexpr int T = tile_size(d, p);                                                            \
        const size_t lds = with_carries(WsLds<d, p, m, c, QXA_FP64, T, true>::bytes(a.qfrag_vec16), a.carry_cap); \
        if (lds > kLdsBytes) return hipErrorInvalidValue;                                             \
        auto k = fused_ws_kernel<d, p, m, c, QXA_FP64, T, false, true>;                               \
        k<<<persistent_grid(k, ws_threads(T, true), lds, jt.n_chains), ws_threads(T, true), lds, st>>>(jt); \
        return hipGetLastError();                                                                     \
    }
    QXA_ISO_CASES(X)
#undef X
    return hipErrorInvalidValue;
}
#undef QXA_ISO_CASES
#endif

}  // namespace qxa
