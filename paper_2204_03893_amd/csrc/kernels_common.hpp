// Device-side building blocks shared by the assembly kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qxa {

// Read-only tables shared by every lane (basis values, weights, Q). Read
// through the constant address space, loads at uniform addresses go through
// the scalar unit (and are batched) instead of one vector load and wait per
// value. The tables are never written while a kernel runs.
template <typename T>
using table_ptr = const T __attribute__((address_space(4))) *;
template <typename T>
__device__ __forceinline__ table_ptr<T> uniform_table(const T *p)
{
    return (table_ptr<T>)(p);
}

struct CoeffDev {
    int kind;  // 0 const, 1 nodal, 2 per (q, e)
    int law;   // 0 identity, 1 poly2, 2 exp
    double value, a0, a1, a2;
    const double *field;
    int nq;    // rows of a per-(q, e) field: the nodes of the caller's rule
    int pad0;
};

// Per-(q, e) value at node q of the compiled rule. A caller's rule shorter than
// the compiled one is padded with zero-weight copies of its node 0, which
// read node 0's value (finite whenever node 0's is, so its zero weight
// cancels it exactly).
__device__ __forceinline__ double qe_value(const CoeffDev &c, int q, int64_t n_elem, int64_t e)
{
    return c.field[int64_t(q < c.nq ? q : 0) * n_elem + e];
}

__device__ __forceinline__ double apply_law(const CoeffDev &c, double s)
{
    if (c.law == 1) return fma(fma(c.a2, s, c.a1), s, c.a0);
    if (c.law == 2) return exp(fma(c.a1, s, c.a0));
    return s;
}

// A = I K I^T from the inverse I = B_e^{-1}, as its d(d+1)/2 upper entries in
// row-major order; K = identity unless aniso (K: upper triangle, row-major, of the
// symmetric conductivity tensor, Section 7).
template <int D>
__device__ __forceinline__ void metric_from_inverse(const double (&I)[D][D], int aniso, const double *K, double *A)
{
    if (!aniso) {
        int g = 0;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b, ++g) {
                double s = I[a][0] * I[b][0];
#pragma unroll
                for (int k = 1; k < D; ++k) s += I[a][k] * I[b][k];
                A[g] = s;
            }
        return;
    }
    double Kf[D][D];
    {
        int g = 0;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b, ++g) Kf[a][b] = Kf[b][a] = K[g];
    }
    int g = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b, ++g) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double t = 0.0;
#pragma unroll
                for (int l = 0; l < D; ++l) t = fma(Kf[k][l], I[b][l], t);
                s = fma(I[a][k], t, s);
            }
            A[g] = s;
        }
}

// Geometry of Section 3 (affine map x = a_0 + B_e xhat, B_e = [a_1-a_0, ..., a_d-a_0])
// and Section 4 (b_e = |det B_e|, W column = vec(A_e), A_e = (B_e^T B_e)^{-1}
// = B_e^{-1} B_e^{-T}), symmetric A_e stored as its d(d+1)/2 upper entries
// in row-major order: 2D (00,01,11), 3D (00,01,02,11,12,22).
template <int D>
__device__ __forceinline__ void element_geometry(const double *__restrict__ xyz, int64_t n_nodes, const int32_t *v,
                                                 double &babs, double *A, int aniso = 0, const double *K = nullptr)
{
    if constexpr (D == 2) {
        const double x0 = xyz[v[0]], y0 = xyz[n_nodes + v[0]];
        const double b00 = xyz[v[1]] - x0, b10 = xyz[n_nodes + v[1]] - y0;
        const double b01 = xyz[v[2]] - x0, b11 = xyz[n_nodes + v[2]] - y0;
        const double det = b00 * b11 - b01 * b10;
        const double r = 1.0 / det;
        // B^{-1} = adj(B) / det
        const double I[2][2] = {{b11 * r, -b01 * r}, {-b10 * r, b00 * r}};
        babs = fabs(det);
        metric_from_inverse<2>(I, aniso, K, A);
    } else {
        double B[3][3];
        const double x0 = xyz[v[0]], y0 = xyz[n_nodes + v[0]], z0 = xyz[2 * n_nodes + v[0]];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            B[0][c] = xyz[v[c + 1]] - x0;
            B[1][c] = xyz[n_nodes + v[c + 1]] - y0;
            B[2][c] = xyz[2 * n_nodes + v[c + 1]] - z0;
        }
        // cofactors: adj(B)[a][k] = cof(B)[k][a]
        const double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
        const double c01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
        const double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
        const double c10 = B[0][2] * B[2][1] - B[0][1] * B[2][2];
        const double c11 = B[0][0] * B[2][2] - B[0][2] * B[2][0];
        const double c12 = B[0][1] * B[2][0] - B[0][0] * B[2][1];
        const double c20 = B[0][1] * B[1][2] - B[0][2] * B[1][1];
        const double c21 = B[0][2] * B[1][0] - B[0][0] * B[1][2];
        const double c22 = B[0][0] * B[1][1] - B[0][1] * B[1][0];
        const double det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02;
        const double r = 1.0 / det;
        // Binv[a][k] = cof[k][a] / det
        const double I[3][3] = {{c00 * r, c10 * r, c20 * r}, {c01 * r, c11 * r, c21 * r}, {c02 * r, c12 * r, c22 * r}};
        babs = fabs(det);
        metric_from_inverse<3>(I, aniso, K, A);
    }
}

// Inputs shared by every formation variant.
struct FormInputs {
    int64_t n_nodes, n_elem;
    const double *coords;  // [dim][n_nodes]
    CoeffDev cm, cc;
    int aniso;    // conductivity tensor K (upper triangle, row-major) instead of the identity
    double K[6];
    const double *w_m, *w_c;      // [nq]
    const double *phi_m, *phi_c;  // [np][nq]
    int *flags;
};

template <int D, int P>
struct Shape {
    static constexpr int NP = (D == 2) ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6;
    static constexpr int NS = NP * (NP + 1) / 2;
    static constexpr int NG = D * (D + 1) / 2;
};

// Geometry (b_e, W) and weighted coefficient columns (S, Lambda) of one
// element: b_e, vec(A_e), Lambda_m[:, e], Lambda_c[:, e]. `eid` is the element
// index used for per-(q, e) coefficient arrays. Returns false when a
// coefficient value is not finite.
template <int D, int P, int NQM, int NQC>
__device__ __forceinline__ bool element_setup(const FormInputs &in, const int32_t *v, int64_t eid, double *A,
                                              double *lm, double *lc)
{
    constexpr int NP = Shape<D, P>::NP;
    double babs;
    element_geometry<D>(in.coords, in.n_nodes, v, babs, A, in.aniso, in.K);
    double um[NP];
    if (in.cm.kind == 1 || in.cc.kind == 1) {
        const double *f = in.cm.kind == 1 ? in.cm.field : in.cc.field;
#pragma unroll
        for (int i = 0; i < NP; ++i) um[i] = f[v[i]];
    }
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NQM; ++q) {
        double s;
        if (in.cm.kind == 0) {
            s = in.cm.value;
        } else if (in.cm.kind == 1) {
            double uh = 0.0;  // u_h(xhat_q) = phi_q^T u_e
#pragma unroll
            for (int i = 0; i < NP; ++i) uh = fma(uniform_table(in.phi_m)[i * NQM + q], um[i], uh);
            s = apply_law(in.cm, uh);
        } else {
            s = apply_law(in.cm, qe_value(in.cm, q, in.n_elem, eid));
        }
        lm[q] = uniform_table(in.w_m)[q] * s * babs;
        ok &= isfinite(lm[q]);
    }
    double uc[NP];
    if (in.cc.kind == 1) {
        if (in.cm.kind == 1 && in.cc.field == in.cm.field) {
#pragma unroll
            for (int i = 0; i < NP; ++i) uc[i] = um[i];
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) uc[i] = in.cc.field[v[i]];
        }
    }
#pragma unroll
    for (int q = 0; q < NQC; ++q) {
        double s;
        if (in.cc.kind == 0) {
            s = in.cc.value;
        } else if (in.cc.kind == 1) {
            double uh = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) uh = fma(uniform_table(in.phi_c)[i * NQC + q], uc[i], uh);
            s = apply_law(in.cc, uh);
        } else {
            s = apply_law(in.cc, qe_value(in.cc, q, in.n_elem, eid));
        }
        lc[q] = uniform_table(in.w_c)[q] * s * babs;
        ok &= isfinite(lc[q]);
    }
    return ok;
}

// Inverse and |det| of a d x d matrix (adjugate over the determinant).
template <int D>
__device__ __forceinline__ void inverse_abs_det(const double (&B)[D][D], double (&I)[D][D], double &adet)
{
    if constexpr (D == 2) {
        const double det = B[0][0] * B[1][1] - B[0][1] * B[1][0], r = 1.0 / det;
        I[0][0] = B[1][1] * r;
        I[0][1] = -B[0][1] * r;
        I[1][0] = -B[1][0] * r;
        I[1][1] = B[0][0] * r;
        adet = fabs(det);
    } else {
        const double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
        const double c01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
        const double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
        const double det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02, r = 1.0 / det;
        I[0][0] = c00 * r;
        I[1][0] = c01 * r;
        I[2][0] = c02 * r;
        I[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) * r;
        I[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) * r;
        I[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) * r;
        I[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) * r;
        I[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) * r;
        I[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) * r;
        adet = fabs(det);
    }
}

// Raw per-element inputs gathered from memory (vertex coordinates and the
// first nodal field at the element's nodes), split from the arithmetic so a
// tile's gathers can be issued while the previous tile computes.
template <int D, int P>
struct RawElem {
    double x[D + 1][D];
    double u[Shape<D, P>::NP];
};

template <int D, int P>
__device__ __forceinline__ void gather_raw(const FormInputs &in, const int32_t *v, RawElem<D, P> &r)
{
#pragma unroll
    for (int k = 0; k <= D; ++k)
#pragma unroll
        for (int c = 0; c < D; ++c) r.x[k][c] = in.coords[c * in.n_nodes + v[k]];
    if (in.cm.kind == 1 || in.cc.kind == 1) {
        const double *f = in.cm.kind == 1 ? in.cm.field : in.cc.field;
#pragma unroll
        for (int i = 0; i < Shape<D, P>::NP; ++i) r.u[i] = f[v[i]];
    }
}

// Geometry from gathered vertex coordinates (same arithmetic as element_geometry).
template <int D>
__device__ __forceinline__ void geometry_from(const double (&x)[D + 1][D], double &babs, double *A, int aniso = 0,
                                              const double *K = nullptr)
{
    if constexpr (D == 2) {
        const double b00 = x[1][0] - x[0][0], b10 = x[1][1] - x[0][1];
        const double b01 = x[2][0] - x[0][0], b11 = x[2][1] - x[0][1];
        const double det = b00 * b11 - b01 * b10;
        const double r = 1.0 / det;
        const double I[2][2] = {{b11 * r, -b01 * r}, {-b10 * r, b00 * r}};
        babs = fabs(det);
        metric_from_inverse<2>(I, aniso, K, A);
    } else {
        double B[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int r = 0; r < 3; ++r) B[r][c] = x[c + 1][r] - x[0][r];
        const double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
        const double c01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
        const double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
        const double c10 = B[0][2] * B[2][1] - B[0][1] * B[2][2];
        const double c11 = B[0][0] * B[2][2] - B[0][2] * B[2][0];
        const double c12 = B[0][1] * B[2][0] - B[0][0] * B[2][1];
        const double c20 = B[0][1] * B[1][2] - B[0][2] * B[1][1];
        const double c21 = B[0][2] * B[1][0] - B[0][0] * B[1][2];
        const double c22 = B[0][0] * B[1][1] - B[0][1] * B[1][0];
        const double det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02;
        const double r = 1.0 / det;
        const double I[3][3] = {{c00 * r, c10 * r, c20 * r}, {c01 * r, c11 * r, c21 * r}, {c02 * r, c12 * r, c22 * r}};
        babs = fabs(det);
        metric_from_inverse<3>(I, aniso, K, A);
    }
}

// Geometry and Lambda columns from gathered inputs. When the two nodal fields
// differ, the second one is read here through the element's connectivity
// (tconn[i * ne + pos]); the gathered values hold the first.
template <int D, int P, int NQM, int NQC>
__device__ __forceinline__ bool setup_from_raw(const FormInputs &in, const RawElem<D, P> &r, const int32_t *tconn,
                                               int64_t pos, int64_t eid, double *A, double *lm, double *lc)
{
    constexpr int NP = Shape<D, P>::NP;
    double babs;
    geometry_from<D>(r.x, babs, A, in.aniso, in.K);
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NQM; ++q) {
        double s;
        if (in.cm.kind == 0) {
            s = in.cm.value;
        } else if (in.cm.kind == 1) {
            double uh = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) uh = fma(uniform_table(in.phi_m)[i * NQM + q], r.u[i], uh);
            s = apply_law(in.cm, uh);
        } else {
            s = apply_law(in.cm, qe_value(in.cm, q, in.n_elem, eid));
        }
        lm[q] = uniform_table(in.w_m)[q] * s * babs;
        ok &= isfinite(lm[q]);
    }
    double uc[NP];
    if (in.cc.kind == 1) {
        if (in.cm.kind != 1 || in.cc.field == in.cm.field) {
#pragma unroll
            for (int i = 0; i < NP; ++i) uc[i] = r.u[i];
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) uc[i] = in.cc.field[tconn[i * in.n_elem + pos]];
        }
    }
#pragma unroll
    for (int q = 0; q < NQC; ++q) {
        double s;
        if (in.cc.kind == 0) {
            s = in.cc.value;
        } else if (in.cc.kind == 1) {
            double uh = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) uh = fma(uniform_table(in.phi_c)[i * NQC + q], uc[i], uh);
            s = apply_law(in.cc, uh);
        } else {
            s = apply_law(in.cc, qe_value(in.cc, q, in.n_elem, eid));
        }
        lc[q] = uniform_table(in.w_c)[q] * s * babs;
        ok &= isfinite(lc[q]);
    }
    return ok;
}

// Workgroup barrier ordering LDS only: outstanding global loads (prefetches
// of the next tile) stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Tiles of a persistent launch, XCD-aware: workgroups are dispatched to the
// 8 XCDs round-robin, so workgroup b (XCD b % 8) walks a contiguous eighth of
// the tile order and each XCD's L2 sees one compact region of the mesh.
struct TileWalk {
    int64_t t, hi, step;
    __device__ TileWalk(int64_t n_tiles)
    {
        const int64_t b = blockIdx.x, G = gridDim.x;
        if (G % 8 == 0 && n_tiles >= G) {
            const int64_t x = b % 8, i = b / 8;
            const int64_t lo = x * n_tiles / 8;
            hi = (x + 1) * n_tiles / 8;
            t = lo + i;
            step = G / 8;
        } else {
            t = b;
            hi = n_tiles;
            step = G;
        }
    }
    // a contiguous range of tiles [t0, t1)
    __device__ TileWalk(int64_t t0, int64_t t1) : t(t0), hi(t1), step(1) {}
    __device__ bool valid(int64_t tt) const { return tt < hi; }
};

// One tile per workgroup (grid = n_tiles): blocks b = x (mod 8) run on XCD x
// and take the contiguous chunk of q + (x < r) tiles starting at
// x*q + min(x, r), q = n/8, r = n%8 (a bijection onto [0, n)).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n)
{
    const int64_t x = b % 8, i = b / 8, q = n / 8, r = n % 8;
    return x * q + (x < r ? x : r) + i;
}

// V_m[:, e] = Q_m X_m[:, e] with X_m = Lambda_m (Algorithm 2, mass matrix); store(s, value)
// receives each symmetric-pair entry.
template <int NS, int NQM, typename CT, class Store>
__device__ __forceinline__ void contract_mass(const CT *__restrict__ Qm, const double *lm, Store &&store)
{
    CT x[NQM];
#pragma unroll
    for (int q = 0; q < NQM; ++q) x[q] = CT(lm[q]);
#pragma unroll 1
    for (int s = 0; s < NS; ++s) {
        CT acc = CT(0);
#pragma unroll
        for (int q = 0; q < NQM; ++q) acc = fma(uniform_table(Qm)[s * NQM + q], x[q], acc);
        store(s, double(acc));
    }
}

// V_c[:, e] = Q_c X_c[:, e] with X_c = Lambda_c (Khatri-Rao) W (Algorithm 2, conductivity matrix).
template <int P, int NS, int NQC, int NG, typename CT, class Store>
__device__ __forceinline__ void contract_stiff(const CT *__restrict__ Qc, const double *lc, const double *A,
                                               Store &&store)
{
    constexpr bool FLAT = NQC * NG <= 96;
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
            for (int g = 0; g < NG; ++g) acc = fma(uniform_table(Qc)[s * NQC * NG + g], x[g], acc);
            store(s, double(acc));
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
            for (int k = 0; k < NQC * NG; ++k) acc = fma(uniform_table(Qc)[s * NQC * NG + k], x[k], acc);
            store(s, double(acc));
        }
    } else {
        // the same product with X_c = Lambda_c (.) W applied column block by block
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
                for (int g = 0; g < NG; ++g) t = fma(uniform_table(Qc)[(s * NQC + q) * NG + g], w[g], t);
                acc = fma(t, l[q], acc);
            }
            store(s, double(acc));
        }
    }
}

}  // namespace qxa
