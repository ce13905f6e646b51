// Device-side building blocks shared by the assembly kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qxa {

struct CoeffDev {
    int kind;  // 0 const, 1 nodal, 2 per (q, e)
    int law;   // 0 identity, 1 poly2, 2 exp
    double value, a0, a1, a2;
    const double *field;
};

__device__ __forceinline__ double apply_law(const CoeffDev &c, double s)
{
    if (c.law == 1) return fma(fma(c.a2, s, c.a1), s, c.a0);
    if (c.law == 2) return exp(fma(c.a1, s, c.a0));
    return s;
}

// Geometry of Section 3 (affine map x = a_0 + B_e xhat, B_e = [a_1-a_0, ..., a_d-a_0])
// and Section 4 (b_e = |det B_e|, W column = vec(A_e), A_e = (B_e^T B_e)^{-1}
// = B_e^{-1} B_e^{-T}), symmetric A_e stored as its d(d+1)/2 upper entries
// in row-major order: 2D (00,01,11), 3D (00,01,02,11,12,22).
template <int D>
__device__ __forceinline__ void element_geometry(const double *__restrict__ xyz, int64_t n_nodes, const int32_t *v,
                                                 double &babs, double *A)
{
    if constexpr (D == 2) {
        const double x0 = xyz[v[0]], y0 = xyz[n_nodes + v[0]];
        const double b00 = xyz[v[1]] - x0, b10 = xyz[n_nodes + v[1]] - y0;
        const double b01 = xyz[v[2]] - x0, b11 = xyz[n_nodes + v[2]] - y0;
        const double det = b00 * b11 - b01 * b10;
        const double r = 1.0 / det;
        // B^{-1} = adj(B) / det
        const double i00 = b11 * r, i01 = -b01 * r, i10 = -b10 * r, i11 = b00 * r;
        babs = fabs(det);
        A[0] = i00 * i00 + i01 * i01;
        A[1] = i00 * i10 + i01 * i11;
        A[2] = i10 * i10 + i11 * i11;
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
        int g = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b, ++g) A[g] = I[a][0] * I[b][0] + I[a][1] * I[b][1] + I[a][2] * I[b][2];
    }
}

}  // namespace qxa
