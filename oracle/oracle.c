/*
 * CPU FP64 reference for the assembly of finite element mass and conductivity
 * matrices (Voet, "On the fast assemblage of finite element matrices with
 * application to nonlinear heat transfer problems").
 *
 * TEST INFRASTRUCTURE. This file is the oracle: only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it. The
 * product library does not link, include or call it, and it shares no code,
 * table or helper with the product.
 *
 * What it computes is the plain definition (Section 2 and Section 3):
 *   M_ij = sum_e sum_q w_q m_qe phi_i(x_q) phi_j(x_q) |det B_e|
 *   C_ij = sum_e sum_q w_q c_qe (J_q A_e J_q^T)_ij |det B_e|,  A_e = (B_e^T B_e)^{-1}
 * in the order of Algorithm 1: a loop over elements, an inner loop over
 * quadrature nodes, then the addition of each local matrix into the global
 * matrix at the rows/columns of its node set N_e.
 *
 * Beyond these, with the same loops: the tensors of the Newton Jacobian of
 * Section 5 contracted with a vector (the full local n_p^3 tensor formed, then
 * contracted), the volume load vector of Section 2, an anisotropic conductivity
 * (a constant tensor, or one per quadrature node, Section 7) and isoparametric
 * elements (B, |det B| and A per quadrature node from every node, Section 7).
 *
 * Deliberately different from any fast implementation:
 *   - the reference Lagrange basis is obtained by solving the monomial
 *     Vandermonde system on the reference nodes (not closed formulas);
 *   - det B_e and B_e^{-1} come from an LU factorisation with partial pivoting;
 *   - the sparsity pattern is built from node->element lists with a sort;
 *   - global sums are taken in ascending element order with Neumaier
 *     compensated summation.
 *
 * Planted-mistake hooks (oracle_set_fault) exist so that tests can show that
 * the pins detect a wrong oracle; fault 0 (the default) is the oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXP 20   /* nodes per element, up to P3 tetrahedra */
#define MAXD 3

static int g_fault = 0;
void oracle_set_fault(int f) { g_fault = f; }

/* ------------------------------------------------------------------ */
/* Local nodes: vertices, then edge nodes, then face nodes (mesh format).  */
/* Returns n_p and the barycentric multi-indices alpha[n_p][dim+1].         */
/* ------------------------------------------------------------------ */
static int local_alpha(int dim, int P, int alpha[MAXP][4])
{
    static const int e2[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    static const int e3[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
    int n = 0;
    memset(alpha, 0, sizeof(int) * MAXP * 4);
    for (int k = 0; k <= dim; ++k) alpha[n++][k] = P;
    int ne = dim == 2 ? 3 : 6;
    for (int s = 0; s < ne; ++s) {
        int a = dim == 2 ? e2[s][0] : e3[s][0];
        int b = dim == 2 ? e2[s][1] : e3[s][1];
        for (int t = 1; t < P; ++t) {
            alpha[n][a] = P - t;
            alpha[n][b] = t;
            ++n;
        }
    }
    if (P == 3) {
        if (dim == 2) {
            alpha[n][0] = alpha[n][1] = alpha[n][2] = 1;
            ++n;
        } else {
            static const int opp[4] = {3, 0, 1, 2};
            for (int f = 0; f < 4; ++f) {
                for (int k = 0; k < 4; ++k) alpha[n][k] = (k == opp[f]) ? 0 : 1;
                ++n;
            }
        }
    }
    return n;
}

int oracle_n_local(int dim, int P)
{
    int alpha[MAXP][4];
    return local_alpha(dim, P, alpha);
}

/* Reference coordinates of the local nodes: xhat_k = alpha_k / P, k = 1..dim. */
int oracle_local_nodes(int dim, int P, double *xref)
{
    int alpha[MAXP][4];
    int n = local_alpha(dim, P, alpha);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) xref[i * dim + k] = (double)alpha[i][k + 1] / P;
    return n;
}

/* Monomial exponents x^a y^b (z^c) with total degree <= P, fixed order. */
static int monomials(int dim, int P, int ex[MAXP][MAXD])
{
    int n = 0;
    for (int t = 0; t <= P; ++t)
        for (int a = t; a >= 0; --a) {
            if (dim == 2) {
                ex[n][0] = a;
                ex[n][1] = t - a;
                ++n;
            } else {
                for (int b = t - a; b >= 0; --b) {
                    ex[n][0] = a;
                    ex[n][1] = b;
                    ex[n][2] = t - a - b;
                    ++n;
                }
            }
        }
    return n;
}

static double ipow(double x, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

/* Solve A X = B (n x n, m right-hand sides) by Gaussian elimination with partial
 * pivoting; A and B are overwritten (B receives X). Returns the determinant. */
static double gauss_solve(int n, double *A, int m, double *B)
{
    double det = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[c * n + k];
                A[c * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            for (int k = 0; k < m; ++k) {
                double t = B[c * m + k];
                B[c * m + k] = B[piv * m + k];
                B[piv * m + k] = t;
            }
            det = -det;
        }
        double p = A[c * n + c];
        det *= p;
        if (p == 0.0) return 0.0;
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / p;
            if (f == 0.0) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            for (int k = 0; k < m; ++k) B[r * m + k] -= f * B[c * m + k];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int k = 0; k < m; ++k) {
            double s = B[c * m + k];
            for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * B[j * m + k];
            B[c * m + k] = s / A[c * n + c];
        }
    }
    return det;
}

/*
 * Reference Lagrange basis on the reference simplex (Section 3, step 3: the
 * basis only needs to be defined on the reference element). phi_i is the
 * polynomial of degree <= P with phi_i(xhat_j) = delta_ij, found by solving the
 * Vandermonde system V c = I over the monomial basis.
 * Outputs phi[npts][n_p] and dphi[npts][n_p][dim] (the rows of J_q).
 */
int oracle_basis(int dim, int P, int npts, const double *pts, double *phi, double *dphi)
{
    int ex[MAXP][MAXD];
    int nm = monomials(dim, P, ex);
    double xref[MAXP * MAXD];
    int n = oracle_local_nodes(dim, P, xref);
    if (n != nm) return -1;
    double V[MAXP * MAXP], Cf[MAXP * MAXP];
    for (int i = 0; i < n; ++i)
        for (int m = 0; m < nm; ++m) {
            double v = 1.0;
            for (int k = 0; k < dim; ++k) v *= ipow(xref[i * dim + k], ex[m][k]);
            V[i * nm + m] = v;
        }
    /* V[i][m] * Cf[m][j] = delta_ij  -> phi_j(x) = sum_m Cf[m][j] mono_m(x) */
    for (int i = 0; i < n * n; ++i) Cf[i] = 0.0;
    for (int i = 0; i < n; ++i) Cf[i * n + i] = 1.0;
    if (gauss_solve(n, V, n, Cf) == 0.0) return -2;
    for (int q = 0; q < npts; ++q) {
        const double *x = pts + (size_t)q * dim;
        double mono[MAXP], dmono[MAXP][MAXD];
        for (int m = 0; m < nm; ++m) {
            double v = 1.0;
            for (int k = 0; k < dim; ++k) v *= ipow(x[k], ex[m][k]);
            mono[m] = v;
            for (int k = 0; k < dim; ++k) {
                if (ex[m][k] == 0) {
                    dmono[m][k] = 0.0;
                    continue;
                }
                double g = (double)ex[m][k];
                for (int l = 0; l < dim; ++l) g *= ipow(x[l], l == k ? ex[m][l] - 1 : ex[m][l]);
                dmono[m][k] = g;
            }
        }
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            double g[MAXD] = {0.0, 0.0, 0.0};
            for (int m = 0; m < nm; ++m) {
                s += Cf[m * n + j] * mono[m];
                for (int k = 0; k < dim; ++k) g[k] += Cf[m * n + j] * dmono[m][k];
            }
            phi[(size_t)q * n + j] = s;
            for (int k = 0; k < dim; ++k) dphi[((size_t)q * n + j) * dim + k] = g[k];
        }
    }
    return n;
}

/* ------------------------------------------------------------------ */
/* Coefficients                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int kind;            /* 0 constant, 1 nodal field interpolated at q, 2 values per (q, e) */
    int law;             /* 0 identity, 1 a0+a1 s+a2 s^2, 2 exp(a0+a1 s) */
    double value;        /* constant value (kind 0) */
    double a[3];
    const double *field; /* kind 1: [n_nodes]; kind 2: [n_q][n_e] */
    const double *tensor; /* conductivity only: upper triangle (row-major) of a symmetric
                             d x d tensor K (Section 7, anisotropic conductivity), or NULL */
    const double *tensor_q; /* conductivity only: a symmetric tensor per quadrature node,
                               [n_q][d(d+1)/2][n_e] upper triangles (Section 7, c_q varying
                               over the domain), or NULL; exclusive with tensor */
} oracle_coeff;

/* Upper triangle of the conductivity tensor at node q of element e (NULL: identity). */
static const double *tensor_at(const oracle_coeff *c, int d, int64_t n_e, int64_t e, int q, double *buf)
{
    if (!c->tensor_q) return c->tensor;
    int ng = d * (d + 1) / 2;
    for (int g = 0; g < ng; ++g) buf[g] = c->tensor_q[((size_t)q * ng + g) * n_e + e];
    return buf;
}

/* A_e = B^{-1} K B^{-T} (K = identity when tensor is NULL), full d x d. */
static void metric(int d, const double *Binv, const double *tensor, double *A)
{
    double K[MAXD * MAXD];
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) K[a * d + b] = (a == b) ? 1.0 : 0.0;
    if (tensor) {
        int g = 0;
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b, ++g) K[a * d + b] = K[b * d + a] = tensor[g];
    }
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            double s = 0.0;
            for (int k = 0; k < d; ++k)
                for (int l = 0; l < d; ++l) s += Binv[a * d + k] * K[k * d + l] * Binv[b * d + l];
            A[a * d + b] = s;
        }
}

static double apply_law(const oracle_coeff *c, double s)
{
    switch (c->law) {
    case 1: return c->a[0] + c->a[1] * s + c->a[2] * s * s;
    case 2: return exp(c->a[0] + c->a[1] * s);
    default: return s;
    }
}

typedef struct {
    int dim, P, n, nq_m, nq_c;
    const double *w_m, *w_c;
    double phi_m[64 * MAXP], dphi_m[64 * MAXP * MAXD];
    double phi_c[64 * MAXP], dphi_c[64 * MAXP * MAXD];
} refdata;

static int ref_setup(refdata *R, int dim, int P, int nq_m, const double *pts_m, const double *w_m,
                     int nq_c, const double *pts_c, const double *w_c)
{
    if (nq_m > 64 || nq_c > 64 || dim < 2 || dim > 3 || P < 1 || P > 3) return -1;
    R->dim = dim;
    R->P = P;
    R->nq_m = nq_m;
    R->nq_c = nq_c;
    R->w_m = w_m;
    R->w_c = w_c;
    int n1 = oracle_basis(dim, P, nq_m, pts_m, R->phi_m, R->dphi_m);
    int n2 = oracle_basis(dim, P, nq_c, pts_c, R->phi_c, R->dphi_c);
    if (n1 < 0 || n2 < 0) return -1;
    R->n = n1;
    return 0;
}

/* Coefficient value at quadrature node q of element e (Section 3: m_q = m(F_e(xhat_q)),
 * Section 5: solution-dependent coefficients evaluated at u_h = phi^T u). */
static double coeff_at(const oracle_coeff *c, const double *phi_q, int n, const int32_t *conn,
                       int64_t n_e, int64_t e, int q)
{
    if (c->kind == 0) return g_fault == 5 ? 1.0 : c->value;
    double s;
    if (c->kind == 1) {
        s = 0.0;
        for (int i = 0; i < n; ++i) s += phi_q[i] * c->field[conn[(size_t)i * n_e + e]];
    } else {
        s = c->field[(size_t)q * n_e + e];
    }
    if (g_fault == 5) return 1.0;
    return apply_law(c, s);
}

/*
 * Element matrices of element e (Algorithm 1, inner loop over q):
 *   M_e += w_q m_q phi_q phi_q^T |det B_e|
 *   C_e += w_q c_q J_q A_e J_q^T |det B_e|
 * with B_e = [a_1 - a_0, ..., a_d - a_0] (affine map of Section 3, step 3) and
 * A_e = (B_e^T B_e)^{-1} = B_e^{-1} B_e^{-T} (chain rule of Section 3).
 * Returns 0, or -3 for a degenerate element.
 */
static int element_matrices(const refdata *R, const double *coords, int64_t n_nodes, const int32_t *conn,
                            int64_t n_e, int64_t e, const oracle_coeff *cm, const oracle_coeff *cc,
                            double *Me, double *Ce)
{
    int d = R->dim, n = R->n;
    double a0[MAXD], B[MAXD * MAXD], Binv[MAXD * MAXD], A[MAXD * MAXD];
    int32_t v0 = conn[e];
    for (int k = 0; k < d; ++k) a0[k] = coords[(size_t)k * n_nodes + v0];
    double maxedge = 0.0;
    for (int c = 0; c < d; ++c) {
        int32_t vc = conn[(size_t)(c + 1) * n_e + e];
        double len2 = 0.0;
        for (int r = 0; r < d; ++r) {
            double t = coords[(size_t)r * n_nodes + vc] - a0[r];
            B[r * d + c] = t;
            len2 += t * t;
        }
        if (len2 > maxedge) maxedge = len2;
    }
    maxedge = sqrt(maxedge);
    /* det and inverse through LU with partial pivoting */
    double LU[MAXD * MAXD];
    memcpy(LU, B, sizeof(double) * d * d);
    for (int i = 0; i < d * d; ++i) Binv[i] = 0.0;
    for (int i = 0; i < d; ++i) Binv[i * d + i] = 1.0;
    double det = gauss_solve(d, LU, d, Binv);
    double adet = fabs(det);
    if (!(adet > 1e-14 * pow(maxedge, d))) return -3;
    if (g_fault == 1) adet = 1.0;           /* planted: dropped |det B_e| */
    /* A_e = B^{-1} B^{-T}, or B^{-1} K B^{-T} for an anisotropic conductivity */
    if (cc->tensor && g_fault != 2) {
        metric(d, Binv, cc->tensor, A);
    } else {
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                double s = 0.0;
                for (int k = 0; k < d; ++k) {
                    if (g_fault == 2) s += Binv[k * d + a] * Binv[k * d + b];   /* planted: B^{-T} B^{-1} */
                    else s += Binv[a * d + k] * Binv[b * d + k];
                }
                A[a * d + b] = s;
            }
    }
    for (int i = 0; i < n * n; ++i) {
        Me[i] = 0.0;
        Ce[i] = 0.0;
    }
    for (int q = 0; q < R->nq_m; ++q) {
        const double *ph = R->phi_m + (size_t)q * n;
        double wq = R->w_m[g_fault == 4 ? (q + 1) % R->nq_m : q];
        double mq = coeff_at(cm, ph, n, conn, n_e, e, q);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double pj = (g_fault == 6) ? ph[i] : ph[j];   /* planted: phi_i^2 */
                Me[i * n + j] += wq * mq * ph[i] * pj * adet;
            }
    }
    for (int q = 0; q < R->nq_c; ++q) {
        const double *ph = R->phi_c + (size_t)q * n;
        const double *Jq = R->dphi_c + (size_t)q * n * d;
        double wq = R->w_c[q];
        double cq = coeff_at(cc, ph, n, conn, n_e, e, q);
        if (cc->tensor_q) {   /* A_qe = B_e^{-1} K_qe B_e^{-T} per node */
            double kq[6];
            metric(d, Binv, tensor_at(cc, d, n_e, e, q, kq), A);
        }
        double JA[MAXP * MAXD];
        for (int i = 0; i < n; ++i)
            for (int b = 0; b < d; ++b) {
                double s = 0.0;
                for (int a = 0; a < d; ++a) {
                    double jia = Jq[i * d + a];
                    if (g_fault == 3 && a == 0) jia = -jia;   /* planted: sign of one gradient component */
                    s += jia * A[a * d + b];
                }
                JA[i * d + b] = s;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int b = 0; b < d; ++b) s += JA[i * d + b] * Jq[j * d + b];
                Ce[i * n + j] += wq * cq * s * adet;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Node -> element lists (ascending element id) and the CSR pattern.    */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t *start; /* [n_nodes+1] */
    int64_t *elem;  /* element ids, ascending per node */
    int8_t *loc;    /* local index of the node in that element */
} adjacency;

static int build_adjacency(int n, int64_t n_nodes, const int32_t *conn, int64_t n_e, adjacency *adj)
{
    adj->start = (int64_t *)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    if (!adj->start) return -5;
    for (int i = 0; i < n; ++i)
        for (int64_t e = 0; e < n_e; ++e) {
            int32_t v = conn[(size_t)i * n_e + e];
            if (v < 0 || v >= n_nodes) return -2;
            adj->start[v + 1]++;
        }
    for (int64_t v = 0; v < n_nodes; ++v) adj->start[v + 1] += adj->start[v];
    int64_t tot = adj->start[n_nodes];
    adj->elem = (int64_t *)malloc(sizeof(int64_t) * (size_t)(tot ? tot : 1));
    adj->loc = (int8_t *)malloc((size_t)(tot ? tot : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_nodes ? n_nodes : 1));
    if (!adj->elem || !adj->loc || !fill) return -5;
    memcpy(fill, adj->start, sizeof(int64_t) * (size_t)n_nodes);
    /* element-major traversal keeps each node's list in ascending element order */
    for (int64_t e = 0; e < n_e; ++e)
        for (int i = 0; i < n; ++i) {
            int32_t v = conn[(size_t)i * n_e + e];
            int64_t p = fill[v]++;
            adj->elem[p] = e;
            adj->loc[p] = (int8_t)i;
        }
    free(fill);
    return 0;
}

static void free_adjacency(adjacency *adj)
{
    free(adj->start);
    free(adj->elem);
    free(adj->loc);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Sorted unique columns of row v: nodes sharing an element with v (Section 3, step 2). */
static int row_columns(int n, const int32_t *conn, int64_t n_e, const adjacency *adj, int64_t v, int32_t *buf)
{
    int cnt = 0;
    for (int64_t p = adj->start[v]; p < adj->start[v + 1]; ++p) {
        int64_t e = adj->elem[p];
        for (int j = 0; j < n; ++j) buf[cnt++] = conn[(size_t)j * n_e + e];
    }
    qsort(buf, cnt, sizeof(int32_t), cmp_i32);
    int u = 0;
    for (int k = 0; k < cnt; ++k)
        if (u == 0 || buf[k] != buf[u - 1]) buf[u++] = buf[k];
    return u;
}

static int64_t max_row_contrib(int n, const adjacency *adj, int64_t n_nodes)
{
    int64_t m = 0;
    for (int64_t v = 0; v < n_nodes; ++v) {
        int64_t c = (adj->start[v + 1] - adj->start[v]) * n;
        if (c > m) m = c;
    }
    return m;
}

/* row_ptr[n_nodes+1] of the structural pattern; returns nnz or a negative code. */
int64_t oracle_pattern_rows(int dim, int P, int64_t n_nodes, int64_t n_e, const int32_t *conn, int64_t *row_ptr)
{
    int n = oracle_n_local(dim, P);
    adjacency adj;
    int rc = build_adjacency(n, n_nodes, conn, n_e, &adj);
    if (rc) return rc;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(max_row_contrib(n, &adj, n_nodes) + 1));
    row_ptr[0] = 0;
    for (int64_t v = 0; v < n_nodes; ++v) row_ptr[v + 1] = row_ptr[v] + row_columns(n, conn, n_e, &adj, v, buf);
    free(buf);
    free_adjacency(&adj);
    return row_ptr[n_nodes];
}

int oracle_pattern_cols(int dim, int P, int64_t n_nodes, int64_t n_e, const int32_t *conn, const int64_t *row_ptr,
                        int32_t *col_idx)
{
    int n = oracle_n_local(dim, P);
    adjacency adj;
    int rc = build_adjacency(n, n_nodes, conn, n_e, &adj);
    if (rc) return rc;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(max_row_contrib(n, &adj, n_nodes) + 1));
    for (int64_t v = 0; v < n_nodes; ++v) {
        int u = row_columns(n, conn, n_e, &adj, v, buf);
        memcpy(col_idx + row_ptr[v], buf, sizeof(int32_t) * u);
    }
    free(buf);
    free_adjacency(&adj);
    return 0;
}

static int64_t find_slot(const int32_t *cols, int64_t lo, int64_t hi, int32_t c)
{
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (cols[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* Neumaier compensated addition */
static inline void kadd(double *s, double *comp, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *comp += (*s - t) + x;
    else *comp += (x - t) + *s;
    *s = t;
}

/*
 * Global assembly for a set of rows (Algorithm 1, lines M(N_e,N_e) += M_e):
 * for each requested row v, the elements containing v are visited in ascending
 * order and their local rows are added into the row's slots. Summation order
 * per slot is ascending element id, identical to a serial run of Algorithm 1.
 * rows == NULL means all rows 0..n_nodes-1 (then out arrays are full CSR).
 * row_ptr/col_idx describe the requested rows only (sub-CSR).
 */
static int assemble_rows(const refdata *R, const double *coords, int64_t n_nodes, const int32_t *conn, int64_t n_e,
                         const oracle_coeff *cm, const oracle_coeff *cc, int64_t n_rows, const int64_t *rows,
                         const int64_t *row_ptr, const int32_t *col_idx, double *Mv, double *Cv,
                         const double *Mebuf, const double *Cebuf, int nthreads, int64_t *bad_elem)
{
    int n = R->n;
    adjacency adj;
    int rc = build_adjacency(n, n_nodes, conn, n_e, &adj);
    if (rc) return rc;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double Me[MAXP * MAXP], Ce[MAXP * MAXP];
        int64_t maxlen = 0;
        for (int64_t r = 0; r < n_rows; ++r) {
            int64_t l = row_ptr[r + 1] - row_ptr[r];
            if (l > maxlen) maxlen = l;
        }
        double *compM = (double *)calloc((size_t)maxlen + 1, sizeof(double));
        double *compC = (double *)calloc((size_t)maxlen + 1, sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
        for (int64_t r = 0; r < n_rows; ++r) {
            int64_t v = rows ? rows[r] : r;
            int64_t lo = row_ptr[r], hi = row_ptr[r + 1];
            for (int64_t k = lo; k < hi; ++k) {
                Mv[k] = 0.0;
                Cv[k] = 0.0;
                compM[k - lo] = 0.0;
                compC[k - lo] = 0.0;
            }
            for (int64_t p = adj.start[v]; p < adj.start[v + 1]; ++p) {
                int64_t e = adj.elem[p];
                int i = adj.loc[p];
                const double *me, *ce;
                if (Mebuf) {
                    me = Mebuf + (size_t)e * n * n;
                    ce = Cebuf + (size_t)e * n * n;
                } else {
                    if (element_matrices(R, coords, n_nodes, conn, n_e, e, cm, cc, Me, Ce)) {
#ifdef _OPENMP
#pragma omp critical
#endif
                        {
                            err = -3;
                            *bad_elem = e;
                        }
                        continue;
                    }
                    me = Me;
                    ce = Ce;
                }
                for (int j = 0; j < n; ++j) {
                    int32_t col = conn[(size_t)j * n_e + e];
                    int64_t s = find_slot(col_idx, lo, hi, col);
                    kadd(&Mv[s], &compM[s - lo], me[i * n + j]);
                    kadd(&Cv[s], &compC[s - lo], ce[i * n + j]);
                }
            }
            for (int64_t k = lo; k < hi; ++k) {
                Mv[k] += compM[k - lo];
                Cv[k] += compC[k - lo];
            }
        }
        free(compM);
        free(compC);
    }
    free_adjacency(&adj);
    return err;
}

/*
 * Full assembly: element matrices of all elements (parallel over elements),
 * then the global CSR values (parallel over rows, ascending elements per slot).
 * row_ptr/col_idx must be the oracle's own pattern (oracle_pattern_*).
 */
/* Wall-clock seconds of the last oracle_assemble call, split as the paper times it
 * (Section 6.1): formation of the element matrices, then their assembly into CSR.
 * Instrumentation only: no effect on any value computed. */
static double g_t_formation = 0.0, g_t_assembly = 0.0;
void oracle_last_timing(double *formation_s, double *assembly_s)
{
    *formation_s = g_t_formation;
    *assembly_s = g_t_assembly;
}

int oracle_assemble(int dim, int P, int64_t n_nodes, const double *coords, int64_t n_e, const int32_t *conn,
                    int nq_m, const double *pts_m, const double *w_m, int nq_c, const double *pts_c,
                    const double *w_c, const oracle_coeff *cm, const oracle_coeff *cc, const int64_t *row_ptr,
                    const int32_t *col_idx, double *Mv, double *Cv, int nthreads, int64_t *bad_elem)
{
    refdata R;
    if (ref_setup(&R, dim, P, nq_m, pts_m, w_m, nq_c, pts_c, w_c)) return -1;
    int n = R.n;
    double *Mebuf = (double *)malloc(sizeof(double) * (size_t)n_e * n * n);
    double *Cebuf = (double *)malloc(sizeof(double) * (size_t)n_e * n * n);
    if (!Mebuf || !Cebuf) {
        free(Mebuf);
        free(Cebuf);
        return -5;
    }
    int err = 0;
    double t0 = 0.0, t1 = 0.0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    t0 = omp_get_wtime();
#pragma omp parallel for schedule(static)
#endif
    for (int64_t e = 0; e < n_e; ++e) {
        if (element_matrices(&R, coords, n_nodes, conn, n_e, e, cm, cc, Mebuf + (size_t)e * n * n,
                             Cebuf + (size_t)e * n * n)) {
#ifdef _OPENMP
#pragma omp critical
#endif
            {
                if (!err || e < *bad_elem) *bad_elem = e;
                err = -3;
            }
        }
    }
#ifdef _OPENMP
    t1 = omp_get_wtime();
#endif
    if (!err)
        err = assemble_rows(&R, coords, n_nodes, conn, n_e, cm, cc, n_nodes, NULL, row_ptr, col_idx, Mv, Cv, Mebuf,
                            Cebuf, nthreads, bad_elem);
#ifdef _OPENMP
    g_t_formation = t1 - t0;
    g_t_assembly = omp_get_wtime() - t1;
#endif
    free(Mebuf);
    free(Cebuf);
    return err;
}

/* Selected rows only; element matrices are recomputed per row (bounded memory). */
int oracle_assemble_rows(int dim, int P, int64_t n_nodes, const double *coords, int64_t n_e, const int32_t *conn,
                         int nq_m, const double *pts_m, const double *w_m, int nq_c, const double *pts_c,
                         const double *w_c, const oracle_coeff *cm, const oracle_coeff *cc, int64_t n_rows,
                         const int64_t *rows, const int64_t *row_ptr, const int32_t *col_idx, double *Mv, double *Cv,
                         int nthreads, int64_t *bad_elem)
{
    refdata R;
    if (ref_setup(&R, dim, P, nq_m, pts_m, w_m, nq_c, pts_c, w_c)) return -1;
    return assemble_rows(&R, coords, n_nodes, conn, n_e, cm, cc, n_rows, rows, row_ptr, col_idx, Mv, Cv, NULL, NULL,
                         nthreads, bad_elem);
}

/* Columns of selected rows (sub-CSR): row_ptr[n_rows+1] then col_idx. Two calls:
 * with col_idx == NULL it fills row_ptr and returns the total. */
int64_t oracle_rows_pattern(int dim, int P, int64_t n_nodes, int64_t n_e, const int32_t *conn, int64_t n_rows,
                            const int64_t *rows, int64_t *row_ptr, int32_t *col_idx)
{
    int n = oracle_n_local(dim, P);
    adjacency adj;
    int rc = build_adjacency(n, n_nodes, conn, n_e, &adj);
    if (rc) return rc;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(max_row_contrib(n, &adj, n_nodes) + 1));
    row_ptr[0] = 0;
    for (int64_t r = 0; r < n_rows; ++r) {
        int u = row_columns(n, conn, n_e, &adj, rows[r], buf);
        if (col_idx) memcpy(col_idx + row_ptr[r], buf, sizeof(int32_t) * u);
        row_ptr[r + 1] = row_ptr[r] + u;
    }
    free(buf);
    free_adjacency(&adj);
    return row_ptr[n_rows];
}

/* Element matrices (full n_p x n_p, row-major) of selected elements. */
int oracle_element_matrices(int dim, int P, int64_t n_nodes, const double *coords, int64_t n_e, const int32_t *conn,
                            int nq_m, const double *pts_m, const double *w_m, int nq_c, const double *pts_c,
                            const double *w_c, const oracle_coeff *cm, const oracle_coeff *cc, int64_t n_sel,
                            const int64_t *elems, double *Me, double *Ce)
{
    refdata R;
    if (ref_setup(&R, dim, P, nq_m, pts_m, w_m, nq_c, pts_c, w_c)) return -1;
    int n = R.n;
    for (int64_t k = 0; k < n_sel; ++k) {
        int rc = element_matrices(&R, coords, n_nodes, conn, n_e, elems[k], cm, cc, Me + (size_t)k * n * n,
                                  Ce + (size_t)k * n * n);
        if (rc) return rc;
    }
    return 0;
}

/* Coefficient values at the quadrature nodes of selected elements (as used above). */
int oracle_qpoint_coeff(int dim, int P, int64_t n_e, const int32_t *conn, int nq, const double *pts,
                        const oracle_coeff *c, int64_t n_sel, const int64_t *elems, double *out)
{
    double phi[64 * MAXP], dphi[64 * MAXP * MAXD];
    int n = oracle_basis(dim, P, nq, pts, phi, dphi);
    if (n < 0) return -1;
    for (int64_t k = 0; k < n_sel; ++k)
        for (int q = 0; q < nq; ++q) out[k * nq + q] = coeff_at(c, phi + (size_t)q * n, n, conn, n_e, elems[k], q);
    return 0;
}

/*
 * Mass tensor of Section 5 contracted with a nodal vector v in its second mode:
 *   M_ijk = sum_e sum_q w_q m'_q phi_i phi_j phi_k |det B_e|,
 *   (M o_2 v)_ik = sum_j M_ijk v_j.
 * Per element the local tensor (n_p^3 entries, phi_q (x) phi_q (x) phi_q weighted
 * by lambda_q = w_q m'_q |det B_e|) is formed in full, then contracted with the
 * element's entries of v; the local matrices are added into the CSR pattern like
 * the mass matrix. cdm carries m' (kind 1: law of the interpolated nodal field).
 */
static int element_abs_det(const refdata *R, const double *coords, int64_t n_nodes, const int32_t *conn, int64_t n_e,
                           int64_t e, double *adet)
{
    int d = R->dim;
    double B[MAXD * MAXD], X[MAXD * MAXD];
    int32_t v0 = conn[e];
    double maxedge = 0.0;
    for (int c = 0; c < d; ++c) {
        int32_t vc = conn[(size_t)(c + 1) * n_e + e];
        double len2 = 0.0;
        for (int r = 0; r < d; ++r) {
            double t = coords[(size_t)r * n_nodes + vc] - coords[(size_t)r * n_nodes + v0];
            B[r * d + c] = t;
            len2 += t * t;
        }
        if (len2 > maxedge) maxedge = len2;
    }
    for (int i = 0; i < d * d; ++i) X[i] = (i % (d + 1) == 0) ? 1.0 : 0.0;
    double det = gauss_solve(d, B, d, X);
    *adet = fabs(det);
    return *adet > 1e-14 * pow(sqrt(maxedge), d) ? 0 : -3;
}

int oracle_mass_tensor_product(int dim, int P, int64_t n_nodes, const double *coords, int64_t n_e, const int32_t *conn,
                               int nq, const double *pts, const double *w, const oracle_coeff *cdm, const double *v,
                               const int64_t *row_ptr, const int32_t *col_idx, double *Tv, int nthreads,
                               int64_t *bad_elem)
{
    refdata R;
    if (ref_setup(&R, dim, P, nq, pts, w, nq, pts, w)) return -1;
    int n = R.n;
    double *Tbuf = (double *)malloc(sizeof(double) * (size_t)n_e * n * n);
    double *dummy = (double *)malloc(sizeof(double) * (size_t)(row_ptr[n_nodes] + 1));
    if (!Tbuf || !dummy) {
        free(Tbuf);
        free(dummy);
        return -5;
    }
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t e = 0; e < n_e; ++e) {
        double adet, Me[MAXP * MAXP * MAXP];
        if (element_abs_det(&R, coords, n_nodes, conn, n_e, e, &adet)) {
#ifdef _OPENMP
#pragma omp critical
#endif
            {
                if (!err || e < *bad_elem) *bad_elem = e;
                err = -3;
            }
            continue;
        }
        for (int t = 0; t < n * n * n; ++t) Me[t] = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double *ph = R.phi_m + (size_t)q * n;
            double lam = w[q] * coeff_at(cdm, ph, n, conn, n_e, e, q) * adet;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    for (int k = 0; k < n; ++k) Me[(i * n + j) * n + k] += lam * ph[i] * ph[j] * ph[k];
        }
        double *T = Tbuf + (size_t)e * n * n;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += Me[(i * n + j) * n + k] * v[conn[(size_t)j * n_e + e]];
                T[i * n + k] = s;
            }
    }
    if (!err)
        err = assemble_rows(&R, coords, n_nodes, conn, n_e, cdm, cdm, n_nodes, NULL, row_ptr, col_idx, Tv, dummy, Tbuf,
                            Tbuf, nthreads, bad_elem);
    free(Tbuf);
    free(dummy);
    return err;
}

/*
 * Conductivity tensor of Section 5 contracted with a nodal vector v in its second
 * mode (the Newton Jacobian term):
 *   C_ijk = sum_e sum_q w_q c'_q (J_q A_e J_q^T)_ij phi_k |det B_e|,
 *   (C o_2 v)_ik = sum_j C_ijk v_j      (not symmetric in i, k).
 * Per element the full local tensor (n_p^3 entries) is formed, then contracted with
 * the element's entries of v; the local matrices (row i, column k) are added into
 * the CSR pattern. cdc carries c' (kind 1: law of the interpolated nodal field).
 */
int oracle_cond_tensor_product(int dim, int P, int64_t n_nodes, const double *coords, int64_t n_e, const int32_t *conn,
                               int nq, const double *pts, const double *w, const oracle_coeff *cdc, const double *v,
                               const int64_t *row_ptr, const int32_t *col_idx, double *Tv, int nthreads,
                               int64_t *bad_elem)
{
    refdata R;
    if (ref_setup(&R, dim, P, nq, pts, w, nq, pts, w)) return -1;
    int n = R.n, d = dim;
    double *Tbuf = (double *)malloc(sizeof(double) * (size_t)n_e * n * n);
    double *dummy = (double *)malloc(sizeof(double) * (size_t)(row_ptr[n_nodes] + 1));
    if (!Tbuf || !dummy) {
        free(Tbuf);
        free(dummy);
        return -5;
    }
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t e = 0; e < n_e; ++e) {
        double B[MAXD * MAXD], Binv[MAXD * MAXD], A[MAXD * MAXD], Ce[MAXP * MAXP * MAXP];
        int32_t v0 = conn[e];
        double maxedge = 0.0;
        for (int c = 0; c < d; ++c) {
            int32_t vc = conn[(size_t)(c + 1) * n_e + e];
            double len2 = 0.0;
            for (int r = 0; r < d; ++r) {
                double t = coords[(size_t)r * n_nodes + vc] - coords[(size_t)r * n_nodes + v0];
                B[r * d + c] = t;
                len2 += t * t;
            }
            if (len2 > maxedge) maxedge = len2;
        }
        for (int i = 0; i < d * d; ++i) Binv[i] = (i % (d + 1) == 0) ? 1.0 : 0.0;
        double det = gauss_solve(d, B, d, Binv);
        double adet = fabs(det);
        if (!(adet > 1e-14 * pow(sqrt(maxedge), d))) {
#ifdef _OPENMP
#pragma omp critical
#endif
            {
                if (!err || e < *bad_elem) *bad_elem = e;
                err = -3;
            }
            continue;
        }
        metric(d, Binv, cdc->tensor, A);
        for (int t = 0; t < n * n * n; ++t) Ce[t] = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double *ph = R.phi_m + (size_t)q * n;
            const double *Jq = R.dphi_m + (size_t)q * n * d;
            double lam = w[q] * coeff_at(cdc, ph, n, conn, n_e, e, q) * adet;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double g = 0.0;   /* (J_q A J_q^T)_ij */
                    for (int a = 0; a < d; ++a)
                        for (int b = 0; b < d; ++b) g += Jq[i * d + a] * A[a * d + b] * Jq[j * d + b];
                    for (int k = 0; k < n; ++k) Ce[(i * n + j) * n + k] += lam * g * ph[k];
                }
        }
        /* contracted with v_j - v_0: the same in exact arithmetic (sum_j grad phi_j = 0, so
         * sum_j C_ijk = 0) and without the cancellation of |v| against its small variation
         * over an element */
        double *T = Tbuf + (size_t)e * n * n;
        const double vbase = v[conn[e]];
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += Ce[(i * n + j) * n + k] * (v[conn[(size_t)j * n_e + e]] - vbase);
                T[i * n + k] = s;
            }
    }
    if (!err)
        err = assemble_rows(&R, coords, n_nodes, conn, n_e, cdc, cdc, n_nodes, NULL, row_ptr, col_idx, Tv, dummy, Tbuf,
                            Tbuf, nthreads, bad_elem);
    free(Tbuf);
    free(dummy);
    return err;
}

/*
 * Volume load vector f_i = int f phi_i (Section 2), in the order of Algorithm 1:
 * per element, per quadrature node of the rule, f_q w_q phi_i(xhat_q) |det B_e| is
 * added into F[N_e(i)]; every entry is summed in ascending element order with
 * compensation. cf: the coefficient f (constant, nodal field through a law, or
 * values per (q, e)).
 */
int oracle_load_vector(int dim, int P, int64_t n_nodes, const double *coords, int64_t n_e, const int32_t *conn, int nq,
                       const double *pts, const double *w, const oracle_coeff *cf, double *F, int64_t *bad_elem)
{
    refdata R;
    if (ref_setup(&R, dim, P, nq, pts, w, nq, pts, w)) return -1;
    int n = R.n;
    double *comp = (double *)calloc((size_t)n_nodes, sizeof(double));
    if (!comp) return -5;
    for (int64_t i = 0; i < n_nodes; ++i) F[i] = 0.0;
    for (int64_t e = 0; e < n_e; ++e) {
        double adet;
        if (element_abs_det(&R, coords, n_nodes, conn, n_e, e, &adet)) {
            *bad_elem = e;
            free(comp);
            return -3;
        }
        double fe[MAXP];
        for (int i = 0; i < n; ++i) fe[i] = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double *ph = R.phi_m + (size_t)q * n;
            double lam = w[q] * coeff_at(cf, ph, n, conn, n_e, e, q) * adet;
            for (int i = 0; i < n; ++i) fe[i] += lam * ph[i];
        }
        for (int i = 0; i < n; ++i) {
            int32_t node = conn[(size_t)i * n_e + e];
            kadd(&F[node], &comp[node], fe[i]);
        }
    }
    for (int64_t i = 0; i < n_nodes; ++i) F[i] += comp[i];
    free(comp);
    return 0;
}

/*
 * Isoparametric elements (Section 7, curved geometry): the element map uses the same
 * Lagrange basis as the unknowns, x(xhat) = sum_i x_i phi_i(xhat), so B is evaluated per
 * quadrature node, B_q = sum_i x_i grad phi_i(xhat_q)^T, with |det B_q| and
 * A_q = B_q^{-1} B_q^{-T} per node (LU per node):
 *   M_e = sum_q w_q m_q phi_q phi_q^T |det B_q|,  C_e = sum_q w_q c_q J_q A_q J_q^T |det B_q|.
 * The local matrices are added into the CSR pattern like the affine ones.
 */
static int element_matrices_iso(const refdata *R, const double *coords, int64_t n_nodes, const int32_t *conn,
                                int64_t n_e, int64_t e, const oracle_coeff *cm, const oracle_coeff *cc, double *Me,
                                double *Ce)
{
    int d = R->dim, n = R->n;
    for (int i = 0; i < n * n; ++i) Me[i] = Ce[i] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        int nq = pass == 0 ? R->nq_m : R->nq_c;
        const double *phi = pass == 0 ? R->phi_m : R->phi_c;
        const double *dphi = pass == 0 ? R->dphi_m : R->dphi_c;
        const double *w = pass == 0 ? R->w_m : R->w_c;
        for (int q = 0; q < nq; ++q) {
            const double *ph = phi + (size_t)q * n, *Jq = dphi + (size_t)q * n * d;
            double B[MAXD * MAXD], Binv[MAXD * MAXD], A[MAXD * MAXD];
            /* B_q = sum_i (x_i - x_0) grad phi_i(xhat_q)^T: the gradients sum to zero, so
             * subtracting vertex 0 changes nothing exactly and keeps the sum free of the
             * cancellation of absolute coordinates on small elements (Section 3 builds B_e
             * from the same differences a_k - a_0) */
            for (int r = 0; r < d; ++r) {
                const double x0 = coords[(size_t)r * n_nodes + conn[e]];
                for (int c = 0; c < d; ++c) {
                    double s = 0.0;
                    for (int i = 0; i < n; ++i)
                        s += (coords[(size_t)r * n_nodes + conn[(size_t)i * n_e + e]] - x0) * Jq[i * d + c];
                    B[r * d + c] = s;
                }
            }
            for (int i = 0; i < d * d; ++i) Binv[i] = (i % (d + 1) == 0) ? 1.0 : 0.0;
            double adet = fabs(gauss_solve(d, B, d, Binv));
            if (!(adet > 0.0)) return -3;
            if (pass == 0) {
                double lam = w[q] * coeff_at(cm, ph, n, conn, n_e, e, q) * adet;
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) Me[i * n + j] += lam * ph[i] * ph[j];
            } else {
                double kq[6];
                metric(d, Binv, tensor_at(cc, d, n_e, e, q, kq), A);
                double lam = w[q] * coeff_at(cc, ph, n, conn, n_e, e, q) * adet;
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        double s = 0.0;
                        for (int a = 0; a < d; ++a)
                            for (int b = 0; b < d; ++b) s += Jq[i * d + a] * A[a * d + b] * Jq[j * d + b];
                        Ce[i * n + j] += lam * s;
                    }
            }
        }
    }
    return 0;
}

int oracle_assemble_iso(int dim, int P, int64_t n_nodes, const double *coords, int64_t n_e, const int32_t *conn,
                        int nq_m, const double *pts_m, const double *w_m, int nq_c, const double *pts_c,
                        const double *w_c, const oracle_coeff *cm, const oracle_coeff *cc, const int64_t *row_ptr,
                        const int32_t *col_idx, double *Mv, double *Cv, int nthreads, int64_t *bad_elem)
{
    refdata R;
    if (ref_setup(&R, dim, P, nq_m, pts_m, w_m, nq_c, pts_c, w_c)) return -1;
    int n = R.n;
    double *Mebuf = (double *)malloc(sizeof(double) * (size_t)n_e * n * n);
    double *Cebuf = (double *)malloc(sizeof(double) * (size_t)n_e * n * n);
    if (!Mebuf || !Cebuf) {
        free(Mebuf);
        free(Cebuf);
        return -5;
    }
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t e = 0; e < n_e; ++e) {
        if (element_matrices_iso(&R, coords, n_nodes, conn, n_e, e, cm, cc, Mebuf + (size_t)e * n * n,
                                 Cebuf + (size_t)e * n * n)) {
#ifdef _OPENMP
#pragma omp critical
#endif
            {
                if (!err || e < *bad_elem) *bad_elem = e;
                err = -3;
            }
        }
    }
    if (!err)
        err = assemble_rows(&R, coords, n_nodes, conn, n_e, cm, cc, n_nodes, NULL, row_ptr, col_idx, Mv, Cv, Mebuf,
                            Cebuf, nthreads, bad_elem);
    free(Mebuf);
    free(Cebuf);
    return err;
}
