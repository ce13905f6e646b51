/*
 * qxa — loop-free assembly of finite element mass and conductivity matrices
 * as one small dense contraction V = Q X, for AMD Instinct MI355X (gfx950).
 *
 * Method: Y. Voet, "On the fast assemblage of finite element matrices with
 * application to nonlinear heat transfer problems".
 *   - Section 2 defines the matrices: M_ij = int m phi_j phi_i and
 *     C_ij = int c grad phi_j . grad phi_i (the conductivity matrix).
 *   - Section 3 maps each simplex affinely to the reference element
 *     (x = a + B_e xhat) and applies quadrature.
 *   - Section 4 (Algorithm 2) vectorises all element matrices at once:
 *       V_m = Q_m X_m,  Q_m = Phi (Khatri-Rao) Phi,  X_m = Lambda_m
 *       V_c = Q_c X_c,  Q_c = [J_q (x) J_q]_q,        X_c = Lambda_c (Khatri-Rao) W
 *       Lambda = S * (w b^T),  b_e = |det B_e|,  W = [vec((B_e^T B_e)^{-1})]_e
 *     and forms the global matrices from V and the index sets N_e.
 *   - Section 5 (summary) notes that only S depends on the unknown, so the
 *     mesh-dependent data (pattern, permutation) is built once per mesh.
 *
 * All functions return a qxa_status (0 = success, negative = error) and never
 * throw; qxa_last_error() returns a message for the last failing call on the
 * calling thread. Indices are 0-based.
 *
 * Memory: the library never frees caller memory. qxa_mesh_create copies the
 * mesh into library-owned device memory. Output value arrays are caller-owned
 * device buffers. "device" pointers are HIP device pointers on the device the
 * mesh was created on; a stream argument is a hipStream_t (NULL = default).
 * An array argument whose length is zero (no elements, no nodes, nnz = 0) may
 * be NULL.
 *
 * Concurrency: a plan owns the scratch its launches use (shared-slot partial
 * sums, the local matrices of the two-pass entry points, the device flag read
 * by qxa_sync), so work queued with one plan must be ordered: one stream, or
 * streams synchronised by the caller. Calls with different plans may overlap.
 * The server (qxa_server_*) keeps its own plans and is thread-safe.
 */
#ifndef QXA_H
#define QXA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QXA_OK = 0,
    QXA_E_INVALID = -1,     /* bad argument (null pointer, size, enum value)        */
    QXA_E_INDEX = -2,       /* connectivity index out of range / repeated in N_e    */
    QXA_E_DEGENERATE = -3,  /* |det B_e| too small: B_e not invertible (Section 3) */
    QXA_E_NONFINITE = -4,   /* non-finite coordinate or coefficient value           */
    QXA_E_NOMEM = -5,       /* device or host allocation failed / over budget      */
    QXA_E_UNSUPPORTED = -6, /* (dim, order, n_q, precision) combination not built   */
    QXA_E_HIP = -7,         /* HIP runtime error                                    */
    QXA_E_BUSY = -8         /* server queue full, or a mesh still in use            */
} qxa_status;

/* Arithmetic of the contraction V = Q X. Geometry (B_e, |det B_e|, W) and the
 * accumulation into CSR are FP64 in every form. */
typedef enum {
    QXA_FP64 = 0,   /* plain FP64                                                   */
    QXA_FP32 = 1,   /* Q and X rounded to FP32, FP32 accumulation                  */
    QXA_F16X2 = 2,  /* Q, X split hi+lo in FP16 (per-element scaled X), MFMA, FP32 acc */
    QXA_BF16X2 = 3, /* Q, X split hi+lo in BF16, MFMA, FP32 accumulation           */
    QXA_BF16X3 = 4  /* three-term BF16 split, MFMA, FP32 accumulation              */
} qxa_precision;

/* Coefficient evaluation at the quadrature nodes, the matrices S_m, S_c of
 * Algorithm 2 (Section 4): constant (no evaluation needed), a law applied to the
 * interpolated nodal field u_h = phi^T u (solution-dependent coefficients,
 * Section 5), or values given per (q, e). */
typedef enum { QXA_COEFF_CONST = 0, QXA_COEFF_NODAL = 1, QXA_COEFF_QPOINT = 2 } qxa_coeff_kind;
typedef enum {
    QXA_LAW_IDENTITY = 0, /* s                     */
    QXA_LAW_POLY2 = 1,    /* a0 + a1 s + a2 s^2    */
    QXA_LAW_EXP = 2       /* exp(a0 + a1 s)        */
} qxa_law;

enum { QXA_MEM_HOST = 0, QXA_MEM_DEVICE = 1 };

/* Quadrature rule on the reference simplex (vertex 0 at the origin, vertex k
 * at e_k): n_q points (row-major [n_q][dim], reference coordinates) and
 * weights summing to 1/dim!. Host pointers; copied at plan creation. */
typedef struct {
    int dim;
    int n_q;
    const double *points;
    const double *weights;
} qxa_quad;

/* A built-in symmetric rule on the reference simplex exact for polynomials of degree
 * `degree` (the lowest built-in degree >= the one asked for: 1, 2, 4 or 6; dim 2 or 3).
 * Points and weights were solved from the orbit moment equations in high precision;
 * they satisfy every moment of that degree to rounding. The tables are library-owned
 * with static lifetime (host memory). Errors: QXA_E_INVALID (null out, dim not 2 or 3),
 * QXA_E_UNSUPPORTED (degree above 6). Host only; needs no GPU. */
qxa_status qxa_quad_builtin(int dim, int degree, qxa_quad *out);

/* kind = QXA_COEFF_CONST: s = value.
 * kind = QXA_COEFF_NODAL: field = device array [n_nodes]; s = law(u_h(x_q)).
 * kind = QXA_COEFF_QPOINT: field = device array [n_q][n_elem]; s = law(field[q][e]).
 * tensor (conductivity coefficients only, else NULL): host array of the upper
 * triangle, row-major, of a constant symmetric d x d tensor K (2D: K00, K01, K11;
 * 3D: K00, K01, K02, K11, K12, K22); the conductivity is then s K, the anisotropic
 * case of Section 7 with A_qe = B_e^{-1} s_q K B_e^{-T}. NULL: isotropic (K = I).
 * Read during the call (qxa_server_submit copies it).
 * tensor_q (conductivity coefficient of qxa_assemble_iso only, else NULL): device
 * array [n_q][d(d+1)/2][n_elem] of upper triangles, row-major, of a symmetric tensor
 * K_qe per node q of the stiffness rule and element e; the conductivity is then
 * s_qe K_qe (Section 7 with c_q varying over the domain: A_qe = B^{-1} s_qe K_qe B^{-T},
 * a metric per node, which the isoparametric path forms anyway and which covers
 * straight-sided meshes exactly). Exclusive with tensor. Other entry points return
 * QXA_E_UNSUPPORTED when it is set. */
typedef struct {
    int kind;
    int law;
    double value;
    double a[3];
    const double *field;
    const double *tensor;
    const double *tensor_q;
} qxa_coeff;

typedef struct qxa_mesh_s *qxa_mesh;
typedef struct qxa_plan_s *qxa_plan;
typedef struct qxa_graph_s *qxa_graph;
typedef struct qxa_server_s *qxa_server;

typedef struct {
    int dim, order, n_p, n_q_mass, n_q_stiff;
    int64_t n_nodes, n_elem, nnz;
    const int64_t *row_ptr; /* device, [n_nodes+1], borrowed until qxa_plan_destroy */
    const int32_t *col_idx; /* device, [nnz], sorted within each row                */
    size_t device_bytes;    /* device memory held by the plan                       */
    double build_ms;        /* wall time of qxa_plan_create                         */
    int64_t n_tiles;        /* element tiles of the fused kernel                    */
    int64_t n_shared;       /* CSR upper slots summed by the fix-up from partials   */
    int64_t n_partials;     /* partial sums written for those slots                 */
    int64_t n_outputs;      /* sums the fused kernel stores (CSR, carry, partial)   */
    int64_t n_units;        /* 16-byte output units read by the fused kernel        */
    int64_t n_pair_units;   /* of which pair units (two outputs each)               */
    int64_t n_chains;       /* chains of tiles (workgroups of one launch)           */
    int64_t n_carry_reads;  /* outputs that add an earlier tile's carried sum       */
    int64_t n_fix_slots;    /* CSR slots written by the fix-up (both triangles)     */
    int64_t n_ext_units;    /* units of outputs of more than six entries, continued */
    int64_t n_empty_units;  /* units that store nothing (holes of that layout)      */
    int carry_cap;          /* LDS carry entries per workgroup                      */
    int carry_used;         /* most carry entries live at once in a chain           */
    int n_q_mass_kernel;    /* rule sizes of the kernels that run the plan: the     */
    int n_q_stiff_kernel;   /* caller's rules padded with zero-weight nodes         */
} qxa_plan_info;

const char *qxa_last_error(void);
const char *qxa_version(void);

/*
 * Mesh (Section 3, steps 2-3): a conforming mesh of straight-sided simplices
 * of Lagrange order `order` (1..3) in dim = 2 or 3.
 *   coords: SoA [dim][n_nodes] FP64 node coordinates (only the d+1 vertices of
 *           each element are read: the map is affine).
 *   conn:   SoA [n_p][n_elem] int32, n_p = C(order+dim, dim). Local order: the
 *           dim+1 vertices; then order-1 equispaced nodes per edge, edges
 *           (0,1),(1,2),(2,0) in 2D and (0,1),(1,2),(2,0),(0,3),(1,3),(2,3) in
 *           3D, each from the first to the second vertex; then for order 3 one
 *           node per face (2D centroid; 3D faces opposite vertex 3,0,1,2).
 *   mem:    QXA_MEM_HOST or QXA_MEM_DEVICE (where coords/conn live).
 * Validates indices (QXA_E_INDEX), finiteness (QXA_E_NONFINITE) and
 * non-degenerate elements (QXA_E_DEGENERATE, the element id is in the message:
 * B_e must be invertible, Section 3). Copies everything; the caller may free
 * its arrays on return.
 */
qxa_status qxa_mesh_create(int device, int dim, int order, int64_t n_nodes, const double *coords, int64_t n_elem,
                           const int32_t *conn, int mem, qxa_mesh *out);
qxa_status qxa_mesh_destroy(qxa_mesh mesh);

/*
 * Plan (built once per mesh and rule pair): the reference tables Phi, J_q,
 * Q_m, Q_c of Algorithm 2 (only the n_p(n_p+1)/2 rows of distinct
 * symmetric pairs, the symmetry saving of Section 7), the CSR pattern (all
 * (i,j) sharing an element; structural zeros kept), and the element-entry to
 * CSR-slot permutation with its slot-sorted segments that the deterministic
 * scatter uses (the global assembly of Algorithm 2). The mesh must outlive the plan.
 * Rules may differ between the two matrices (Algorithm 2, "Input").
 */
qxa_status qxa_plan_create(qxa_mesh mesh, const qxa_quad *mass_rule, const qxa_quad *stiff_rule, qxa_plan *out);
qxa_status qxa_plan_destroy(qxa_plan plan);
qxa_status qxa_plan_get_info(qxa_plan plan, qxa_plan_info *out);

/* Host-only construction of the CSR pattern (no device needed): with
 * row_ptr == NULL only *nnz is returned; otherwise row_ptr[n_nodes+1] and
 * col_idx[*nnz] (host arrays) are filled. conn is a host SoA array as in
 * qxa_mesh_create; indices are validated (QXA_E_INDEX). */
qxa_status qxa_pattern_host(int dim, int order, int64_t n_nodes, int64_t n_elem, const int32_t *conn,
                            int64_t *row_ptr, int32_t *col_idx, int64_t *nnz);

/* Host-only build and check of the whole plan (pattern, permutation, tile
 * plan of the fused kernel): the plan is executed on the host with exact
 * integer sums (every element entry a pseudo-random 64-bit value) and each
 * CSR slot must receive exactly its element entries; every index the kernels
 * use is in bounds, every CSR slot and partial is written once, and carry
 * entries are race-free within a tile. The same check runs inside
 * qxa_plan_create. chains <= 0 and carry_cap < 0 take the values a plan on
 * an MI355X gets (256 chains, the LDS left beside the kernel). Null rules take the built-in one of
 * degree 2*order; the rules are checked and padded as by qxa_plan_create.
 * `out` (optional) receives the figures qxa_plan_get_info reports, without
 * the device fields (row_ptr and col_idx NULL, device_bytes and build_ms 0). */
qxa_status qxa_plan_check_host(int dim, int order, int64_t n_nodes, const double *coords, int64_t n_elem,
                               const int32_t *conn, const qxa_quad *mass_rule, const qxa_quad *stiff_rule,
                               int64_t chains, int carry_cap, qxa_plan_info *out);

/* Test support for the plan check above (for its callers: the tests that show it
 * rejects broken plans): the plan qxa_plan_check_host builds (built-in rules), with one
 * deliberate corruption, then checked. mutation 1: a CSR output retargeted to the slot
 * of another output of its tile; 2: an entry of an output dropped; 3: an LDS index past
 * the staged pairs (the first carry entry, which no earlier tile wrote); 4: two outputs' entries exchanged; 5: a partial written twice (and
 * another never); 6: a fix-up mirror slot changed. Returns the check's status
 * (QXA_E_INVALID with its message when the corruption is caught), QXA_E_UNSUPPORTED when
 * the plan has nothing the mutation changes (no pair units, no partials), QXA_E_INVALID
 * for a mutation outside 1..6. Host only; needs no GPU. */
qxa_status qxa_plan_check_host_corrupted(int dim, int order, int64_t n_nodes, const double *coords, int64_t n_elem,
                                         const int32_t *conn, int64_t chains, int carry_cap, int mutation);

/* Copy the CSR pattern into caller-owned device arrays row_ptr[n_nodes+1] and
 * col_idx[nnz] (either may be NULL), asynchronously on `stream`. */
qxa_status qxa_plan_copy_pattern(qxa_plan plan, int64_t *row_ptr, int32_t *col_idx, void *stream);

/*
 * One assembly (Algorithm 2 after its reference tables): geometry b, W from the mesh,
 * coefficients S at the quadrature nodes, Lambda, X, V = Q X, then the
 * deterministic segmented-reduction scatter into CSR values (no float
 * atomics; bitwise identical across runs). M_vals / C_vals: caller-owned
 * device arrays of length nnz in the plan's CSR order; either may be NULL to
 * skip that matrix. Asynchronous on `stream`; argument errors are returned
 * immediately, device-detected non-finite coefficients at qxa_sync.
 */
qxa_status qxa_assemble(qxa_plan plan, const qxa_coeff *mass, const qxa_coeff *stiff, int precision, double *M_vals,
                        double *C_vals, void *stream);

/*
 * Formation only (the element matrices of Algorithm 2): V_m and V_c as device arrays
 * [n_p*n_p][n_elem] (entry (i*n_p+j, e) at index (i*n_p+j)*n_elem + e; the
 * element matrices are symmetric so this is also the paper's column-major
 * vec). Either output may be NULL.
 */
qxa_status qxa_element_matrices(qxa_plan plan, const qxa_coeff *mass, const qxa_coeff *stiff, int precision,
                                double *Vm, double *Vc, void *stream);

/*
 * Allocation-free variant of qxa_element_matrices, for callers that cannot
 * allocate device memory: code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc. Same arguments, kernels and results (bitwise)
 * as qxa_element_matrices, which allocates its pair-major staging of V_m, V_c on
 * first use; here that staging lives in a fixed 64 MiB device array of the
 * library (one per GPU, held until the process ends, its address resolved when
 * the first mesh is created on that GPU). It calls no hipMalloc, hipFree or
 * allocating routine. Limit: 2 * n_p(n_p+1)/2 * n_elem <= 8,388,608 doubles,
 * else QXA_E_UNSUPPORTED with a message (e.g. 3D P2: up to 76,260 elements).
 * The staging is fully written before it is read, so nothing needs clearing.
 * All calls on one GPU share the array: calls that overlap in time on one GPU
 * (different streams or host threads) race and must be ordered by the caller.
 */
qxa_status qxa_element_matrices_noalloc(qxa_plan plan, const qxa_coeff *mass, const qxa_coeff *stiff, int precision,
                                        double *Vm, double *Vc, void *stream);

/*
 * Coefficient of the mass tensor contracted with a nodal vector (Section 5, the
 * Newton Jacobian): the mass tensor M_ijk = int m'(u_h) phi_i phi_j phi_k
 * contracted with v in its second mode, (M o_2 v)_ik = int m'(u_h) v_h phi_i phi_k,
 * is the mass matrix of the coefficient s = m'(u_h) v_h; the local tensor
 * (Phi (.) Phi (.) Phi) Lambda contracted with v_e equals (Phi (.) Phi)(Lambda * Phi^T v_e).
 * This call evaluates s at the quadrature nodes of one of the plan's rules:
 *   S[q][e] = law(u_h(xhat_q)) * v_h(xhat_q),  u = c->field, v nodal,
 * for every element in mesh order. Passed to qxa_assemble as a QXA_COEFF_QPOINT
 * mass coefficient with the identity law, S gives M o_2 v in the plan's CSR
 * pattern (symmetric, as M is symmetric in all modes).
 * rule: 0 = the plan's mass rule, 1 = its stiffness rule. c: kind
 * QXA_COEFF_NODAL, its law that of m' (m = a0 + a1 s + a2 s^2 has m' = a1 + 2 a2 s,
 * law poly2 (a1, 2 a2, 0)). v: device [n_nodes]. S: caller-owned device
 * [n_q][n_elem], written asynchronously on `stream`. Errors: QXA_E_INVALID for
 * null pointers, a bad rule index, another kind or a plan owned by a server; a
 * non-finite s is reported by qxa_sync as QXA_E_NONFINITE.
 */
qxa_status qxa_coeff_product(qxa_plan plan, int rule, const qxa_coeff *c, const double *v, double *S, void *stream);

/*
 * Conductivity tensor contracted with a nodal vector in its second mode (Section 5,
 * the Newton Jacobian term): C_ijk = int c'(u_h) grad phi_i . grad phi_j phi_k,
 *   (C o_2 v)_ik = sum_j C_ijk v_j = int c'(u_h) (grad phi_i . grad v_h) phi_k,
 * written as CSR values in the plan's pattern (row i, column k; the result is not
 * symmetric). Per element the local matrix is Q X with Q = [phi_q (x) J_q] and
 * X[(q, c), e] = lambda_q (A_e J_q^T v_e)_c, lambda_q = w_q c'_q |det B_e|, on the
 * plan's stiffness rule; it goes to a plan-owned buffer, and one thread per CSR slot
 * sums the slot's element entries in ascending element order (deterministic).
 * c: kind QXA_COEFF_NODAL with the law of c' (c = a0 + a1 s + a2 s^2 has
 * c' = a1 + 2 a2 s). v: device [n_nodes]. T_vals: caller-owned device [nnz].
 * The first call on a plan builds the slot -> entries map on the host and
 * allocates 8 n_p^2 n_elem + 4 n_p^2 n_elem + 8 (nnz + 1) bytes of device memory,
 * kept until qxa_plan_destroy; later calls allocate nothing. Asynchronous on
 * `stream`. Errors: QXA_E_INVALID (null pointers, another kind, a plan owned by a
 * server), QXA_E_UNSUPPORTED (n_p^2 n_elem >= 2^31), QXA_E_NOMEM; a non-finite
 * c' value is reported by qxa_sync as QXA_E_NONFINITE.
 */
qxa_status qxa_cond_tensor_product(qxa_plan plan, const qxa_coeff *c, const double *v, double *T_vals, void *stream);

/*
 * Volume load vector (Section 2): F_i = int f phi_i, on the plan's mass rule, as
 * the vector analogue of Algorithm 2: element vectors Phi Lambda_f with
 * Lambda_f[q, e] = w_q f_qe |det B_e| (one thread per element, to a plan-owned
 * buffer), then one thread per node sums the node's element entries in ascending
 * element order (deterministic). f: any coefficient (constant, nodal field through
 * a law, values per (q, e) in mesh element order). F: caller-owned device
 * [n_nodes]. The first call on a plan builds the node -> entries map on the host
 * and allocates 12 n_p n_elem + 8 (n_nodes + 1) bytes, kept until
 * qxa_plan_destroy. Asynchronous on `stream`. Errors as qxa_assemble; a non-finite
 * value is reported by qxa_sync as QXA_E_NONFINITE. (The reaction matrix of
 * Section 2, A_ij = int a phi_j phi_i, is the mass matrix of the coefficient a:
 * qxa_assemble with a as the mass coefficient.)
 */
qxa_status qxa_load_vector(qxa_plan plan, const qxa_coeff *f, double *F, void *stream);

/*
 * Isoparametric (curved) elements (Section 7): the element map uses the P-order
 * basis and the positions of all of an element's nodes, x(xhat) = sum_i x_i phi_i(xhat),
 * so B, |det B| and A = B^{-1} K B^{-T} are evaluated at every quadrature node (X_m and
 * X_c per (q, e); Q_m and Q_c unchanged). Same coefficients, outputs and pattern as
 * qxa_assemble, in FP64. One pass where the shape's matrix-core kernel stages Q^T in
 * LDS (2D P2, 2D P3, 3D P2), the plan's mass and stiffness rules are the same rule and
 * the reference gradients fit in LDS beside the plan's carry entries (2D P2, 2D P3 and
 * 3D P2 with their default rules): that kernel forms X per quadrature node from the node
 * positions and reduces V = Q X through the plan's output units, then the fix-up.
 * Otherwise two passes: the local matrices of every element (X per quadrature node,
 * then V = Q X, once per symmetric pair) to a plan-owned buffer in the plan's tile
 * order, then the reduction of the fused assembly (the plan's output units, chains and
 * carries, and its fix-up). Either way every CSR slot is summed in the plan's fixed
 * order (deterministic, bitwise symmetric). The first two-pass call on a plan allocates
 * 16 n_s n_elem bytes of local matrices (n_s = n_p (n_p + 1) / 2, n_elem rounded up to
 * a multiple of 64); later calls, and one-pass calls, allocate nothing. Errors as
 * qxa_assemble, plus, on the two-pass path, QXA_E_UNSUPPORTED when n_s n_elem >= 2^31
 * or when the rules' staging exceeds the LDS, and QXA_E_INVALID for
 * tensor_q on the mass coefficient or with tensor; a non-finite coefficient or tensor
 * entry, or a map with det B_q = 0 at a quadrature node, is reported by qxa_sync as
 * QXA_E_NONFINITE. The stiffness coefficient may carry a per-node tensor (tensor_q).
 */
qxa_status qxa_assemble_iso(qxa_plan plan, const qxa_coeff *mass, const qxa_coeff *stiff, double *M_vals,
                            double *C_vals, void *stream);

/*
 * Per-kernel timing with HIP events recorded on the launch stream around every
 * kernel this plan launches (off by default). qxa_plan_timing_report waits for
 * the recorded events, writes a JSON object
 *   {"<kernel>": {"n": launches, "ms": total milliseconds}, ...}
 * into buf (cap bytes, NUL-terminated) and clears the record.
 */
qxa_status qxa_plan_set_timing(qxa_plan plan, int enable);
qxa_status qxa_plan_timing_report(qxa_plan plan, char *buf, size_t cap);

/*
 * Reassembly graph (Section 5, summary: only the coefficient matrix S depends
 * on the unknown, so Q, W, b and the sparsity data are reused and only the
 * launches are replayed). Captures one qxa_assemble with these arguments into
 * a HIP graph: the coefficient field pointers and the output arrays are baked
 * in, so the caller updates the field contents in place between replays (on
 * the replay stream, or synchronised with it). Outputs are overwritten by
 * every replay and are bitwise equal to a direct qxa_assemble of the same
 * inputs. The graph borrows the plan and the buffers; destroy it first.
 */
qxa_status qxa_graph_create(qxa_plan plan, const qxa_coeff *mass, const qxa_coeff *stiff, int precision,
                            double *M_vals, double *C_vals, qxa_graph *out);
qxa_status qxa_graph_launch(qxa_graph graph, void *stream);
qxa_status qxa_graph_destroy(qxa_graph graph);

/*
 * Serving: a continuous-batching assembly loop run by a worker thread of the
 * library, for many independent jobs (mesh + rules + coefficients).
 *
 * - qxa_server_submit queues a job and returns a ticket at once (QXA_E_BUSY
 *   when queue_capacity jobs are waiting).
 * - Admission, in arrival order, takes an in-flight slot (max_inflight) and
 *   the job's device buffers (both CSR value arrays, partial sums, a status
 *   word) from a device-memory budget of hbm_budget_bytes, which also holds
 *   the resident plans. The budget is one device allocation made at creation;
 *   nothing in the serving loop allocates or frees device memory. A job that
 *   does not fit waits until released results or evicted plans make room;
 *   when only its own plan is left and the plan's buffers split the free
 *   space, the plan is rebuilt into the empty budget; QXA_E_NOMEM only when it
 *   cannot fit even in an otherwise empty budget.
 * - Plans (pattern, permutation, tiles, reference tables) stay resident in an
 *   LRU cache keyed by mesh and rule pair: only S changes between assemblies
 *   of one mesh (Section 5, summary), so a cache hit skips the plan build.
 *   Plans of new meshes are built by plan_builders host threads while other
 *   jobs run (a small mesh need not wait behind a large one).
 *   Unreferenced plans are evicted (least recently used first) when the
 *   budget is short or more than plan_cache_entries are resident.
 * - Admitted jobs with fewer than batch_tile_limit element tiles that share a
 *   kernel (dim, order, rules, precision QXA_FP64 or QXA_FP32) run together
 *   in one persistent launch: a device job table maps each global tile to
 *   (job, tile). Other jobs launch alone. Launches rotate over n_streams
 *   streams (default priority) so that they overlap.
 * - Each job's values are bitwise identical to qxa_assemble of the same job
 *   alone: every CSR slot is summed by one thread in a fixed order, whatever
 *   the batch.
 * - qxa_server_poll returns completed jobs (including failed ones, with their
 *   status). Every polled ticket must be released with qxa_server_release,
 *   which returns its buffers to the budget. Results live on the device.
 * A mesh must outlive its jobs and resident plans: once every job on it is
 * released, qxa_server_drop_mesh frees its plans and the mesh may be
 * destroyed. Coefficient fields must stay valid and unchanged until the job
 * completes. One server per device; all functions are thread-safe.
 */
typedef struct {
    int device;
    size_t hbm_budget_bytes;  /* plans + job buffers (0: 4 GiB)                       */
    int max_inflight;         /* admitted, not yet completed jobs (0: 64)             */
    int n_streams;            /* streams launches rotate over (0: 4)                  */
    int64_t batch_tile_limit; /* jobs with fewer tiles are batched (0: 512)           */
    int queue_capacity;       /* waiting jobs beyond which submit fails (0: 65536)    */
    int plan_cache_entries;   /* resident plans kept (0: bounded by the budget only)  */
    int plan_builders;        /* host threads building plans of new meshes (0: 4)     */
} qxa_server_opts;

typedef struct {
    qxa_mesh mesh;
    qxa_quad mass_rule, stiff_rule; /* host arrays, copied at submit                  */
    qxa_coeff mass, stiff;          /* device fields read when the job runs           */
    int precision;                  /* a qxa_precision                                */
    uint64_t user_tag;              /* returned with the completion                   */
} qxa_job;

typedef struct {
    uint64_t ticket, user_tag;
    int status;               /* QXA_OK or the job's error                          */
    int plan_cached;          /* 1: the plan was resident when the job arrived      */
    int batched;              /* jobs in the launch that ran this one               */
    int64_t n_nodes, nnz;
    const double *M, *C;      /* device [nnz], valid until the ticket is released   */
    const int64_t *row_ptr;   /* device [n_nodes+1], valid until released           */
    const int32_t *col_idx;   /* device [nnz]                                       */
    double queue_ms;          /* submit -> launch (host clock)                      */
    double run_ms;            /* its launch on the device (HIP events)              */
    double total_ms;          /* submit -> completion seen by the server            */
    double plan_ms;           /* submit -> its plan resident (0 for a resident plan) */
    char message[160];        /* error text when status != QXA_OK                   */
} qxa_completion;

qxa_status qxa_server_create(const qxa_server_opts *opts, qxa_server *out);
qxa_status qxa_server_submit(qxa_server server, const qxa_job *job, uint64_t *ticket);
/* Up to `max` completions in completion order; *n_done = how many. */
qxa_status qxa_server_poll(qxa_server server, qxa_completion *done, int max, int *n_done);
/* Copies a completed job's values into caller device buffers (either may be NULL),
 * asynchronously on `stream`; an event recorded there after the copies is kept with
 * the ticket. */
qxa_status qxa_server_copy_result(qxa_server server, uint64_t ticket, double *M_vals, double *C_vals, void *stream);
/* Returns a polled job's buffers to the budget. It first waits for every copy that
 * qxa_server_copy_result queued for this ticket, so the copied values are never
 * those of a later job that reuses the buffer; no synchronisation of the copy stream
 * is needed before it. The job's device pointers (qxa_completion.M, .C) are invalid
 * afterwards. */
qxa_status qxa_server_release(qxa_server server, uint64_t ticket);
/* paused != 0: admit nothing (submissions still queue); 0: resume. */
qxa_status qxa_server_pause(qxa_server server, int paused);
/* Frees the resident plans of `mesh` (a client done with a mesh, for instance a
 * request that brought a new one), after which the caller may destroy it.
 * QXA_E_BUSY while a job on the mesh is queued, running or not released, or a
 * plan of it is being built. */
qxa_status qxa_server_drop_mesh(qxa_server server, qxa_mesh mesh);
/* counters: [0] submitted [1] completed [2] plan-cache hits [3] plan builds
 * [4] evictions [5] launches [6] batched launches [7] most jobs in one launch
 * [8] budget bytes in use [9] peak bytes in use [10] queued [11] in flight
 * [12] budget bytes */
qxa_status qxa_server_stats(qxa_server server, int64_t *counters, int n);
/* Waits for launched work, drops jobs not yet launched, frees everything. */
qxa_status qxa_server_destroy(qxa_server server);

/* Wait for `stream` and report device-side conditions (QXA_E_NONFINITE). */
qxa_status qxa_sync(qxa_plan plan, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QXA_H */
