/*
 * mbem -- MI355X (gfx950) library for the nodal P2 Mueller boundary-element
 * method of Y. Luo, "A High-Order Nodal Galerkin Formulation for the Mueller
 * Equation: Bypassing Divergence Conformity via Kernel Cancellation"
 * (arXiv 2604.21181).
 *
 * The library fills the dense complex Galerkin matrix Z of the global
 * system (Sec. 4.3, eq. global_system)
 *
 *        [ (i/w) K1             (eps_i+eps_a)/2 M + K2^eps ] [ c_j  ]   [ b_E ]
 *        [ (mu_i+mu_a)/2 M + K2^mu       -(i/w) K1         ] [ c_jm ] = [ b_H ]
 *
 * over every pair of curved P2 triangles (regular pairs by a 7-point rule,
 * coincident / common-edge / common-vertex pairs by Sauter-Schwab
 * quadrature, Sec. 4.1-4.2 and 6.1), applies it, and solves it with GMRES
 * right-preconditioned by the Morton block-Jacobi matrix (Sec. 5).
 *
 * Conventions
 *  - Every function returns MBEM_OK (0) or a negative mbem_status; the
 *    message of the last failure on the calling thread is mbem_last_error().
 *    No C++ exception crosses this interface.
 *  - Units: exterior medium vacuum, eps_a = mu_a = 1, eta_a = 1,
 *    omega = k_a = k0; k_i = k0 sqrt(eps_r mu_r) with Im k_i >= 0.
 *  - Ownership: the library owns the handles and everything they allocate;
 *    the caller owns every pointer argument and the library never frees
 *    caller memory.  "device" pointers are HIP device memory on the
 *    context's device (e.g. torch tensor data pointers), "host" pointers are
 *    ordinary host memory.
 *  - Streams: all device work is enqueued on the context's stream (borrowed,
 *    never destroyed by the library).  Functions that write host outputs
 *    synchronise that stream before returning.
 *  - Ordering: the library renumbers nodes and triangles in Morton (Z-order)
 *    order (Sec. 5).  All device vectors (right-hand sides, solutions) are
 *    in that order: x = [c_j ; c_jm], each block of length 2 n_nodes with
 *    index 2 m + alpha, m the Morton position of the node and alpha in {0,1}
 *    selecting the tangent t_1 or t_2.  mbem_mesh_permutation() maps the
 *    caller's numbering to Morton positions.  N = 4 n_nodes unknowns.
 *  - Complex numbers are interleaved (re, im) pairs: mbem_c128 is two
 *    doubles (C99 double _Complex, torch.complex128); "c64" buffers are two
 *    floats (torch.complex64).
 */
#ifndef MBEM_H
#define MBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } mbem_c128;

typedef enum {
    MBEM_OK = 0,
    MBEM_EINVAL = -1,     /* bad argument, size or handle                 */
    MBEM_ENOMEM = -2,     /* device or host allocation failed             */
    MBEM_EDEVICE = -3,    /* HIP runtime error                             */
    MBEM_ENOCONV = -4,    /* iteration limit reached; outputs still valid  */
    MBEM_ESINGULAR = -5,  /* zero pivot in a preconditioner block          */
    MBEM_EMESH = -6       /* mesh is not a closed, oriented P2 2-manifold  */
} mbem_status;

typedef enum {
    MBEM_FP64 = 0,   /* all pairs in FP64, Z stored complex128             */
    MBEM_MIXED = 1   /* far regular pairs in FP32, near and singular pairs
                        in FP64, Z stored complex64 (or, with near_store,
                        the near and singular part in an FP64 sparse store
                        beside it); FP64 Arnoldi and an FP64-accumulated
                        refinement residual                               */
} mbem_precision;

typedef struct mbem_ctx mbem_ctx;    /* device ordinal + borrowed stream      */
typedef struct mbem_mesh mbem_mesh;  /* Morton-ordered mesh, device tables    */
typedef struct mbem_op mbem_op;      /* filled operator + preconditioner      */

typedef struct {
    double k0;                  /* vacuum wavenumber = omega                 */
    double eps_r_re, eps_r_im;  /* interior relative permittivity            */
    double mu_r_re, mu_r_im;    /* interior relative permeability            */
    int32_t ssq_order;          /* Gauss points per dimension of the
                                   Sauter-Schwab rule (0 -> 4, Sec. 6.1)     */
    int32_t precision;          /* mbem_precision                            */
    double near_radius;         /* MIXED: element pairs whose gap is below
                                   this are computed in FP64; <= 0 selects
                                   1.89 / sqrt|k_a^2 - k_i^2|                */
    int32_t quadrature;         /* MBEM_QUAD_DEFAULT or MBEM_QUAD_PAPER      */
    int32_t frame;              /* MBEM_FRAME_INTERPOLATED or MBEM_FRAME_NODAL */
    int32_t near_store;         /* MIXED, default quadrature: 1 keeps the
                                   near and singular element pairs' part of
                                   Z in FP64 (see below); 0 rounds it into
                                   the complex64 blocks.  Ignored for FP64  */
} mbem_params;

/* The FP64 near store (MIXED with near_store = 1).  The kernel differences
 * cancel as R -> 0 (Sec. 2.3), so the element pairs closer than the near
 * radius and the singular pairs are evaluated in FP64; with the store their
 * contributions are also accumulated and kept in FP64: for every node pair
 * (i, j) touched by such an element pair, a 2 x 2 (alpha, beta) block of
 * K1, K2^eps and K2^mu in complex128 on the node-pair pattern of those
 * pairs (built on the device at every fill), while the far element pairs
 * go to the complex64 blocks.  Z = complex64 blocks + store.  The products
 * (mbem_matvec, the solves' residuals, the transposed product), the
 * block-Jacobi blocks and the exports read both.  mbem_solve_block folds
 * the store into the complex64 blocks first (its block product runs on
 * complex64 entries).                                                      */

/* Quadrature of the operator blocks.
 * MBEM_QUAD_DEFAULT: the 7-point rule on every regular element pair (closed
 *   forms, or the Taylor series to n = 16 below max|k| R = 1/2), Sauter-
 *   Schwab on the full kernels of every singular pair.
 * MBEM_QUAD_PAPER: the paper's own scheme (Sec. 4.1-4.2, 6.1): the 12-point
 *   degree-6 rule on every regular pair with the closed-form kernels;
 *   Sauter-Schwab on the singular kernels kappa^s only (their terms of
 *   negative order in R), the remainder kappa - kappa^s by the 12-point rule
 *   on the same pair with the Taylor series truncated after n = 6.  Fill and
 *   solve only: mbem_fill_deps and mbem_grad_sigma_ext reject it.          */
enum { MBEM_QUAD_DEFAULT = 0, MBEM_QUAD_PAPER = 1 };

/* Tangential basis.
 * MBEM_FRAME_INTERPOLATED: the basis function of node j, component beta, is
 *   N_j(y) t_beta(y) with t_beta(y) the continuous frame of Sec. 3.3 (nodal
 *   triads of Sec. 3.2 interpolated, projected on the tangent plane at y and
 *   Gram-Schmidt orthonormalised); test functions alike (Sec. 4.1).  Where a
 *   triangle's nodes took different reference axes (Sec. 3.2) this frame
 *   turns fast inside the triangle, and far fields converge at about O(h).
 * MBEM_FRAME_NODAL: node-attached tangents, N_j(y) P(y) t_beta,j with
 *   t_beta,j the node's own triad tangent and P(y) = I - n(y) n(y)^T; the
 *   rotated test vector is t_alpha,i x n(x).  Same kernels (Sec. 4), same
 *   unknown layout; the mass matrix couples alpha and beta.  Its span does
 *   not depend on the reference-axis choice and far fields converge at high
 *   order.  Either quadrature; every entry point takes it except
 *   mbem_grad_sigma_ext's shape outputs with the paper quadrature (the
 *   gradient is built for the default quadrature).
 * Post-processing calls (right-hand side, far field, cross sections, far-
 * field functional) take the same value as the fill of the solution.      */
enum { MBEM_FRAME_INTERPOLATED = 0, MBEM_FRAME_NODAL = 1 };

typedef struct {
    double tol;          /* relative residual target |b - Z x| / |b|, met by
                            the explicit FP64-accumulated residual          */
    int32_t maxit;       /* GMRES iteration limit (Krylov dimension)         */
    int32_t max_refine;  /* MIXED: outer refinement sweeps (0 -> 8); FP64:
                            GMRES runs in all, the first on b and the others
                            from the explicit residual when the Arnoldi
                            estimate met tol but the explicit residual did
                            not (0 -> 3)                                     */
    double inner_tol;    /* MIXED: inner GMRES tolerance (0 -> max(tol, 1e-8)) */
} mbem_solve_opts;

typedef struct {
    int32_t iters;        /* GMRES iterations (sum over refinement sweeps)   */
    int32_t outer_iters;  /* refinement sweeps (MIXED), 1 otherwise          */
    double rel_resid;     /* final |b - Z x| / |b| (FP64 accumulation)       */
    double t_fill_ms;     /* geometry tables + all pair classes + mass       */
    double t_setup_ms;    /* preconditioner gather + LU + inverse             */
    double t_solve_ms;    /* GMRES wall time                                 */
    int64_t n_near_pairs; /* MIXED: regular pairs computed in FP64           */
    /* device time of single launches, from HIP events on the context stream */
    double t_geom_ms;     /* nodal frames + quadrature-point tables           */
    double t_regular_ms;  /* regular-pair kernel (FP64 path: all regular
                             pairs; MIXED: the FP32 far-pair launch)         */
    double t_near_ms;     /* MIXED: the FP64 near-pair launch                 */
    double t_ssq_ms;      /* Sauter-Schwab kernel                            */
    double t_mass_ms;     /* mass matrix                                     */
    double t_matvec_ms;   /* solve: sum of the timed dense GEMV kernel times
                             (the products of the third and fourth Arnoldi
                             steps of every GMRES run: a sample, not the
                             total)                                          */
    int32_t n_matvec;     /* solve: number of GEMV launches timed             */
    int64_t n_regular_pairs; /* regular element pairs (all launches)          */
    /* mbem_grad_sigma_ext: wall times of its phases                          */
    double t_adjoint_ms;  /* Z^T lambda = g                                   */
    double t_deps_ms;     /* dZ/deps_r fill and lambda^T dZ x                 */
    double t_shape_ms;    /* reverse pass over the geometry                   */
} mbem_stats;

/* ---- context ---------------------------------------------------------- */

/* Bind a context to HIP device `device` and the caller's stream
 * (hipStream_t passed as void*, NULL = the null stream).                    */
int mbem_ctx_create(int device, void *hip_stream, mbem_ctx **out);
void mbem_ctx_destroy(mbem_ctx *ctx);

/* ---- mesh (Sec. 3 and 5) ------------------------------------------------ */

/* Host preprocessing: validates that the triangles form a closed, oriented
 * P2 2-manifold (every edge shared by exactly two triangles with opposite
 * orientation and the same mid-edge node), applies the double Morton
 * permutation (nodes, then triangles by vertex centroid; Sec. 5), builds
 * the singular-pair lists (coincident, common edge, common vertex;
 * Sec. 4.2) and copies the mesh to the device.
 *   xyz   host [n_nodes*3] float64, node coordinates
 *   tri6  host [n_tris*6] int64, nodes (v0 v1 v2 m01 m12 m20), counter-
 *         clockwise seen from outside
 * Errors: MBEM_EINVAL (sizes, indices), MBEM_EMESH (topology).            */
int mbem_mesh_create(mbem_ctx *ctx, const double *xyz, int64_t n_nodes,
                     const int64_t *tri6, int64_t n_tris, mbem_mesh **out);
void mbem_mesh_destroy(mbem_mesh *mesh);

/* Nodal frames (Sec. 3.1-3.2): metric-weighted normal n, t1 = normalize(
 * v_ref x n) with v_ref = x if |n.z| > 0.9 else z, t2 = n x t1.
 *   frames host [n_nodes*9] float64 (n, t1, t2 per node, caller's order).  */
int mbem_mesh_frames(mbem_ctx *ctx, const mbem_mesh *mesh, double *frames);

/* host outputs: node_order[m] = caller's node at Morton position m,
 * tri_order[t] = caller's triangle at Morton position t (either may be
 * NULL).                                                                    */
int mbem_mesh_permutation(const mbem_mesh *mesh, int64_t *node_order,
                          int64_t *tri_order);

/* host output info[8] = {n_nodes, n_tris, n_unknowns, coincident pairs,
 * common-edge ordered pairs, common-vertex ordered pairs, 0, 0}.            */
int mbem_mesh_info(const mbem_mesh *mesh, int64_t *info);

/* The Morton permutation alone, on the host, without a device (Sec. 5):
 * keys from the bounding box's largest side, 21 bits per axis, x in bit 3b,
 * y in 3b+1, z in 3b+2; stable sort.  Same outputs as
 * mbem_mesh_permutation().                                                  */
int mbem_morton_order(const double *xyz, int64_t n_nodes, const int64_t *tri6,
                      int64_t n_tris, int64_t *node_order, int64_t *tri_order);

/* ---- fill (Sec. 4, 6.1) ---------------------------------------------------- */

/* Geometry tables (metric-weighted nodal normals and frames, Sec. 3;
 * quadrature-point frames), every element pair (K1, K2^eps, K2^mu; eqs.
 * K1_matrix_entry, K2_matrix_entry) and the mass matrix (eq. mass_matrix).
 * stats may be NULL; t_fill_ms and n_near_pairs are written.               */
int mbem_fill(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *params,
              mbem_op **out, mbem_stats *stats);
void mbem_op_destroy(mbem_op *op);

/* Copy the operator blocks K1, K2^eps, K2^mu ((2 n_nodes)^2 each,
 * row-major, Morton order) to device buffers of complex128.  Any pointer
 * may be NULL.                                                              */
int mbem_op_export_blocks(mbem_ctx *ctx, const mbem_op *op, mbem_c128 *K1,
                          mbem_c128 *K2e, mbem_c128 *K2m);

/* Dense Z (N x N, row-major, Morton order) into a device complex128 buffer. */
int mbem_op_export_dense(mbem_ctx *ctx, const mbem_op *op, mbem_c128 *Z);

/* y = Z x for nrhs column-major device vectors of length N (complex128).   */
int mbem_matvec(mbem_ctx *ctx, const mbem_op *op, const mbem_c128 *x,
                int32_t nrhs, mbem_c128 *y);

/* y = Z x like mbem_matvec, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no allocation or release of any kind and no host wait -- the
 * products are enqueued on the context's stream and the call returns; the
 * caller synchronises before reading y.  The partial sums live in a 4 MiB
 * array in device memory that the library holds on every device it runs
 * on until the process ends, so op must have 2 n_nodes <= 65536 (MBEM_EINVAL
 * otherwise, nothing enqueued).  Every call on one device uses that
 * device's one array: calls that overlap on a device (other streams,
 * other threads) race and must be serialised by the caller.               */
int mbem_matvec_noalloc(mbem_ctx *ctx, const mbem_op *op, const mbem_c128 *x,
                        int32_t nrhs, mbem_c128 *y);

/* ---- preconditioner (Sec. 5, eq. precond_block) --------------------------- */

/* Morton block-Jacobi: clusters of `block` consecutive indices of one
 * current's vector (block <= 512); each block is the 2 block x 2 block
 * restriction of Z, LU-factorised with partial pivoting (blocked, in FP64)
 * and inverted explicitly (the apply is then one matrix-vector product).
 * MBEM_ESINGULAR on a zero pivot, MBEM_EINVAL for block > 512.
 * block <= 0 removes the preconditioner.                                   */
int mbem_precond_setup(mbem_ctx *ctx, mbem_op *op, int32_t block,
                       mbem_stats *stats);

/* z = P^-1 v (device, length N, complex128): one product of every block's
 * explicit inverse with its 2 block entries of v.                          */
int mbem_precond_apply(mbem_ctx *ctx, const mbem_op *op, const mbem_c128 *v,
                       mbem_c128 *z);

/* ---- excitation, solve, post-processing ------------------------------------ */

/* b = [b_E ; b_H] (eqs. rhs_E, rhs_H) for plane waves
 * E = pol e^{i k_a khat.x}, H = khat x E.
 *   khat  host [nrhs*3] unit directions;  pol host [nrhs*3] complex
 *   b     device [N*nrhs] complex128, column-major                         */
int mbem_rhs_planewave(mbem_ctx *ctx, const mbem_mesh *mesh,
                       const mbem_params *params, const double *khat,
                       const mbem_c128 *pol, int32_t nrhs, mbem_c128 *b);

/* Solve Z x = b by GMRES (x0 = 0, classical Gram-Schmidt twice in FP64,
 * right-preconditioned by the Morton block-Jacobi matrix if set up; Sec. 5).
 * For a MIXED operator the inner GMRES applies the complex64 matrix and an
 * outer FP64-accumulated residual refines x.  b, x: device [N*nrhs]
 * complex128.  A column is converged when its explicit residual
 * |b - Z x| / |b| (FP64 accumulation) is at most tol; a zero column gives
 * x = 0.  MBEM_EINVAL if a column of b is not finite (nothing is solved);
 * MBEM_ENOCONV if some column did not converge within maxit (and the
 * refinement sweeps): x holds the last iterate and stats->rel_resid the
 * worst explicit residual.                                                 */
int mbem_solve(mbem_ctx *ctx, mbem_op *op, const mbem_c128 *b, int32_t nrhs,
               const mbem_solve_opts *opts, mbem_c128 *x, mbem_stats *stats);

/* ---- adjoint and gradients of sigma_ext (extension of Sec. 6) ------------- */

/* Solve Z^T lambda = g (transpose, no conjugation) by the same GMRES
 * (right-preconditioned by the transposed block-Jacobi matrix; MIXED
 * operators refine in FP64 as mbem_solve).  g, lambda device [N*nrhs].      */
int mbem_solve_adjoint(mbem_ctx *ctx, mbem_op *op, const mbem_c128 *g,
                       int32_t nrhs, const mbem_solve_opts *opts,
                       mbem_c128 *lambda, mbem_stats *stats);

/* Fill dZ/d eps_r at fixed k_0, mu_r (FP64): the same Galerkin quadrature
 * as mbem_fill applied to the derivatives of the kernel differences with
 * respect to eps_i through k_i = k_0 sqrt(eps_r mu_r) and the eps_i factor
 * of G_eps (Sec. 2.3 and 4), plus the derivative (1/2) M of the mass term.
 * The returned operator works with mbem_matvec and the export calls.       */
int mbem_fill_deps(mbem_ctx *ctx, const mbem_mesh *mesh,
                   const mbem_params *params, mbem_op **out,
                   mbem_stats *stats);

/* g (device [N] complex128) with g^T x = e . F(rhat) for every solution x,
 * F the far-field amplitude of mbem_farfield.  rhat, e host [3].          */
int mbem_farfield_functional(mbem_ctx *ctx, const mbem_mesh *mesh,
                             const mbem_params *params, const double *rhat,
                             const mbem_c128 *e, mbem_c128 *g);

/* sigma_ext = (4 pi / k_a) Im(conj(pol) . F(khat)) of the solution x of
 * Z x = b(khat, pol) and its derivatives by the adjoint method:
 *   lambda: Z^T lambda = g (g from mbem_farfield_functional, e = conj pol),
 *   d sigma / d eps_r = (4 pi / k_a) (-lambda^T (dZ/deps_r) x)  (holomorphic:
 *   d/dRe eps_r = Im, d/dIm eps_r = Re of the bracket times 4 pi / k_a),
 *   d sigma / d theta = (4 pi / k_a) d/dtheta Im(g^T x + lambda^T b
 *   - lambda^T Z x) with x, lambda frozen for the node positions theta: a
 *   reverse pass over every quadrature point and point pair of the fill
 *   (regular and Sauter-Schwab), the P2 map, the continuous frame and the
 *   nodal triads and normals (Sec. 3), with the singular-pair classes and
 *   the reference-vector choice of every node held fixed.
 *   disp_dir host [n_nodes*3] float64 or NULL: displacement direction d_v
 *     of every node (Morton order); NULL selects the nodal normals n_v of
 *     this mesh (Sec. 3.1).  A caller that displaced the nodes along the
 *     normals of an earlier mesh passes those normals here;
 *   out host [3]: sigma_ext, d/dRe eps_r, d/dIm eps_r;
 *   lambda_out device [N] or NULL;
 *   dsig_dnode device [n_nodes] float64 or NULL: derivative for the
 *     displacement x_v -> x_v + delta_v d_v of node v (Morton order);
 *   dsig_dx device [n_nodes*3] float64 or NULL: derivative for every
 *     coordinate of every node (Morton order);
 *   stats: the adjoint solve.
 * params and op must use the same frame and mesh must be op's mesh (EINVAL
 * otherwise, and for non-finite disp_dir).  With
 * MBEM_FRAME_NODAL the reverse pass goes through the projections of the
 * node-attached fields and the nodal triads instead of the point frame.    */
int mbem_grad_sigma_ext(mbem_ctx *ctx, mbem_op *op, const mbem_mesh *mesh,
                        const mbem_params *params, const mbem_c128 *x,
                        const double *khat, const mbem_c128 *pol,
                        const double *disp_dir,
                        const mbem_solve_opts *opts, double *out,
                        mbem_c128 *lambda_out, double *dsig_dnode,
                        double *dsig_dx, mbem_stats *stats);

/* ---- many right-hand sides (Sec. 5 and 6: block Krylov extension) ------- */

typedef struct {
    double tol;          /* per column: |b - Z x| <= tol |b| (FP64 residual) */
    double inner_tol;    /* reduction of every column per refinement sweep
                            (0 -> 1e-5)                                      */
    int32_t maxit;       /* block iterations per sweep (0 -> 60)            */
    int32_t max_refine;  /* refinement sweeps (0 -> 10)                      */
    int32_t block;       /* columns per block, <= 32 and dividing nrhs
                            (0 -> the largest such divisor)                  */
    int32_t gemm_config; /* FP32 GEMM tile shape 0..5; -1 -> autotuned      */
} mbem_block_opts;

typedef struct {
    int32_t iters;       /* block iterations summed over sweeps             */
    int32_t sweeps;      /* refinement sweeps                                */
    int32_t block;       /* columns per block used                           */
    int32_t gemm_config; /* FP32 GEMM tile shape used                        */
    double rel_resid;    /* max over columns of |b - Z x| / |b|              */
    double t_solve_ms;   /* wall time of the call                            */
    double t_gemm_ms;    /* sum of the block matrix-product GEMM launches    */
    int32_t n_gemm;      /* number of those launches                         */
    int32_t shifted;     /* 1 if a Cholesky QR needed a diagonal shift       */
} mbem_block_stats;

/* Solve Z X = B for nrhs columns at once: block GMRES right-preconditioned
 * by the Morton block-Jacobi matrix (if set up), blocks of `block` columns
 * sharing every launch; the dense part of each block product Z P^-1 V runs
 * as one complex FP32 GEMM on the matrix cores (an FP64 operator is copied
 * to complex64 once for this), the Arnoldi process (classical Gram-Schmidt
 * twice, Cholesky QR twice) in FP64, and an outer FP64 residual B - Z X of
 * the stored operator refines X.
 *   b, x device [nrhs][N] complex128 (x overwritten, x0 = 0)
 * Errors: MBEM_EINVAL (block size, a zero column of b), MBEM_ENOMEM,
 * MBEM_ENOCONV (x holds the last iterate).                                  */
int mbem_solve_block(mbem_ctx *ctx, mbem_op *op, const mbem_c128 *b,
                     int32_t nrhs, const mbem_block_opts *opts, mbem_c128 *x,
                     mbem_block_stats *stats);

/* Time every FP32 GEMM tile shape on the block product of `op` with nrhs
 * columns (a warm-up and `reps` timed launches each) and keep the fastest in
 * the context for later calls of mbem_solve_block with nrhs columns on
 * operators of the same size (mbem_solve_block tunes by itself when the
 * context holds no choice for its size).
 *   ms host [6] (best time of each shape, may be NULL); best host [1].     */
int mbem_gemm_autotune(mbem_ctx *ctx, mbem_op *op, int32_t nrhs, int32_t reps,
                       float *ms, int32_t *best);

/* The complex GEMM of the block solve on its own:
 *   C[b][m] = sum_k op(A[m][k]) B[b][k],  m < M, b < Nb, k < K,
 * all row-major device arrays (leading dimensions in elements).
 *   dtype 0: complex64 A, B, C, FP32 accumulation (matrix cores; three
 *            real products per complex one: (A_re + A_im) B_re,
 *            A_re (B_im - B_re), A_im (B_re + B_im)), tile shape `config`
 *            (0..5), conj_a must be 0; lda, ldb even and A, B 16-byte
 *            aligned;
 *   dtype 1: complex128 A, B, C, FP64 accumulation (matrix cores);
 *   dtype 2: complex64 A, complex128 B and C, FP64 accumulation.
 * op = conj when conj_a (dtypes 1 and 2).                                   */
int mbem_cgemm(mbem_ctx *ctx, int32_t dtype, int32_t conj_a, int64_t M,
               int64_t Nb, int64_t K, const void *A, int64_t lda,
               const void *B, int64_t ldb, void *C, int64_t ldc,
               int32_t config);

/* Far-field amplitude F(r) of the solution currents, E_s ~ F e^{ik r}/r:
 * F = (i k_a / 4 pi) r x sum_qp w J e^{-i k_a r.y} (eta_a j x r - j_m).
 *   x device [N*nrhs]; rhat device [ndir*3]; F device [nrhs][ndir][3]
 *   complex128.                                                            */
int mbem_farfield(mbem_ctx *ctx, const mbem_mesh *mesh,
                  const mbem_params *params, const mbem_c128 *x, int32_t nrhs,
                  const double *rhat, int64_t ndir, mbem_c128 *F);

/* Cross sections of one solution for unit incidence (khat, pol host [3]):
 * out[0] = C_ext (optical theorem), out[1] = C_sca (Gauss-Legendre in
 * cos theta x trapezoid in phi, ntheta x 2 ntheta directions),
 * out[2] = C_abs = Re int n.(j_m x conj j).  out host [3].                 */
int mbem_cross_sections(mbem_ctx *ctx, const mbem_mesh *mesh,
                        const mbem_params *params, const mbem_c128 *x,
                        const double *khat, const mbem_c128 *pol,
                        int32_t ntheta, double *out);

/* ---- block low-rank operator (compressed far interactions) ---------------- */

/* The paper leaves compressed far-field interactions to future work (Sec. 7, Conclusion);
 * this operator stores far tiles of K1, K2^eps, K2^mu in low-rank form.
 * Clusters: the leaves of the octree of the nodes' Morton keys (Sec. 5),
 * cells of more than `cluster` nodes split into their eight children, each
 * leaf a run of the Morton order; a cluster's support box bounds the nodes
 * of every element touching it; a cluster pair
 * is admissible when its boxes are apart and max(diam) <= eta * dist.  Every
 * admissible tile is approximated by adaptive cross approximation with
 * partial pivoting to relative Frobenius accuracy eps (at most rmax terms);
 * it is kept low-rank when that converged and stores less than the dense
 * tile (or always, keep_lowrank = 1), else dense.  Other tiles are dense.
 * The dense operator is never formed: rows are filled one band of whole
 * clusters at a time into a scratch of 3 x 2(band + halo) x 2 n_nodes
 * entries, and every cluster's tiles are approximated from them.            */
typedef struct {
    int32_t cluster;       /* largest nodes per cluster, 1..2048            */
    double eta;            /* admissibility parameter, > 0                  */
    double eps;            /* cross-approximation tolerance, (0, 1)         */
    int32_t rmax;          /* largest rank, 1..128                          */
    int32_t keep_lowrank;  /* 1: keep every converged approximation low-rank */
    int32_t band;          /* nodes per row band of the assembly (whole
                              clusters); 0: about 16 GB of band buffers      */
} mbem_blr_opts;

typedef struct {
    int64_t stored_bytes;  /* dense and low-rank tiles                      */
    int64_t dense_bytes;   /* the three dense blocks it stands for          */
    int32_t n_clusters;
    int32_t n_tiles;       /* 3 n_clusters^2                                */
    int32_t n_admissible;  /* admissible tiles (all three blocks)           */
    int32_t n_lowrank;     /* tiles stored low-rank                         */
    int32_t max_rank;
    double mean_rank;      /* over the low-rank tiles                       */
    double t_fill_ms;      /* band fills (regular and singular pairs)       */
    double t_aca_ms;       /* cross approximation                           */
    double t_total_ms;     /* the whole call                                */
} mbem_blr_stats;

/* Fill a block low-rank operator (FP64, default quadrature only).  The
 * returned operator works with mbem_matvec, mbem_precond_setup/apply,
 * mbem_solve and mbem_op_export_blocks (which expands it; small meshes);
 * mbem_op_export_dense, mbem_solve_adjoint, mbem_solve_block,
 * mbem_gemm_autotune and mbem_grad_sigma_ext reject it (MBEM_EINVAL).  The
 * far field and cross sections take the solution only.  MBEM_EINVAL for
 * options out of range, MBEM_ENOMEM when the band scratch or the tiles do
 * not fit.  stats may be NULL (t_fill_ms: the whole call); bstats may be
 * NULL.                                                                     */
int mbem_fill_compressed(mbem_ctx *ctx, const mbem_mesh *mesh,
                         const mbem_params *params, const mbem_blr_opts *opts,
                         mbem_op **out, mbem_stats *stats,
                         mbem_blr_stats *bstats);

/* ---- spectrum sweep (Sec. 6.3, Benchmark II: the LSPR spectrum) ----------- */

/* The single-frequency path repeated over npts (k0, eps_r, mu_r) points on
 * one mesh for one plane wave: at each point the operator is refilled in
 * place (the geometry tables are built once for the sweep), the block-
 * Jacobi preconditioner set up again (block > 0; block <= 0 solves without
 * it), the right-hand side formed (mbem_rhs_planewave), the system solved
 * (mbem_solve with opts) and the cross sections evaluated
 * (mbem_cross_sections with ntheta; ntheta <= 0 picks 2 k0 a_max + 20 per
 * point).  One operator, one preconditioner and one Krylov workspace serve
 * the whole sweep; all are released before the call returns.
 *   params  precision, quadrature, ssq_order and near_radius of every
 *           point; its k0 and materials are ignored
 *   k0      host [npts], each > 0;  eps_r host [npts];  mu_r host [npts]
 *           or NULL (non-magnetic, mu_r = 1)
 *   khat    host [3] unit direction;  pol host [3] polarisation
 *   sigma   host [npts*3]: C_ext, C_sca, C_abs of point i at 3i..3i+2
 *   iters   host [npts] GMRES iterations per point, or NULL
 *   stats   NULL, or times and iteration counts summed over the points
 *           (t_geom_ms: the one geometry build; t_fill_ms: device time of
 *           the fills; rel_resid: the worst)
 * MBEM_EINVAL for a bad argument (nothing is run), MBEM_ENOCONV when some
 * point missed the tolerance (every point is still solved and written),
 * MBEM_ESINGULAR on a singular preconditioner block (sigma holds the points
 * before it).                                                              */
int mbem_spectrum(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *params,
                  int32_t npts, const double *k0, const mbem_c128 *eps_r,
                  const mbem_c128 *mu_r, const double *khat, const mbem_c128 *pol,
                  int32_t block, const mbem_solve_opts *opts, int32_t ntheta,
                  double *sigma, int32_t *iters, mbem_stats *stats);

const char *mbem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MBEM_H */
