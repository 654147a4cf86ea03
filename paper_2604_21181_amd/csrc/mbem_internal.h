// Internal declarations of the mbem library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mbem.h"

namespace mbem {
struct KernelConst;
struct BlrOp;
struct FillState;

// ---------------------------------------------------------------- errors --
void set_error(const std::string &msg);
// Wait until *tag (pinned host memory written by a kernel on stream s after
// a system-scope fence) equals seq; MBEM_EDEVICE with a message naming
// `what` if the stream fails or drains without it, or after a minute.
int wait_host_tag(const unsigned long long *tag, unsigned long long seq, hipStream_t s, const char *what);

#define MBEM_HIP(call)                                                       \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) {                                              \
            ::mbem::set_error(std::string(#call) + ": " +                    \
                              hipGetErrorString(e_));                        \
            return MBEM_EDEVICE;                                             \
        }                                                                    \
    } while (0)

#define MBEM_TRY(call)                                                       \
    do {                                                                     \
        int s_ = (call);                                                     \
        if (s_ != MBEM_OK) return s_;                                        \
    } while (0)

// ------------------------------------------------------------ constants --
constexpr int kQP = 7;          // regular rule points per triangle
constexpr int kQP12 = 12;       // points of the 12-point rule (paper's scheme)
constexpr int kMaxBlock = 512;  // largest supported block-Jacobi cluster size B
constexpr int kQPF = 19;        // doubles per quadrature point in the table
constexpr int kMaxSSQ = 8;      // largest Sauter-Schwab order supported
constexpr int kChunk = 4;       // trial triangles per regular-pair workgroup
// per trial chunk: n_slots, slot nodes[24], incidence offsets[25],
// incidences[24] (chunk-local triangle * 8 + local node)
constexpr int kChunkRec = 1 + 24 + 25 + 24;
// Column ranges of the regular-pair fill: rng consecutive (Morton) nodes;
// per range the trial triangles that touch it, in batches of nb, one record
// of rec() ints per batch: n, triangles[nb], per range-local node
// the offsets[rng + 1] into incidences[6 nb] (batch-local triangle * 8 +
// local node) of the nodes of the range.
struct RngLayout {
    int rng, nb;
    constexpr int off() const { return 1 + nb; }
    constexpr int inc() const { return off() + rng + 1; }
    constexpr int rec() const { return inc() + 6 * nb; }
};
constexpr RngLayout kRng = {64, 5};
// quadrature-point table fields (structure of arrays, each n_tris*7 long)
enum QpField {
    QX = 0, QW = 3, QN = 4, QT1 = 7, QT2 = 10, QS1 = 13, QS2 = 16
};

struct cplx {  // plain complex double for host-side bookkeeping
    double re, im;
};

// The FP64 near store of a MIXED operator (see near.hip): the node-pair
// pattern of the near and singular element pairs as bit rows (bit j of row
// i, nw 32-bit words per row) with the count of set bits before every word
// of its row, and as a CSR; values [nnz][12] complex128, component
// 4 op + 2 alpha + beta (op: K1, K2^eps, K2^mu).  bits == nullptr: no store.
struct NearView {
    const uint32_t *bits = nullptr;
    const int32_t *wpre = nullptr;   // [nn][nw]
    const int32_t *rptr = nullptr;   // [nn + 1]
    const int32_t *col = nullptr;    // [nnz]
    double2 *val = nullptr;          // [nnz][12]
    int64_t nw = 0;
};

// ---------------------------------------------------------- handles --------
}  // namespace mbem

struct mbem_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // FP32 GEMM tile shape measured fastest for the block product of an
    // operator with n2 rows per block and ncol right-hand sides
    int64_t tuned_n2 = 0;
    int tuned_ncol = 0, tuned_cfg = 0;
};

struct mbem_mesh {
    mbem_ctx *ctx = nullptr;
    int64_t nn = 0, nt = 0;
    std::vector<int64_t> node_order, tri_order;  // Morton position -> caller
    std::vector<double> xyz;                     // Morton order [nn*3]
    std::vector<uint64_t> node_key;              // Morton keys, Morton order
    std::vector<int32_t> tri;                    // Morton numbering [nt*6]
    double amax = 0.0;                           // max |x| over nodes
    int64_t n_single[4] = {0, 0, 0, 0};          // ordered pairs per class
    // device copies
    double *d_xyz = nullptr;
    int32_t *d_tri = nullptr;
    int32_t *d_inc_ptr = nullptr;  // node -> (elem*8 + local) CSR
    int32_t *d_inc = nullptr;
    int32_t *d_spairs = nullptr;   // singular ordered pairs, int4 each
    int64_t n_spairs = 0;
    // geometry tables (rebuilt by every fill)
    double *d_frames = nullptr;    // [nn][9]: n, t1, t2
    double *d_qp = nullptr;        // [kQPF][nt*7]
    float *d_qp32 = nullptr;       // [kQPF][nt*7]
    double *d_qp12 = nullptr;      // [kQPF][nt*12], the 12-point rule (paper's scheme)
    float *d_qp12_32 = nullptr;    // [kQPF][nt*12]
    double *d_elem = nullptr;      // [nt][4]: centroid, radius
    // mass-matrix pattern (node CSR) and element -> CSR slot map
    std::vector<int32_t> m_ptr, m_col;
    int32_t *d_mptr = nullptr, *d_mcol = nullptr, *d_mslot = nullptr;
    int32_t *d_chunks = nullptr;   // trial-chunk records, kChunkRec ints each
    // column ranges: batch records (kRng.rec() ints each) and, per range,
    // the first record (one more than ranges)
    int64_t nrng = 0;
    int32_t *d_rng_off = nullptr, *d_rng_rec = nullptr;
    int32_t *d_row_first = nullptr;   // per triangle: first writer of its nodes' rows
    int32_t *d_col_first = nullptr;   // per trial chunk: first writer of its slots' columns
    // colour classes of the race-free regular-pair fill, and the class of
    // every test triangle and trial chunk
    std::vector<int32_t> tcol_off, ccol_off;
    int32_t *d_tcol = nullptr, *d_ccol = nullptr;
    int32_t *d_tcolour = nullptr, *d_ccolour = nullptr;
    // host copies for band fills: the test colour lists and singular pairs
    std::vector<int32_t> tcol_list, spairs;
};

struct mbem_op {
    mbem_ctx *ctx = nullptr;
    const mbem_mesh *mesh = nullptr;
    mbem_params p{};
    int prec = MBEM_FP64;
    int64_t n2 = 0;                 // 2 n_nodes: one current's length
    double2 ka{}, ki{}, eps_i{}, mu_i{};
    double2 iw{}, ce{}, cm{};       // i/omega, (eps_i+1)/2, (mu_i+1)/2
    void *K[3] = {nullptr, nullptr, nullptr};  // c128 or c64 dense blocks
    double *d_mval = nullptr;       // mass values on the node CSR pattern
    int64_t n_near = 0;
    double t_phase[5] = {0, 0, 0, 0, 0};  // geom, regular, near, ssq, mass (ms)
    mbem::KernelConst *d_kconst = nullptr;   // device copy of the kernel constants
    // node-attached tangents: per triangle and rule point the 2 x 2
    // components of its nodes' tangents in the point frame, times N_k
    // ([nt][points][6][2][2], in the precision of the regular-pair kernel)
    void *d_rtab = nullptr;
    size_t rtab_bytes = 0;
    // Morton block-Jacobi
    int32_t B = 0, nb = 0;
    double2 *d_minv = nullptr;      // [nb][2B][2B] inverses
    double2 *d_minv_t = nullptr;    // their transposes (adjoint solves)
    // complex64 copies of both for the GMRES steps of a MIXED operator
    // (made with the inverses and with their transposes)
    float2 *d_minv32 = nullptr, *d_minv_t32 = nullptr;
    double2 *d_lu = nullptr;        // scratch of the factorisation
    size_t minv_bytes = 0, lu_bytes = 0;   // sizes of d_minv and d_lu
    // solver workspace
    double2 *d_work = nullptr;
    size_t work_elems = 0;
    double2 *h_pin = nullptr;       // pinned host copies of Hessenberg columns
    size_t pin_elems = 0;
    // multi-right-hand-side solve: complex64 copy of an FP64 operator's
    // blocks for the FP32 GEMM
    void *K32[3] = {nullptr, nullptr, nullptr};
    // block low-rank operator: set instead of K
    mbem::BlrOp *blr = nullptr;
    // events and staging of the last enqueued fill
    mbem::FillState *fs = nullptr;
    // MIXED with params.near_store: the FP64 near store (near.hip) and, per
    // (test triangle, trial chunk), the bit mask of the chunk's triangles
    // that are near (regular) partners of the test triangle
    bool near_on = false;
    uint32_t *d_nbits = nullptr;
    int32_t *d_nwpre = nullptr, *d_nrptr = nullptr, *d_ncol = nullptr;
    double2 *d_nval = nullptr;
    uint8_t *d_nmask = nullptr;
    unsigned long long *d_ncount = nullptr;   // near pairs, nnz, then per launch its near tiles
    int64_t near_nw = 0, near_nnz = 0, near_cap = 0;
    // (test triangle, trial chunk) tiles with near pairs, grouped by the
    // (test colour, chunk colour) launch of the regular-pair fill
    int2 *d_ntiles = nullptr;
    unsigned long long *d_ncursor = nullptr;
    int64_t near_tile_cap = 0;
    std::vector<int64_t> near_tile_off;       // host: launch -> first tile, one more
    mbem::NearView near_view() const {
        mbem::NearView v;
        if (!near_on) return v;
        v.bits = d_nbits; v.wpre = d_nwpre; v.rptr = d_nrptr; v.col = d_ncol; v.val = d_nval; v.nw = near_nw;
        return v;
    }
};

namespace mbem {

// host preprocessing (host_mesh.cpp)
struct MeshTables {
    std::vector<int32_t> inc_ptr, inc;      // node -> elem*8 + local
    std::vector<int32_t> spairs;            // e, f, class, perm codes
    int64_t n_single[4] = {0, 0, 0, 0};
    std::vector<int32_t> m_ptr, m_col, m_slot;
    std::vector<int32_t> chunks;            // kChunkRec ints per trial chunk
    std::vector<int32_t> rng_off, rng_rec;  // column ranges: first record, records
    // per test triangle, bit a: the triangle is the first of its colour
    // order to write the rows of its local node a (the lowest colour among
    // the node's triangles)
    std::vector<int32_t> row_first;
    // per trial chunk, bit sl: the chunk is the first of its colour order to
    // write the columns of its slot node sl
    std::vector<int32_t> col_first;
    // colour classes: test triangles sharing no node, trial chunks sharing
    // no node (offsets into the concatenated lists, one more than classes)
    std::vector<int32_t> tcol_list, tcol_off, ccol_list, ccol_off;
};
int build_tables(const mbem_mesh *m, MeshTables &T);
int build_mesh_host(const double *xyz, int64_t nn, const int64_t *tri6,
                    int64_t nt, mbem_mesh *m);
// node_keys (optional): the nodes' Morton keys in Morton order
int morton_order_host(const double *xyz, int64_t nn, const int64_t *tri6,
                      int64_t nt, std::vector<int64_t> &node_order,
                      std::vector<int64_t> &tri_order, std::vector<uint64_t> *node_keys = nullptr);
void gauss_legendre(int n, double *x, double *w);   // on [-1, 1]

// geometry (geom.hip)
// with12: also the 12-point quadrature tables (the paper's scheme)
int geom_build(const mbem_mesh *m, hipStream_t s, bool with12 = false);

// fill (fill.hip)
// deriv: fill dK/deps_i instead of K (FP64 operators only)
// geom = false: the mesh's geometry tables are already built (a sweep that
// refills the same mesh)
int fill_run(mbem_op *op, hipStream_t s, bool deriv = false, bool geom = true);
// The kernel constants of the op's wavenumbers on the device (first step of
// every fill), through the op's pinned staging buffer.
int fill_prepare(mbem_op *op, hipStream_t s, bool deriv);
// fill_run in two halves: enqueue every launch of the fill on s without
// waiting (fill_run = fill_enqueue + fill_collect); fill_collect waits for
// the fill's last event and reads its phase times, the near-pair count and,
// if asked, the device time from its first launch to its last.
int fill_enqueue(mbem_op *op, hipStream_t s, bool deriv, bool geom);
int fill_collect(mbem_op *op, double *t_total_ms);
void fill_state_free(FillState *f);
// A band of test rows (compressed fill): every regular and singular pair
// whose test triangle is listed, added into band buffers whose rows are
// numbered by row_map.
struct FillBand {
    const int32_t *tcol = nullptr;        // device: the band's test triangles by colour class
    std::vector<int32_t> tcol_off;        // host offsets, one more than the classes
    const int32_t *spairs = nullptr;      // device: the band's singular pairs (4 ints each)
    int64_t n_spairs = 0;
    const int32_t *row_map = nullptr;     // device [nn]: node -> band row node
    void *Z[3] = {nullptr, nullptr, nullptr};   // band buffers, leading dimension 2 nn
};
// FP64, default scheme; the geometry tables and kernel constants are current.
int fill_band_run(mbem_op *op, const FillBand &band, hipStream_t s);

// block low-rank operator (blr.hip)
struct BlrTile {
    int32_t op, t, s, rank;   // block, row / column cluster; rank < 0: dense
    int32_t m, n;             // rows, columns (twice the cluster sizes)
    int64_t r0, c0;           // first row / column in the block
    double2 *a;               // dense m x n row-major, or U^T (rank x m, row-major)
    double2 *vt;              // V^T (rank x n, row-major); null when dense
    int64_t w;                // offset of this tile's V^T x in the product workspace
    int64_t z;                // offset of this tile's row products (m per vector)
};
struct BlrView {              // what device code needs to read entries
    int32_t nc;
    const int32_t *cl_of;     // node -> cluster
    const BlrTile *tiles;     // tile (op, t, s) at (op nc + t) nc + s
};
// One entry of block op, row r, column q.
__device__ inline double2 blr_entry(const BlrView &v, int op, int64_t r, int64_t q) {
    const int64_t t = v.cl_of[r >> 1], sc = v.cl_of[q >> 1];
    const BlrTile &T = v.tiles[((int64_t)op * v.nc + t) * v.nc + sc];
    const int64_t lr = r - T.r0, lc = q - T.c0;
    if (T.rank < 0) return T.a[lr * T.n + lc];
    double2 z = {0.0, 0.0};
    for (int k = 0; k < T.rank; ++k) {
        const double2 u = T.a[(int64_t)k * T.m + lr], w = T.vt[(int64_t)k * T.n + lc];
        z.x += u.x * w.x - u.y * w.y;
        z.y += u.x * w.y + u.y * w.x;
    }
    return z;
}
int blr_fill_run(mbem_op *op, const mbem_blr_opts *o, mbem_blr_stats *bs, hipStream_t s);
// t = [K1 xj, K1 xm, K2e xm, K2m xj] (4 n2), as the dense product
int blr_gemv_run(const mbem_op *op, const double2 *xj, const double2 *xm, double2 *t, hipStream_t s);
// the three blocks expanded into dense n2 x n2 buffers (any may be null)
int blr_expand_run(const mbem_op *op, double2 *K0, double2 *K1, double2 *K2, hipStream_t s);
BlrView blr_view(const mbem_op *op);
void blr_free(BlrOp *b);
int mass_run(mbem_op *op, hipStream_t s);

// linear algebra (linalg.hip)
int matvec_run(const mbem_op *op, const double2 *x, double2 *y, double2 *tmp,
               hipStream_t s, hipEvent_t after_gemv = nullptr);
int export_dense_run(const mbem_op *op, double2 *Z, hipStream_t s);
int export_blocks_run(const mbem_op *op, double2 *K1, double2 *K2e,
                      double2 *K2m, hipStream_t s);
// keep = true: the factorisation scratch stays allocated for the next setup
// of the same block size (sweeps); the inverses are reused whenever the size
// matches
int mbj_setup_run(mbem_op *op, int B, hipStream_t s, bool keep = false);
// trans: apply P^-T (mbj_transpose_run must have run)
// *dst (allocated when null) = src rounded to complex64, n elements
int mbj_copy_c64(const double2 *src, float2 **dst, int64_t n, hipStream_t s);
// lowp: with the complex64 copy of the inverses when there is one (the
// GMRES steps of a MIXED operator, which apply the same copy throughout)
int mbj_apply_run(const mbem_op *op, const double2 *v, double2 *z,
                  hipStream_t s, bool trans = false, bool lowp = false);
int vec_norm2(const double2 *v, int64_t n, double *out_dev, hipStream_t s);
// Classical Gram-Schmidt with one reorthogonalisation of win (n rows; the
// result goes to w, which may be win) against the k orthonormal columns of
// V (leading dimension ldv).  The
// coefficients of both passes go to the device column hcol[0..k) = h1,
// hcol[k..2k) = h2, and the chunks' parts of |w|^2 to npart.  With finish,
// arnoldi_finish follows.  part: 2 k arnoldi_chunks(n) complex and npart:
// arnoldi_chunks(n) doubles of device scratch.
int64_t arnoldi_chunks(int64_t n);
int arnoldi_cgs2(const double2 *win, double2 *w, double2 *V, int64_t ldv, int k, int64_t n, double2 *part,
                 double *npart, double2 *hcol, bool finish, double2 *pin, unsigned long long *tag,
                 unsigned long long seq, hipStream_t s);
// V_k = w / |w| (column k of V; 0 when w vanishes), |w| from npart; then
// the step's column is published to host-mapped memory: pin[0..2k) = hcol,
// pin[2k].x = |w| and, after a system-scope fence, *tag = seq, so a host
// that reads the tag reads the whole column.
int arnoldi_finish(const double2 *w, double2 *V, int64_t ldv, int k, int64_t n, const double *npart,
                   const double2 *hcol, double2 *pin, unsigned long long *tag, unsigned long long seq,
                   hipStream_t s);
// arnoldi_finish fused with the block-Jacobi product of the next step:
// vk = w / |w|, z = P^-1 vk (P^-T with trans), and the finished step's
// column (k coefficients per pass) published as by arnoldi_finish.  Needs
// a preconditioner (mbj_present).
bool mbj_present(const mbem_op *op);
int mbj_scale_apply_run(const mbem_op *op, const double2 *w, const double *npart, int64_t n, double2 *vk,
                        double2 *z, const double2 *hcol, int k, double2 *pin, unsigned long long *tag,
                        unsigned long long seq, hipStream_t s, bool trans, bool lowp);
int vec_scale_copy(double2 *dst, const double2 *src, double2 a, int64_t n,
                   hipStream_t s);
int vec_axpy(double2 *y, const double2 *x, double2 a, int64_t n,
             hipStream_t s);
int vec_combine(double2 *out, const double2 *V, int64_t ldv, int k,
                const double2 *y_dev, int64_t n, hipStream_t s);
// r = b - sum_{j<k} W_j y_j (columns of W with leading dimension ldw; r may
// be b)
int vec_resid_products(double2 *r, const double2 *b, const double2 *W, int64_t ldw, int k, const double2 *y_dev,
                       int64_t n, hipStream_t s);

// adjoint (adjoint.hip)
int ff_functional_run(const mbem_mesh *m, const mbem_params *p, const double *rhat, const double2 *e,
                      double2 *g, hipStream_t s);
int matvec_t_run(const mbem_op *op, const double2 *x, double2 *y, double2 *part, hipStream_t s);
int64_t matvec_t_work(const mbem_op *op);
int mbj_transpose_run(mbem_op *op, hipStream_t s);
int dotu_run(const double2 *a, const double2 *b, int64_t n, double2 *out, hipStream_t s);
// shape.hip: d sigma / d(node positions) from x and lambda (Morton order)
// dir: device [nn*3] displacement directions for dnode, or null (nodal normals)
int shape_grad_run(const mbem_op *op, const mbem_params *p, const double2 *x, const double2 *lam,
                   const double *khat, const double2 *pol, const double *dir, double *dnode, double *dx,
                   hipStream_t s);

// FP64 near store (near.hip)
// Builds the near mask and the node-pair pattern of the near and singular
// element pairs for the op's near radius, sizes and zeroes the values (one
// host wait for the pattern size).  MIXED ops with params.near_store only.
int near_build_run(mbem_op *op, double near_r, hipStream_t s);
// Adds the store into the complex64 blocks and releases it (the op then
// holds its whole Z in complex64).
int near_fold_run(mbem_op *op, hipStream_t s);
void near_free(mbem_op *op);
// K1, K2e, K2m (complex128, n2 x n2, any may be null) += the store
int near_add_dense_run(const mbem_op *op, double2 *K1, double2 *K2e, double2 *K2m, hipStream_t s);

// multi-right-hand-side solve (block.hip)
int block_solve_run(mbem_op *op, const double2 *B, int ncol, const mbem_block_opts *o, double2 *X,
                    mbem_block_stats *st, hipStream_t s);
int ensure_c64_copy(mbem_op *op, hipStream_t s);

// post-processing (post.hip)
int rhs_run(const mbem_mesh *m, const mbem_params *p, const double *khat,
            const double2 *pol, int nrhs, double2 *b, hipStream_t s);
int farfield_run(const mbem_mesh *m, const mbem_params *p, const double2 *x,
                 int nrhs, const double *rhat, int64_t ndir, double2 *F,
                 hipStream_t s);
int absorbed_run(const mbem_mesh *m, const mbem_params *p, const double2 *x, double *out_dev,
                 hipStream_t s);
int weighted_norm_run(int64_t ndir, const double2 *F, const double *w,
                      double *out, hipStream_t s);

// derived material constants
void derive_constants(const mbem_params *p, double2 *ka, double2 *ki,
                      double2 *eps_i, double2 *mu_i);

}  // namespace mbem
