// Matrix-vector product with the stored Galerkin operator, export of Z, the
// Morton block-Jacobi preconditioner (Sec. 5) and the vector kernels of
// GMRES.
//
// Z is applied from its three distinct dense blocks and the sparse mass
// matrix (eq. global_system):
//   y_j  = (i/w) K1 x_j + K2^eps x_m + c_eps (M (x) I2) x_m
//   y_m  = K2^mu x_j + c_mu (M (x) I2) x_j - (i/w) K1 x_m
// so every dense entry is read once per product; K1 feeds two dot products.
#include <mutex>
#include <type_traits>

#include "gemm.h"
#include "mbem_internal.h"
#include "near_store.h"
#include "wave.h"

namespace mbem {

constexpr int kW = 64;

__device__ inline double2 cmul(double2 a, double2 b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ inline double2 cadd(double2 a, double2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline double2 csub(double2 a, double2 b) { return {a.x - b.x, a.y - b.y}; }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = kW / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kW);
    return v;
}

// ---------------------------------------------------------------- GEMV --
// One wavefront per R consecutive stored rows of one block; lanes stream
// the rows with 16-byte loads, and every load of the right-hand vector(s)
// (FP64, from L2) serves all R rows.  The c64 variant loads two entries per
// lane and row per step and accumulates in FP64; with eight rows per
// wavefront its vector loads no longer outweigh the matrix stream (measured
// per product on the 1280-triangle sphere: 158 us at one row, 118 us at
// eight, 440 us at sixteen; c128: 221 us at one row, slower at two).
template <typename TS> constexpr int gemv_rows_per_wave();
template <> constexpr int gemv_rows_per_wave<double2>() { return 1; }
template <> constexpr int gemv_rows_per_wave<float2>() { return 8; }
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
// streaming loads of the matrix: each entry is used exactly once per product
__device__ inline double2 ntload(const double2 *p) {
    const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2 *>(p));
    return {v.x, v.y};
}
__device__ inline float4 ntload(const float4 *p) {
    const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4 *>(p));
    return {v.x, v.y, v.z, v.w};
}

// re/im[k][v] += row r0 + k of K (row length n) . xs[v], for k < nr
// (nr is uniform over the wavefront)
template <int NV, int R>
__device__ inline void rows_dots(const double2 *__restrict__ K, int64_t n, int64_t r0, int nr,
                                 const double2 *const xs[NV], double re[R][NV], double im[R][NV]) {
    const int lane = threadIdx.x % kW;
    const double2 *row[R];
#pragma unroll
    for (int k = 0; k < R; ++k) row[k] = K + (r0 + (k < nr ? k : 0)) * n;
#pragma unroll 4
    for (int64_t c = lane; c < n; c += kW) {
        double2 x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = xs[v][c];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k >= nr) break;
            const double2 z = ntload(row[k] + c);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                re[k][v] += z.x * x[v].x - z.y * x[v].y;
                im[k][v] += z.x * x[v].y + z.y * x[v].x;
            }
        }
    }
}

template <int NV, int R>
__device__ inline void rows_dots(const float2 *__restrict__ K, int64_t n, int64_t r0, int nr,
                                 const double2 *const xs[NV], double re[R][NV], double im[R][NV]) {
    const int lane = threadIdx.x % kW;
    const int64_t n4 = n / 2;   // n is even (2 unknowns per node)
    const float4 *row[R];
#pragma unroll
    for (int k = 0; k < R; ++k)
        row[k] = reinterpret_cast<const float4 *>(K + (r0 + (k < nr ? k : 0)) * n);
#pragma unroll 2
    for (int64_t c = lane; c < n4; c += kW) {
        double2 x0[NV], x1[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) { x0[v] = xs[v][2 * c]; x1[v] = xs[v][2 * c + 1]; }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k >= nr) break;
            const float4 z = ntload(row[k] + c);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                re[k][v] += (double)z.x * x0[v].x - (double)z.y * x0[v].y +
                            (double)z.z * x1[v].x - (double)z.w * x1[v].y;
                im[k][v] += (double)z.x * x0[v].y + (double)z.y * x0[v].x +
                            (double)z.z * x1[v].y + (double)z.w * x1[v].x;
            }
        }
    }
}

// t[0] = K1 x_j, t[1] = K1 x_m, t[2] = K2e x_m, t[3] = K2m x_j (each n2).
template <typename TS, int NV, int R>
__device__ inline void gemv_rows(const TS *K, int64_t n2, int64_t r0, int nr,
                                 const double2 *const xs[NV], double2 *const ts[NV]) {
    double re[R][NV], im[R][NV];
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) re[k][v] = im[k][v] = 0.0;
    rows_dots<NV, R>(K, n2, r0, nr, xs, re, im);
    const int lane = threadIdx.x % kW;
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double2 o = {wave_sum(re[k][v]), wave_sum(im[k][v])};
            if (lane == 0 && k < nr) ts[v][r0 + k] = o;
        }
}

template <typename TS>
__global__ __launch_bounds__(256) void k_gemv3(int64_t n2, const TS *K1, const TS *K2e,
                                               const TS *K2m, const double2 *xj,
                                               const double2 *xm, double2 *t) {
    constexpr int R = gemv_rows_per_wave<TS>();
    const int64_t nwr = (n2 + R - 1) / R;                    // wavefronts per block
    const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kW;
    if (wid >= 3 * nwr) return;
    const int blk = (int)(wid / nwr);
    const int64_t r0 = (wid % nwr) * R;
    const int nr = (int)(n2 - r0 < R ? n2 - r0 : R);
    if (blk == 0) {
        const double2 *xs[2] = {xj, xm};
        double2 *ts[2] = {t, t + n2};
        gemv_rows<TS, 2, R>(K1, n2, r0, nr, xs, ts);
    } else {
        const double2 *xs[1] = {blk == 1 ? xm : xj};
        double2 *ts[1] = {t + (1 + blk) * n2};
        gemv_rows<TS, 1, R>(blk == 1 ? K2e : K2m, n2, r0, nr, xs, ts);
    }
}

struct Coef { double2 iw, ce, cm; };

// LANES consecutive lanes per row split the row's mass slots (a vertex
// node has 19, each a dependent index-then-value load) and, with the near
// store, its stored node pairs (about 70 per node on the 5120-triangle
// spheroid: sixteen lanes then), and add their partial sums by shuffles in a
// fixed order.
constexpr int kCombLanes = 8, kCombLanesNear = 16;
// With the FP64 near store (nv.bits non-null) its blocks are added to the
// four products: row 2 i + al takes V[4 op + 2 al + be] of every stored
// node pair (i, j) times x at 2 j + be.
template <int LANES>
__global__ __launch_bounds__(256) void k_combine(int64_t n2, const double2 *__restrict__ t,
                                                 const int32_t *__restrict__ mptr, const int32_t *__restrict__ mcol,
                                                 const double *__restrict__ mval, const double2 *__restrict__ xj,
                                                 const double2 *__restrict__ xm, Coef c, NearView nv,
                                                 double2 *__restrict__ y) {
    const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t r = gt / LANES;
    const int l = (int)(gt % LANES);
    double mj[2] = {0, 0}, mm[2] = {0, 0};
    double nq[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};   // K1 xj, K1 xm, K2e xm, K2m xj (store)
    if (r < n2) {
        const int64_t i = r / 2;
        const int al = (int)(r % 2);
        // mass: 2 x 2 block per node pair, value (al, be) at mval[4 s + 2 al + be]
        for (int32_t s = mptr[i] + l; s < mptr[i + 1]; s += LANES) {
            const int64_t col = 2 * (int64_t)mcol[s];
            const double v0 = mval[4 * s + 2 * al], v1 = mval[4 * s + 2 * al + 1];
            mj[0] += v0 * xj[col].x + v1 * xj[col + 1].x; mj[1] += v0 * xj[col].y + v1 * xj[col + 1].y;
            mm[0] += v0 * xm[col].x + v1 * xm[col + 1].x; mm[1] += v0 * xm[col].y + v1 * xm[col + 1].y;
        }
        if (nv.bits)
            for (int32_t s = nv.rptr[i] + l; s < nv.rptr[i + 1]; s += LANES) {
                const int64_t col = 2 * (int64_t)nv.col[s];
                const double2 *V = nv.val + 12 * (int64_t)s + 2 * al;
                const double2 a0 = xj[col], a1 = xj[col + 1], b0 = xm[col], b1 = xm[col + 1];
                const double2 p[4] = {cadd(cmul(V[0], a0), cmul(V[1], a1)), cadd(cmul(V[0], b0), cmul(V[1], b1)),
                                      cadd(cmul(V[4], b0), cmul(V[5], b1)), cadd(cmul(V[8], a0), cmul(V[9], a1))};
#pragma unroll
                for (int k = 0; k < 4; ++k) { nq[k][0] += p[k].x; nq[k][1] += p[k].y; }
            }
    }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            mj[k] += __shfl_xor(mj[k], o, LANES);
            mm[k] += __shfl_xor(mm[k], o, LANES);
        }
        if (nv.bits)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                nq[k][0] += __shfl_xor(nq[k][0], o, LANES);
                nq[k][1] += __shfl_xor(nq[k][1], o, LANES);
            }
    }
    if (r >= n2 || l != 0) return;
    const double2 Mj = {mj[0], mj[1]}, Mm = {mm[0], mm[1]};
    const double2 t0 = cadd(t[r], double2{nq[0][0], nq[0][1]}), t1 = cadd(t[n2 + r], double2{nq[1][0], nq[1][1]});
    const double2 t2 = cadd(t[2 * n2 + r], double2{nq[2][0], nq[2][1]});
    const double2 t3 = cadd(t[3 * n2 + r], double2{nq[3][0], nq[3][1]});
    y[r] = cadd(cadd(cmul(c.iw, t0), t2), cmul(c.ce, Mm));
    y[n2 + r] = csub(cadd(t3, cmul(c.cm, Mj)), cmul(c.iw, t1));
}

static Coef coef_of(const mbem_op *op) { return {op->iw, op->ce, op->cm}; }

int matvec_run(const mbem_op *op, const double2 *x, double2 *y, double2 *tmp, hipStream_t s,
               hipEvent_t after_gemv) {
    const int64_t n2 = op->n2;
    auto blocks = [n2](int R) { return (unsigned)((3 * ((n2 + R - 1) / R) * kW + 255) / 256); };
    if (op->blr)
        MBEM_TRY(blr_gemv_run(op, x, x + n2, tmp, s));
    else if (op->prec == MBEM_FP64)
        hipLaunchKernelGGL((k_gemv3<double2>), dim3(blocks(gemv_rows_per_wave<double2>())), dim3(256), 0, s,
                           n2, (const double2 *)op->K[0], (const double2 *)op->K[1],
                           (const double2 *)op->K[2], x, x + n2, tmp);
    else
        hipLaunchKernelGGL((k_gemv3<float2>), dim3(blocks(gemv_rows_per_wave<float2>())), dim3(256), 0, s,
                           n2, (const float2 *)op->K[0], (const float2 *)op->K[1],
                           (const float2 *)op->K[2], x, x + n2, tmp);
    MBEM_HIP(hipGetLastError());
    if (after_gemv) MBEM_HIP(hipEventRecord(after_gemv, s));
    const mbem_mesh *m = op->mesh;
    const NearView nv = op->near_view();
    if (nv.bits)
        hipLaunchKernelGGL(k_combine<kCombLanesNear>, dim3((unsigned)((n2 * kCombLanesNear + 255) / 256)), dim3(256),
                           0, s, n2, tmp, m->d_mptr, m->d_mcol, op->d_mval, x, x + n2, coef_of(op), nv, y);
    else
        hipLaunchKernelGGL(k_combine<kCombLanes>, dim3((unsigned)((n2 * kCombLanes + 255) / 256)), dim3(256), 0, s,
                           n2, tmp, m->d_mptr, m->d_mcol, op->d_mval, x, x + n2, coef_of(op), nv, y);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

// ------------------------------------------------------- entries of Z --
template <typename TS>
__device__ inline double2 kval(const void *K, int64_t idx) {
    if constexpr (std::is_same<TS, double2>::value) return ((const double2 *)K)[idx];
    else { const float2 v = ((const float2 *)K)[idx]; return {(double)v.x, (double)v.y}; }
}

// mass entry of unknowns (2 i + al, 2 j + be)
__device__ inline double mass_entry(const int32_t *mptr, const int32_t *mcol, const double *mval,
                                    int64_t i, int64_t j, int al, int be) {
    for (int32_t s = mptr[i]; s < mptr[i + 1]; ++s)
        if (mcol[s] == j) return mval[4 * s + 2 * al + be];
    return 0.0;
}

// entry (r, q) of block op: the stored value plus the near store's
template <typename TS>
__device__ inline double2 kentry(const void *const K[3], const NearView &nv, int op, int64_t n2, int64_t r,
                                 int64_t q) {
    return cadd(kval<TS>(K[op], r * n2 + q), near_value(nv, op, r / 2, q / 2, (int)(r % 2), (int)(q % 2)));
}

// Z[(ci n2 + r), (cc n2 + q)] for current indices ci, cc in {0, 1}
template <typename TS>
__device__ inline double2 z_entry(const void *const K[3], const int32_t *mptr,
                                  const int32_t *mcol, const double *mval, Coef c,
                                  int64_t n2, int ci, int64_t r, int cc, int64_t q, const NearView &nv) {
    double2 z;
    if (ci == 0 && cc == 0) z = cmul(c.iw, kentry<TS>(K, nv, 0, n2, r, q));
    else if (ci == 1 && cc == 1) { const double2 k = cmul(c.iw, kentry<TS>(K, nv, 0, n2, r, q)); z = {-k.x, -k.y}; }
    else {
        z = kentry<TS>(K, nv, ci == 0 ? 1 : 2, n2, r, q);
        const double mv = mass_entry(mptr, mcol, mval, r / 2, q / 2, (int)(r % 2), (int)(q % 2));
        const double2 cf = ci == 0 ? c.ce : c.cm;
        z.x += cf.x * mv; z.y += cf.y * mv;
    }
    return z;
}

template <typename TS>
__global__ void k_export_dense(int64_t n2, const void *K0, const void *K1, const void *K2,
                               const int32_t *mptr, const int32_t *mcol, const double *mval,
                               Coef c, NearView nv, double2 *Z) {
    const int64_t N = 2 * n2;
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= N * N) return;
    const int64_t R = id / N, C = id % N;
    const void *K[3] = {K0, K1, K2};
    Z[id] = z_entry<TS>(K, mptr, mcol, mval, c, n2, (int)(R / n2), R % n2, (int)(C / n2), C % n2, nv);
}

int export_dense_run(const mbem_op *op, double2 *Z, hipStream_t s) {
    if (op->blr) { set_error("a block low-rank operator exports its blocks only"); return MBEM_EINVAL; }
    const int64_t N = 2 * op->n2;
    const mbem_mesh *m = op->mesh;
    const unsigned blocks = (unsigned)((N * N + 255) / 256);
    if (op->prec == MBEM_FP64)
        hipLaunchKernelGGL((k_export_dense<double2>), dim3(blocks), dim3(256), 0, s, op->n2,
                           op->K[0], op->K[1], op->K[2], m->d_mptr, m->d_mcol, op->d_mval, coef_of(op), NearView{}, Z);
    else
        hipLaunchKernelGGL((k_export_dense<float2>), dim3(blocks), dim3(256), 0, s, op->n2,
                           op->K[0], op->K[1], op->K[2], m->d_mptr, m->d_mcol, op->d_mval, coef_of(op),
                           op->near_view(), Z);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

__global__ void k_c64_to_c128(int64_t n, const float2 *a, double2 *b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = {(double)a[i].x, (double)a[i].y};
}

int export_blocks_run(const mbem_op *op, double2 *K1, double2 *K2e, double2 *K2m, hipStream_t s) {
    if (op->blr) return blr_expand_run(op, K1, K2e, K2m, s);
    double2 *dst[3] = {K1, K2e, K2m};
    const int64_t n = op->n2 * op->n2;
    for (int o = 0; o < 3; ++o) {
        if (!dst[o]) continue;
        if (op->prec == MBEM_FP64) {
            MBEM_HIP(hipMemcpyAsync(dst[o], op->K[o], 16 * n, hipMemcpyDeviceToDevice, s));
        } else {
            hipLaunchKernelGGL(k_c64_to_c128, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                               (const float2 *)op->K[o], dst[o]);
            MBEM_HIP(hipGetLastError());
        }
    }
    if (op->near_on) MBEM_TRY(near_add_dense_run(op, K1, K2e, K2m, s));
    return MBEM_OK;
}

// ------------------------------------------------- Morton block-Jacobi --
// Block m covers indices I_m = [m B, m B + b) of each current (b = B except
// possibly the last); A_m is the 2b x 2b restriction of Z to I_m in both
// currents (eq. precond_block), stored with leading dimension 2B.
template <typename TS>
__global__ void k_mbj_gather(int64_t n2, int B, const void *K0, const void *K1, const void *K2,
                             const int32_t *mptr, const int32_t *mcol, const double *mval,
                             Coef c, NearView nv, double2 *A) {
    const int m = blockIdx.y;
    const int64_t b = min((int64_t)B, n2 - (int64_t)m * B);
    const int64_t ld = 2 * B, n = 2 * b;
    const void *K[3] = {K0, K1, K2};
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < n * n;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = id / n, q = id % n;
        const int ci = r < b ? 0 : 1, cc = q < b ? 0 : 1;
        const int64_t gr = (int64_t)m * B + (r % b), gq = (int64_t)m * B + (q % b);
        A[(int64_t)m * ld * ld + r * ld + q] = z_entry<TS>(K, mptr, mcol, mval, c, n2, ci, gr, cc, gq, nv);
    }
}

// The same restrictions read from a block low-rank operator.
__global__ void k_mbj_gather_blr(int64_t n2, int B, BlrView v, const int32_t *mptr, const int32_t *mcol,
                                 const double *mval, Coef c, double2 *A) {
    const int m = blockIdx.y;
    const int64_t b = min((int64_t)B, n2 - (int64_t)m * B);
    const int64_t ld = 2 * B, n = 2 * b;
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < n * n;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = id / n, q = id % n;
        const int ci = r < b ? 0 : 1, cc = q < b ? 0 : 1;
        const int64_t gr = (int64_t)m * B + (r % b), gq = (int64_t)m * B + (q % b);
        double2 z;
        if (ci == cc) {
            const double2 k = cmul(c.iw, blr_entry(v, 0, gr, gq));
            z = ci == 0 ? k : double2{-k.x, -k.y};
        } else {
            z = blr_entry(v, ci == 0 ? 1 : 2, gr, gq);
            const double mv = mass_entry(mptr, mcol, mval, gr / 2, gq / 2, (int)(gr % 2), (int)(gq % 2));
            const double2 cf = ci == 0 ? c.ce : c.cm;
            z.x += cf.x * mv;
            z.y += cf.y * mv;
        }
        A[(int64_t)m * ld * ld + r * ld + q] = z;
    }
}

// Blocked right-looking LU with partial pivoting (largest modulus), one
// workgroup per block, panels of kPW columns: the panel is factorised
// column by column, U12 = L11^-1 A12 is formed, and the trailing matrix is
// updated from L21 and U12 staged in LDS (one pass over A22 per panel).
// Instantiated for blocks up to 512 (B <= 256, panels of 8) and up to 1024
// (B <= 512, panels of 4, so that L21 and U12 still fit in LDS).

template <int MAXN, int kPW>
__global__ __launch_bounds__(1024) void k_mbj_lu(int64_t n2, int B, double2 *A, int32_t *piv,
                                                 int32_t *info) {
    __shared__ double s_v[1024 / kW];
    __shared__ int s_i[1024 / kW];
    __shared__ double2 s_L[MAXN * kPW];    // L21, rows below the panel
    __shared__ double2 s_U[kPW * MAXN];    // U12, columns right of it
    __shared__ int32_t s_pv[MAXN];         // row interchange of each step
    const int m = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
    const int b = (int)min((int64_t)B, n2 - (int64_t)m * B);
    const int n = 2 * b, ld = 2 * B;
    double2 *a = A + (int64_t)m * ld * ld;
    int32_t *pv = piv + (int64_t)m * ld;
    for (int j0 = 0; j0 < n; j0 += kPW) {
        const int jw = min(kPW, n - j0), je = j0 + jw;
        // 1. panel columns j0 .. je-1
        for (int k = j0; k < je; ++k) {
            double best = -1.0;
            int bi = k;
            for (int i = k + tid; i < n; i += nth) {
                const double2 v = a[(int64_t)i * ld + k];
                const double mag = v.x * v.x + v.y * v.y;
                if (mag > best) { best = mag; bi = i; }
            }
            // arg-max: within each wavefront by shuffles, then over the
            // wavefronts' winners (largest modulus, lowest row on ties)
#pragma unroll
            for (int off = kW / 2; off > 0; off >>= 1) {
                const double o = __shfl_xor(best, off, kW);
                const int oi = __shfl_xor(bi, off, kW);
                if (o > best || (o == best && oi < bi)) { best = o; bi = oi; }
            }
            if (tid % kW == 0) { s_v[tid / kW] = best; s_i[tid / kW] = bi; }
            __syncthreads();
            double pb = s_v[0];
            int p = s_i[0];
            for (int q = 1; q < nth / kW; ++q)
                if (s_v[q] > pb || (s_v[q] == pb && s_i[q] < p)) { pb = s_v[q]; p = s_i[q]; }
            const bool zero = !(pb > 0.0);
            __syncthreads();
            if (tid == 0) { s_pv[k] = p; if (zero && *info == 0) *info = m + 1; }
            if (zero) continue;
            if (p != k)
                for (int q = tid; q < n; q += nth) {
                    const double2 t = a[(int64_t)k * ld + q];
                    a[(int64_t)k * ld + q] = a[(int64_t)p * ld + q];
                    a[(int64_t)p * ld + q] = t;
                }
            __syncthreads();
            const double2 d = a[(int64_t)k * ld + k];
            const double dn = d.x * d.x + d.y * d.y;
            const double2 inv = {d.x / dn, -d.y / dn};
            for (int i = k + 1 + tid; i < n; i += nth) a[(int64_t)i * ld + k] = cmul(a[(int64_t)i * ld + k], inv);
            __syncthreads();
            const int rc = je - k - 1;   // remaining panel columns
            if (rc > 0)
                for (int64_t id = tid; id < (int64_t)(n - k - 1) * rc; id += nth) {
                    const int i = k + 1 + (int)(id / rc), q = k + 1 + (int)(id % rc);
                    double2 &t = a[(int64_t)i * ld + q];
                    t = csub(t, cmul(a[(int64_t)i * ld + k], a[(int64_t)k * ld + q]));
                }
            __syncthreads();
        }
        if (je >= n) break;
        const int nr = n - je;
        // 2. U12 = L11^-1 A12 (unit lower L11), one thread per column
        for (int q = je + tid; q < n; q += nth) {
            for (int r = 0; r < jw; ++r) {
                double2 t = a[(int64_t)(j0 + r) * ld + q];
                for (int c = 0; c < r; ++c)
                    t = csub(t, cmul(a[(int64_t)(j0 + r) * ld + j0 + c], s_U[c * nr + (q - je)]));
                a[(int64_t)(j0 + r) * ld + q] = t;
                s_U[r * nr + (q - je)] = t;
            }
        }
        for (int64_t id = tid; id < (int64_t)nr * jw; id += nth) {
            const int i = (int)(id / jw), c = (int)(id % jw);
            s_L[i * jw + c] = a[(int64_t)(je + i) * ld + j0 + c];
        }
        __syncthreads();
        // 3. A22 -= L21 U12
        for (int64_t id = tid; id < (int64_t)nr * nr; id += nth) {
            const int i = (int)(id / nr), q = (int)(id % nr);
            double2 t = a[(int64_t)(je + i) * ld + je + q];
            for (int c = 0; c < jw; ++c) t = csub(t, cmul(s_L[i * jw + c], s_U[c * nr + q]));
            a[(int64_t)(je + i) * ld + je + q] = t;
        }
        __syncthreads();
    }
    // the interchanges as one gather: row i of P A is row pv[i] of A
    __syncthreads();
    if (tid == 0) {
        for (int i = 0; i < n; ++i) s_L[i].x = i;
        for (int k = 0; k < n; ++k) {
            const int p = s_pv[k];
            const double t = s_L[k].x;
            s_L[k].x = s_L[p].x;
            s_L[p].x = t;
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += nth) pv[i] = (int32_t)s_L[i].x;
}

// Inverse of every block from its LU factors: A^-1 e_j for kCols columns j
// per workgroup, solving L U x = P e_j in panels of 64 rows.  The panel's
// diagonal block is staged in LDS and solved by one wavefront per column
// with lane shuffles; every remaining row of every column is then updated
// with the panel's solution.  The factors are read once per workgroup.
// Instantiated as (512, 8) and (1024, 4) like the factorisation.
template <int MAXN, int kCols>
__global__ __launch_bounds__(1024) void k_mbj_inverse(int64_t n2, int B, const double2 *LU,
                                                      const int32_t *piv, double2 *Minv) {
    __shared__ double2 y[kCols][MAXN];
    __shared__ double2 s_P[kW][kW + 1];
    const int m = blockIdx.x, tid = threadIdx.x, lane = tid % kW, wv = tid / kW;
    const int b = (int)min((int64_t)B, n2 - (int64_t)m * B);
    const int n = 2 * b, ld = 2 * B;
    const int c0 = blockIdx.y * kCols;
    if (c0 >= n) return;
    const int nc = min(kCols, n - c0);
    const double2 *a = LU + (int64_t)m * ld * ld;
    const int32_t *pv = piv + (int64_t)m * ld;
    for (int id = tid; id < nc * n; id += blockDim.x) {
        const int c = id / n, r = id % n;
        y[c][r] = double2{pv[r] == c0 + c ? 1.0 : 0.0, 0.0};   // (P e_j)[r]
    }
    __syncthreads();
    // forward substitution, unit L
    for (int p0 = 0; p0 < n; p0 += kW) {
        const int pw = min(kW, n - p0);
        for (int id = tid; id < pw * pw; id += blockDim.x)
            s_P[id / pw][id % pw] = a[(int64_t)(p0 + id / pw) * ld + p0 + id % pw];
        __syncthreads();
        if (wv < nc) {
            double2 yi = lane < pw ? y[wv][p0 + lane] : double2{0, 0};
            for (int k = 0; k < pw - 1; ++k) {
                const double2 yk = {__shfl(yi.x, k, kW), __shfl(yi.y, k, kW)};
                if (lane > k && lane < pw) yi = csub(yi, cmul(s_P[lane][k], yk));
            }
            if (lane < pw) y[wv][p0 + lane] = yi;
        }
        __syncthreads();
        const int rows = n - p0 - pw;
        for (int id = tid; id < rows * nc; id += blockDim.x) {
            const int i = p0 + pw + id / nc, c = id % nc;
            const double2 *row = a + (int64_t)i * ld + p0;
            double2 acc = y[c][i];
#pragma unroll 8
            for (int k = 0; k < pw; ++k) acc = csub(acc, cmul(row[k], y[c][p0 + k]));
            y[c][i] = acc;
        }
        __syncthreads();
    }
    // backward substitution, U
    for (int pe = n; pe > 0; pe -= kW) {
        const int p0 = max(0, pe - kW), pw = pe - p0;
        for (int id = tid; id < pw * pw; id += blockDim.x)
            s_P[id / pw][id % pw] = a[(int64_t)(p0 + id / pw) * ld + p0 + id % pw];
        __syncthreads();
        if (wv < nc) {
            double2 yi = lane < pw ? y[wv][p0 + lane] : double2{0, 0};
            for (int k = pw - 1; k >= 0; --k) {
                if (lane == k) {
                    const double2 d = s_P[k][k];
                    const double dn = d.x * d.x + d.y * d.y;
                    yi = cmul(yi, double2{d.x / dn, -d.y / dn});
                }
                const double2 yk = {__shfl(yi.x, k, kW), __shfl(yi.y, k, kW)};
                if (lane < k) yi = csub(yi, cmul(s_P[lane][k], yk));
            }
            if (lane < pw) y[wv][p0 + lane] = yi;
        }
        __syncthreads();
        for (int id = tid; id < p0 * nc; id += blockDim.x) {
            const int i = id / nc, c = id % nc;
            const double2 *row = a + (int64_t)i * ld + p0;
            double2 acc = y[c][i];
#pragma unroll 8
            for (int k = 0; k < pw; ++k) acc = csub(acc, cmul(row[k], y[c][p0 + k]));
            y[c][i] = acc;
        }
        __syncthreads();
    }
    double2 *x = Minv + (int64_t)m * ld * ld;
    for (int id = tid; id < nc * n; id += blockDim.x) {
        const int r = id / nc, c = id % nc;
        x[(int64_t)r * ld + c0 + c] = y[c][r];
    }
}

// ---- block-Jacobi setup for large blocks: panel kernels + FP64 MFMA GEMM --
// For blocks of 2B >= kMbjGemmMin rows the factorisation and the inverse
// run on every compute unit: the blocks are padded to ld x ld with the
// identity (so that every block of the batch has one shape), each panel of
// kMbjPW columns is factorised by one workgroup per block, the trailing
// matrix is updated by the batched complex GEMM, and the inverse is formed
// column-wise as X^T = (U^-1 L^-1 P)^T: per panel of 64 rows a triangular
// solve of the diagonal block for every column (one wavefront each), then a
// GEMM update of the remaining rows; X^T is transposed in place at the end.
constexpr int kMbjPW = 16;
constexpr int kMbjGemmMin = 128;

// Rows and columns n .. ld-1 of the last block become the identity.
__global__ void k_mbj_pad(int ld, int n, double2 *A) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= (int64_t)ld * ld) return;
    const int r = (int)(id / ld), q = (int)(id % ld);
    if (r >= n || q >= n) A[id] = {r == q ? 1.0 : 0.0, 0.0};
}

// Columns j0 .. j0 + kMbjPW - 1 of every block, held in registers (thread t
// owns row j0 + t of the panel): partial pivoting over the rows below the
// diagonal, the interchange (recorded in swp; k_mbj_laswp applies it to the
// columns outside the panel), scaling of the column below the pivot and
// the rank-one update of the panel's remaining columns.
__global__ __launch_bounds__(1024) void k_mbj_panel(int ld, int j0, double2 *A, int32_t *swp, int32_t *info) {
    __shared__ double s_v[1024 / kW];
    __shared__ int s_i[1024 / kW];
    __shared__ double2 s_k[kMbjPW], s_p[kMbjPW];   // rows k and p before the interchange
    const int m = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
    double2 *a = A + (int64_t)m * ld * ld;
    const int jw = min(kMbjPW, ld - j0);
    const int i = j0 + tid;
    const bool own = i < ld;
    double2 r[kMbjPW];
#pragma unroll
    for (int c = 0; c < kMbjPW; ++c) r[c] = (own && c < jw) ? a[(int64_t)i * ld + j0 + c] : double2{0, 0};
#pragma unroll
    for (int kk = 0; kk < kMbjPW; ++kk) {
        if (kk < jw) {
            const int k = j0 + kk;
            double best = (own && i >= k) ? r[kk].x * r[kk].x + r[kk].y * r[kk].y : -1.0;
            int bi = i;
#pragma unroll
            for (int off = kW / 2; off > 0; off >>= 1) {
                const double o = __shfl_xor(best, off, kW);
                const int oi = __shfl_xor(bi, off, kW);
                if (o > best || (o == best && oi < bi)) { best = o; bi = oi; }
            }
            if (tid % kW == 0) { s_v[tid / kW] = best; s_i[tid / kW] = bi; }
            __syncthreads();
            double pb = s_v[0];
            int p = s_i[0];
            for (int q = 1; q < nth / kW; ++q)
                if (s_v[q] > pb || (s_v[q] == pb && s_i[q] < p)) { pb = s_v[q]; p = s_i[q]; }
            const bool zero = !(pb > 0.0);
            if (zero) p = k;
            if (tid == 0) {
                swp[(int64_t)m * ld + k] = p;
                if (zero) atomicCAS(info, 0, m + 1);
            }
            if (i == k) {
#pragma unroll
                for (int c = 0; c < kMbjPW; ++c) s_k[c] = r[c];
            }
            if (i == p) {
#pragma unroll
                for (int c = 0; c < kMbjPW; ++c) s_p[c] = r[c];
            }
            __syncthreads();
            if (!zero) {
                if (i == k && p != k) {
#pragma unroll
                    for (int c = 0; c < kMbjPW; ++c) r[c] = s_p[c];
                } else if (i == p && p != k) {
#pragma unroll
                    for (int c = 0; c < kMbjPW; ++c) r[c] = s_k[c];
                }
                // the pivot row is the former row p
                const double2 d = s_p[kk];
                const double dn = d.x * d.x + d.y * d.y;
                const double2 inv = {d.x / dn, -d.y / dn};
                if (own && i > k) {
                    const double2 l = cmul(r[kk], inv);
                    r[kk] = l;
#pragma unroll
                    for (int c = kk + 1; c < kMbjPW; ++c) r[c] = csub(r[c], cmul(l, s_p[c]));
                }
            }
            // s_k, s_p are rewritten only after the next step's first barrier
        }
    }
    if (own)
#pragma unroll
        for (int c = 0; c < kMbjPW; ++c)
            if (c < jw) a[(int64_t)i * ld + j0 + c] = r[c];
}

// The interchanges of panel j0 applied to every column outside the panel
// (one thread per column, in the order they were chosen).
__global__ __launch_bounds__(256) void k_mbj_laswp(int ld, int j0, double2 *A, const int32_t *swp) {
    const int m = blockIdx.y;
    const int jw = min(kMbjPW, ld - j0);
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ld - jw) return;
    if (q >= j0) q += jw;                     // skip the panel's columns
    double2 *a = A + (int64_t)m * ld * ld;
    const int32_t *sw = swp + (int64_t)m * ld;
    for (int k = j0; k < j0 + jw; ++k) {
        const int p = sw[k];
        if (p != k) {
            const double2 t = a[(int64_t)k * ld + q];
            a[(int64_t)k * ld + q] = a[(int64_t)p * ld + q];
            a[(int64_t)p * ld + q] = t;
        }
    }
}

// U12 = L11^-1 A12 for the columns right of the panel (one thread per
// column, L11 staged in LDS), written in place and transposed into UT
// ([column][panel row], leading dimension kMbjPW) for the GEMM.
__global__ __launch_bounds__(256) void k_mbj_trsm(int ld, int j0, double2 *A, double2 *UT) {
    __shared__ double2 sL[kMbjPW][kMbjPW + 1];
    const int m = blockIdx.y, tid = threadIdx.x;
    const int je = min(j0 + kMbjPW, ld), jw = je - j0;
    double2 *a = A + (int64_t)m * ld * ld;
    for (int t = tid; t < jw * jw; t += blockDim.x) sL[t / jw][t % jw] = a[(int64_t)(j0 + t / jw) * ld + j0 + t % jw];
    __syncthreads();
    const int q = je + blockIdx.x * blockDim.x + tid;
    if (q >= ld) return;
    double2 u[kMbjPW];
    double2 *ut = UT + (int64_t)m * ld * kMbjPW + (int64_t)(q - je) * kMbjPW;
#pragma unroll
    for (int r = 0; r < kMbjPW; ++r) {
        if (r < jw) {
            double2 t = a[(int64_t)(j0 + r) * ld + q];
#pragma unroll
            for (int c = 0; c < r; ++c) t = csub(t, cmul(sL[r][c], u[c]));
            u[r] = t;
            a[(int64_t)(j0 + r) * ld + q] = t;
            ut[r] = t;
        }
    }
}

// The interchanges of every block as one gather: row i of P A is row
// pv[i] of A (composed in LDS by one thread per block).
__global__ __launch_bounds__(64) void k_mbj_perm(int ld, const int32_t *swp, int32_t *pv) {
    __shared__ int32_t o[1024], sw[1024];
    const int m = blockIdx.x;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        o[i] = i;
        sw[i] = swp[(int64_t)m * ld + i];
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < ld; ++k) {
            const int p = sw[k];
            const int32_t t = o[k];
            o[k] = o[p];
            o[p] = t;
        }
    __syncthreads();
    for (int i = threadIdx.x; i < ld; i += blockDim.x) pv[(int64_t)m * ld + i] = o[i];
}

// X^T[j][r] = (P e_j)[r]
__global__ void k_mbj_inv_init(int ld, int nb, const int32_t *pv, double2 *XT) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)ld * ld;
    if (id >= per * nb) return;
    const int64_t m = id / per, r = id % per;
    const int j = (int)(r / ld), i = (int)(r % ld);
    XT[id] = {pv[m * ld + i] == j ? 1.0 : 0.0, 0.0};
}

// Rows p0 .. p0 + pw of every column j: solve with the diagonal block of L
// (unit, UPPER = false) or U (UPPER = true); one wavefront per two columns
// (two independent shuffle chains), the reciprocals of U's diagonal formed
// once per workgroup.
template <bool UPPER>
__global__ __launch_bounds__(1024) void k_mbj_inv_diag(int ld, int p0, int pw, const double2 *LU, double2 *XT) {
    __shared__ double2 s_P[kW][kW + 1];
    __shared__ double2 s_inv[kW];
    const int m = blockIdx.y, tid = threadIdx.x, lane = tid % kW, wv = tid / kW;
    const double2 *a = LU + (int64_t)m * ld * ld;
    for (int id = tid; id < pw * pw; id += blockDim.x)
        s_P[id / pw][id % pw] = a[(int64_t)(p0 + id / pw) * ld + p0 + id % pw];
    if (UPPER && tid < pw) {
        const double2 d = a[(int64_t)(p0 + tid) * ld + p0 + tid];
        const double dn = d.x * d.x + d.y * d.y;
        s_inv[tid] = {d.x / dn, -d.y / dn};
    }
    __syncthreads();
    const int j = 2 * (blockIdx.x * (blockDim.x / kW) + wv);
    if (j >= ld) return;
    const bool two = j + 1 < ld;
    double2 *x0 = XT + (int64_t)m * ld * ld + (int64_t)j * ld + p0;
    double2 *x1 = x0 + ld;
    double2 y0 = lane < pw ? x0[lane] : double2{0, 0};
    double2 y1 = (two && lane < pw) ? x1[lane] : double2{0, 0};
    if (!UPPER) {
        for (int k = 0; k < pw - 1; ++k) {
            const double2 a0 = {__shfl(y0.x, k, kW), __shfl(y0.y, k, kW)};
            const double2 a1 = {__shfl(y1.x, k, kW), __shfl(y1.y, k, kW)};
            if (lane > k && lane < pw) {
                const double2 l = s_P[lane][k];
                y0 = csub(y0, cmul(l, a0));
                y1 = csub(y1, cmul(l, a1));
            }
        }
    } else {
        for (int k = pw - 1; k >= 0; --k) {
            if (lane == k) {
                y0 = cmul(y0, s_inv[k]);
                y1 = cmul(y1, s_inv[k]);
            }
            const double2 a0 = {__shfl(y0.x, k, kW), __shfl(y0.y, k, kW)};
            const double2 a1 = {__shfl(y1.x, k, kW), __shfl(y1.y, k, kW)};
            if (lane < k) {
                const double2 u = s_P[lane][k];
                y0 = csub(y0, cmul(u, a0));
                y1 = csub(y1, cmul(u, a1));
            }
        }
    }
    if (lane < pw) {
        x0[lane] = y0;
        if (two) x1[lane] = y1;
    }
}

// In-place transpose of every ld x ld block, 32 x 32 tiles: the workgroup
// of tile (ti, tj), ti <= tj, swaps it with tile (tj, ti).
__global__ __launch_bounds__(256) void k_mbj_transpose(int ld, double2 *X) {
    __shared__ double2 t0[32][33], t1[32][33];
    const int nt = (ld + 31) / 32;
    int ti = 0, rem = blockIdx.x;
    while (rem >= nt - ti) { rem -= nt - ti; ++ti; }
    const int tj = ti + rem;
    double2 *x = X + (int64_t)blockIdx.y * ld * ld;
    for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
        const int r = e / 32, c = e % 32;
        const int i0 = ti * 32 + r, j0 = tj * 32 + c, i1 = tj * 32 + r, j1 = ti * 32 + c;
        if (i0 < ld && j0 < ld) t0[r][c] = x[(int64_t)i0 * ld + j0];
        if (i1 < ld && j1 < ld) t1[r][c] = x[(int64_t)i1 * ld + j1];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
        const int r = e / 32, c = e % 32;
        const int i0 = ti * 32 + r, j0 = tj * 32 + c, i1 = tj * 32 + r, j1 = ti * 32 + c;
        if (i0 < ld && j0 < ld) x[(int64_t)i0 * ld + j0] = t1[c][r];
        if (i1 < ld && j1 < ld) x[(int64_t)i1 * ld + j1] = t0[c][r];
    }
}

// C[b][m] += alpha sum_k A[m][k] B[b][k] over the nb blocks (strides ld^2;
// sa overrides A's stride)
static int mbj_gemm(const double2 *A, int64_t lda, int64_t sa, const double2 *B, int64_t ldb, double2 *C,
                    int64_t ldc, int64_t ld, int64_t M, int64_t Nb, int64_t K, int nb, hipStream_t s) {
    if (M <= 0 || Nb <= 0 || K <= 0) return MBEM_OK;
    CgemmList L;
    L.np = 1;
    CgemmProb &P = L.p[0];
    P.A = A; P.lda = lda; P.sa = sa;
    P.B = B; P.ldb = ldb; P.sb = ld * ld;
    P.C = C; P.ldc = ldc; P.sc = ld * ld;
    P.M = M; P.Nb = Nb; P.K = K; P.batch = nb;
    return cgemm_f64_run(L, false, false, 1, nullptr, s, true, -1.0);
}

// LU (in LUbuf, [nb][ld][ld], gathered and padded) and inverses (Minv) of
// every block; UT: ld * kMbjPW per block; swp, pv: ld per block.
static int mbj_factor_invert_gemm(int ld, int nb, int n_last, double2 *LUb, int32_t *swp, int32_t *pv,
                                  int32_t *info, double2 *UT, double2 *Minv, hipStream_t s) {
    if (n_last < ld) {
        const int64_t tot = (int64_t)ld * ld;
        hipLaunchKernelGGL(k_mbj_pad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ld, n_last,
                           LUb + (int64_t)(nb - 1) * ld * ld);
        MBEM_HIP(hipGetLastError());
    }
    for (int j0 = 0; j0 < ld; j0 += kMbjPW) {
        const int je = std::min(j0 + kMbjPW, ld);
        hipLaunchKernelGGL(k_mbj_panel, dim3(nb), dim3(1024), 0, s, ld, j0, LUb, swp, info);
        MBEM_HIP(hipGetLastError());
        if (ld - (je - j0) > 0) {
            hipLaunchKernelGGL(k_mbj_laswp, dim3((unsigned)((ld - (je - j0) + 255) / 256), nb), dim3(256), 0, s, ld,
                               j0, LUb, (const int32_t *)swp);
            MBEM_HIP(hipGetLastError());
        }
        if (je >= ld) break;
        hipLaunchKernelGGL(k_mbj_trsm, dim3((unsigned)((ld - je + 255) / 256), nb), dim3(256), 0, s, ld, j0, LUb, UT);
        MBEM_HIP(hipGetLastError());
        MBEM_TRY(mbj_gemm(UT, kMbjPW, (int64_t)ld * kMbjPW, LUb + (int64_t)je * ld + j0, ld,
                          LUb + (int64_t)je * ld + je, ld, ld, ld - je, ld - je, je - j0, nb, s));
    }
    hipLaunchKernelGGL(k_mbj_perm, dim3(nb), dim3(64), 0, s, ld, (const int32_t *)swp, pv);
    MBEM_HIP(hipGetLastError());
    const int64_t tot = (int64_t)ld * ld * nb;
    hipLaunchKernelGGL(k_mbj_inv_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ld, nb, pv, Minv);
    MBEM_HIP(hipGetLastError());
    const dim3 gd((unsigned)((ld + 31) / 32), nb);
    for (int p0 = 0; p0 < ld; p0 += kW) {
        const int pw = std::min(kW, ld - p0);
        hipLaunchKernelGGL(k_mbj_inv_diag<false>, gd, dim3(1024), 0, s, ld, p0, pw, LUb, Minv);
        MBEM_HIP(hipGetLastError());
        MBEM_TRY(mbj_gemm(LUb + (int64_t)(p0 + pw) * ld + p0, ld, (int64_t)ld * ld, Minv + p0, ld,
                          Minv + p0 + pw, ld, ld, ld - p0 - pw, ld, pw, nb, s));
    }
    for (int pe = ld; pe > 0; pe -= kW) {
        const int p0 = std::max(0, pe - kW), pw = pe - p0;
        hipLaunchKernelGGL(k_mbj_inv_diag<true>, gd, dim3(1024), 0, s, ld, p0, pw, LUb, Minv);
        MBEM_HIP(hipGetLastError());
        MBEM_TRY(mbj_gemm(LUb + p0, ld, (int64_t)ld * ld, Minv + p0, ld, Minv, ld, ld, p0, ld, pw, nb, s));
    }
    const int nt = (ld + 31) / 32;
    hipLaunchKernelGGL(k_mbj_transpose, dim3((unsigned)(nt * (nt + 1) / 2), nb), dim3(256), 0, s, ld, Minv);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

__device__ inline double2 ld_c(const double2 *p) { return *p; }
__device__ inline double2 ld_c(const float2 *p) { const float2 v = *p; return {(double)v.x, (double)v.y}; }

// z = blockdiag(A_m^-1) v; one wavefront per row of a block.  TM: the
// stored inverses' type (complex128, or the complex64 copy); FP64 sums.
template <typename TM>
__global__ __launch_bounds__(256) void k_mbj_apply(int64_t n2, int B, int nb, const TM *Minv,
                                                   const double2 *v, double2 *z) {
    const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kW;
    const int lane = threadIdx.x % kW;
    const int64_t ld = 2 * B;
    const int64_t m = wid / ld, r = wid % ld;
    if (m >= nb) return;
    const int64_t b = min((int64_t)B, n2 - m * B);
    const int64_t n = 2 * b;
    if (r >= n) return;
    const TM *row = Minv + m * ld * ld + r * ld;
    double re = 0, im = 0;
    for (int64_t q = lane; q < n; q += kW) {
        const int64_t g = (q < b ? 0 : n2) + m * B + (q % b);
        const double2 a = ld_c(row + q), x = v[g];
        re += a.x * x.x - a.y * x.y;
        im += a.x * x.y + a.y * x.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) z[(r < b ? 0 : n2) + m * B + (r % b)] = {re, im};
}

int mbj_setup_run(mbem_op *op, int B, hipStream_t s, bool keep) {
    // the transposed inverses belong to the previous blocks (and so does the
    // complex64 copy, which is rewritten below; its allocation is kept when
    // the size matches)
    if (op->d_minv_t) { MBEM_HIP(hipFree(op->d_minv_t)); op->d_minv_t = nullptr; }
    if (op->d_minv_t32) { MBEM_HIP(hipFree(op->d_minv_t32)); op->d_minv_t32 = nullptr; }
    op->B = 0; op->nb = 0;
    if (B > kMaxBlock) { set_error("preconditioner block above 512 is not supported"); return MBEM_EINVAL; }
    const int64_t n2 = op->n2;
    if (B > n2) B = (int)n2;
    const int nb = B > 0 ? (int)((n2 + B - 1) / B) : 0;
    const int64_t ld = 2 * (int64_t)B;
    const size_t bytes = B > 0 ? sizeof(double2) * nb * ld * ld : 0;
    // factors and pivots in one scratch allocation: [nb][ld][ld] + [nb][ld] + info
    const size_t lu_bytes = B > 0 ? bytes + sizeof(int32_t) * (nb * ld + 1) : 0;
    if (op->d_minv && op->minv_bytes != bytes) {
        MBEM_HIP(hipFree(op->d_minv)); op->d_minv = nullptr; op->minv_bytes = 0;
        if (op->d_minv32) { MBEM_HIP(hipFree(op->d_minv32)); op->d_minv32 = nullptr; }
    }
    if (op->d_lu && op->lu_bytes != lu_bytes) {
        MBEM_HIP(hipFree(op->d_lu)); op->d_lu = nullptr; op->lu_bytes = 0;
    }
    if (B <= 0) return MBEM_OK;
    if (!op->d_lu) { MBEM_HIP(hipMalloc((void **)&op->d_lu, lu_bytes)); op->lu_bytes = lu_bytes; }
    if (!op->d_minv) { MBEM_HIP(hipMalloc((void **)&op->d_minv, bytes)); op->minv_bytes = bytes; }
    int32_t *piv = (int32_t *)((char *)op->d_lu + bytes);
    int32_t *info = piv + nb * ld;
    MBEM_HIP(hipMemsetAsync(info, 0, sizeof(int32_t), s));
    const mbem_mesh *m = op->mesh;
    dim3 g(64, nb);
    if (op->blr)
        hipLaunchKernelGGL(k_mbj_gather_blr, g, dim3(256), 0, s, n2, B, blr_view(op), m->d_mptr, m->d_mcol,
                           op->d_mval, coef_of(op), op->d_lu);
    else if (op->prec == MBEM_FP64)
        hipLaunchKernelGGL((k_mbj_gather<double2>), g, dim3(256), 0, s, n2, B, op->K[0], op->K[1],
                           op->K[2], m->d_mptr, m->d_mcol, op->d_mval, coef_of(op), NearView{}, op->d_lu);
    else
        hipLaunchKernelGGL((k_mbj_gather<float2>), g, dim3(256), 0, s, n2, B, op->K[0], op->K[1],
                           op->K[2], m->d_mptr, m->d_mcol, op->d_mval, coef_of(op), op->near_view(), op->d_lu);
    MBEM_HIP(hipGetLastError());
    double2 *UT = nullptr;
    int32_t *swp = nullptr;
    if (ld >= kMbjGemmMin) {
        // panels on one workgroup per block, updates on the whole chip
        MBEM_HIP(hipMalloc((void **)&UT, sizeof(double2) * nb * ld * kMbjPW + sizeof(int32_t) * nb * ld));
        swp = (int32_t *)(UT + (int64_t)nb * ld * kMbjPW);
        const int n_last = (int)(2 * (n2 - (int64_t)(nb - 1) * B));
        const int st = mbj_factor_invert_gemm((int)ld, nb, n_last, op->d_lu, swp, piv, info, UT, op->d_minv, s);
        if (st != MBEM_OK) { (void)hipStreamSynchronize(s); (void)hipFree(UT); return st; }
    } else if (ld <= 512) {
        hipLaunchKernelGGL((k_mbj_lu<512, 8>), dim3(nb), dim3(1024), 0, s, n2, B, op->d_lu, piv, info);
        MBEM_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_mbj_inverse<512, 8>), dim3(nb, (unsigned)((ld + 7) / 8)), dim3(1024), 0, s,
                           n2, B, op->d_lu, piv, op->d_minv);
    } else {
        hipLaunchKernelGGL((k_mbj_lu<1024, 4>), dim3(nb), dim3(1024), 0, s, n2, B, op->d_lu, piv, info);
        MBEM_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_mbj_inverse<1024, 4>), dim3(nb, (unsigned)((ld + 3) / 4)), dim3(1024), 0, s,
                           n2, B, op->d_lu, piv, op->d_minv);
    }
    MBEM_HIP(hipGetLastError());
    int32_t h = 0;
    MBEM_HIP(hipMemcpyAsync(&h, info, sizeof(h), hipMemcpyDeviceToHost, s));
    MBEM_HIP(hipStreamSynchronize(s));
    if (UT) MBEM_HIP(hipFree(UT));
    if (!keep) { MBEM_HIP(hipFree(op->d_lu)); op->d_lu = nullptr; op->lu_bytes = 0; }
    if (h) {
        set_error("zero pivot in preconditioner block " + std::to_string(h - 1));
        MBEM_HIP(hipFree(op->d_minv));
        op->d_minv = nullptr;
        op->minv_bytes = 0;
        if (op->d_minv32) { MBEM_HIP(hipFree(op->d_minv32)); op->d_minv32 = nullptr; }
        return MBEM_ESINGULAR;
    }
    op->B = B;
    op->nb = nb;
    if (op->prec == MBEM_MIXED) MBEM_TRY(mbj_copy_c64(op->d_minv, &op->d_minv32, (int64_t)nb * ld * ld, s));
    return MBEM_OK;
}

// The GMRES steps of a MIXED operator apply the inverses rounded to
// complex64 (half the bytes of the product that starts every step); right
// preconditioning takes any fixed P^-1, and the solution is formed with the
// same copy, so only the preconditioner changes, not the system solved.
__global__ void k_round_c64(const double2 *a, float2 *b, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = {(float)a[i].x, (float)a[i].y};
}
int mbj_copy_c64(const double2 *src, float2 **dst, int64_t n, hipStream_t s) {
    if (!*dst) MBEM_HIP(hipMalloc((void **)dst, sizeof(float2) * n));
    hipLaunchKernelGGL(k_round_c64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, *dst, n);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

int mbj_apply_run(const mbem_op *op, const double2 *v, double2 *z, hipStream_t s, bool trans, bool lowp) {
    if (!op->d_minv || op->nb == 0) {
        MBEM_HIP(hipMemcpyAsync(z, v, sizeof(double2) * 2 * op->n2, hipMemcpyDeviceToDevice, s));
        return MBEM_OK;
    }
    const int64_t rows = (int64_t)op->nb * 2 * op->B;
    const dim3 grid((unsigned)((rows * kW + 255) / 256));
    const float2 *m32 = lowp ? (trans ? op->d_minv_t32 : op->d_minv32) : nullptr;
    if (m32)
        hipLaunchKernelGGL(k_mbj_apply<float2>, grid, dim3(256), 0, s, op->n2, op->B, op->nb, m32, v, z);
    else
        hipLaunchKernelGGL(k_mbj_apply<double2>, grid, dim3(256), 0, s, op->n2, op->B, op->nb,
                           (const double2 *)(trans ? op->d_minv_t : op->d_minv), v, z);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

// ---------------------------------------------------- GMRES vectors ---
// Classical Gram-Schmidt with one reorthogonalisation (CGS2) of the new
// Krylov vector w against k orthonormal basis vectors, and its
// normalisation, in four launches over 256-row chunks of the vectors:
//   k_cgs_dots:           partial projections part[j][c] = (V_j^H w) over
//                         chunk c (one workgroup per chunk and 8 vectors)
//   k_cgs_update<true>:   h_j = sum_c part[j][c]; w -= V h over the chunk;
//                         partial projections of the updated w
//   k_cgs_update<false>:  the same second pass, then the chunk's |w|^2
//   k_cgs_scale:          V_k = w / |w|, and the step's Hessenberg column
//                         with a completion tag into host-mapped memory
//                         (with a preconditioner, k_mbj_scale_apply does
//                         this as the first launch of the next step)
// Every reduction runs in a fixed order and every workgroup sums the same
// partials, so all workgroups use bit-identical coefficients.  At the sizes
// of a GMRES step (a 10 248-row vector is 41 chunks) the kernels are bound
// by memory latency and by the cross-lane sums, not by bandwidth: the loads
// of several vectors are issued together, and the sums over a chunk go
// through LDS (eight vectors at a time, each summed by half a wavefront)
// rather than one wavefront-wide sum per vector and wavefront.
constexpr int kChunkN = 256;   // rows per workgroup: four wavefronts, one row per lane
constexpr int kDotG = 8;       // basis vectors per round of chunk sums (one per half-wavefront)
constexpr int kRedG = 64;      // coefficients per round of k_cgs_update (one per four lanes)
static_assert(kDotG * 32 == kChunkN && kRedG * 4 == kChunkN, "one thread group per vector");

// Sum over each row of 16 lanes, returned to every lane of the row (all
// lanes active): the first four steps of wsum_all.
__device__ inline double rsum16(double v) {
    v += dpp_move(v, 0);
    v += dpp_move(v, 1);
    v += dpp_move(v, 2);
    v += dpp_move(v, 3);
    return v;
}

// part[(j0 + g) nch + c] = sum over the workgroup's threads of conj(a[g]) b,
// for j0 + g < k.  sp: kDotG x kChunkN complex of LDS.  Thread t sums the
// products of vector g = t / 32 from threads t % 32 + 32 i (i < 8), then
// each half-wavefront's two rows of 16 lanes are summed.  Every thread of
// the workgroup calls this.
__device__ inline void chunk_dots(const double2 (&a)[kDotG], double2 b, double2 *sp, int j0, int k,
                                  double2 *part, int64_t nch, int64_t c) {
    const int t = threadIdx.x, lane = t % kW, wv = t / kW;
#pragma unroll
    for (int g = 0; g < kDotG; ++g)
        sp[g * kChunkN + t] = {a[g].x * b.x + a[g].y * b.y, a[g].x * b.y - a[g].y * b.x};
    __syncthreads();
    const int g = t / 32, q = t % 32;
    double re = 0, im = 0;
#pragma unroll
    for (int i = 0; i < kChunkN / 32; ++i) {
        const double2 v = sp[g * kChunkN + q + 32 * i];
        re += v.x;
        im += v.y;
    }
    re = rsum16(re);
    im = rsum16(im);
    // vector 2 wv: rows at lanes 0, 16; vector 2 wv + 1: lanes 32, 48
    const double2 s0 = {lane_value(re, 0) + lane_value(re, 16), lane_value(im, 0) + lane_value(im, 16)};
    const double2 s1 = {lane_value(re, 32) + lane_value(re, 48), lane_value(im, 32) + lane_value(im, 48)};
    if (lane == 0) {
        if (j0 + 2 * wv < k) part[(int64_t)(j0 + 2 * wv) * nch + c] = s0;
        if (j0 + 2 * wv + 1 < k) part[(int64_t)(j0 + 2 * wv + 1) * nch + c] = s1;
    }
    __syncthreads();   // sp is reused
}

// a[g] = V_{j0 + g} over the thread's row, 0 outside the vectors
__device__ inline void load_rows(double2 (&a)[kDotG], const double2 *V, int64_t ldv, int j0, int k, int64_t i,
                                 bool in) {
#pragma unroll
    for (int g = 0; g < kDotG; ++g) a[g] = (in && j0 + g < k) ? V[(int64_t)(j0 + g) * ldv + i] : double2{0, 0};
}

// grid (xdim, ceil(k / kDotG)) with xdim >= nch a multiple of 8, so that
// workgroup (c, y) runs on the same XCD as workgroup c of the update
// kernels (workgroups are dealt to the eight XCDs in launch order)
__global__ __launch_bounds__(kChunkN) void k_cgs_dots(const double2 *V, int64_t ldv, int k, const double2 *w,
                                                     int64_t n, double2 *part, int64_t nch) {
    __shared__ double2 sp[kDotG * kChunkN];
    const int64_t c = blockIdx.x;
    if (c >= nch) return;   // the whole workgroup
    const int64_t i = c * kChunkN + threadIdx.x;
    const int j0 = blockIdx.y * kDotG;
    const bool in = i < n;
    const double2 b = in ? w[i] : double2{0, 0};
    double2 a[kDotG];
    load_rows(a, V, ldv, j0, k, i, in);
    chunk_dots(a, b, sp, j0, k, part, nch, c);
}

// h_j sums part[j][0 .. npin); w = win - V h (win may be w).  DOTS: `next` receives the partial
// projections of the updated w (the second pass's part, one per chunk);
// otherwise npart[c] receives the chunk's |w|^2.  hout[j] = h_j is written
// by workgroup 0.  One workgroup per chunk.
template <bool DOTS>
__global__ __launch_bounds__(kChunkN) void k_cgs_update(const double2 *win, double2 *w, const double2 *V,
                                                       int64_t ldv, int k, const double2 *part, int64_t npin,
                                                       double2 *hout, int64_t n, double2 *next, double *npart) {
    __shared__ double2 s_h[kRedG];
    __shared__ double2 sp[kDotG * kChunkN];
    const int wv = threadIdx.x / kW, lane = threadIdx.x % kW;
    const int64_t c = blockIdx.x, nch = gridDim.x, i = c * kChunkN + threadIdx.x;
    const bool in = i < n;
    double2 t = in ? win[i] : double2{0, 0};
    for (int j0 = 0; j0 < k; j0 += kRedG) {
        const int nb = k - j0 < kRedG ? k - j0 : kRedG;
        {   // h_{j0 + jj}, jj = thread / 4: each of four lanes sums every fourth chunk
            const int jj = threadIdx.x / 4, q = threadIdx.x % 4;
            double re = 0, im = 0;
            if (jj < nb) {
                const double2 *pj = part + (int64_t)(j0 + jj) * npin;
#pragma unroll 8
                for (int64_t cc = q; cc < npin; cc += 4) {
                    const double2 p = pj[cc];
                    re += p.x;
                    im += p.y;
                }
            }
            re += dpp_move(re, 0);
            re += dpp_move(re, 1);
            im += dpp_move(im, 0);
            im += dpp_move(im, 1);
            if (q == 0 && jj < nb) s_h[jj] = {re, im};
        }
        __syncthreads();
        if (blockIdx.x == 0 && threadIdx.x < nb) hout[j0 + threadIdx.x] = s_h[threadIdx.x];
        if (in) {
#pragma unroll 16
            for (int jj = 0; jj < nb; ++jj) t = csub(t, cmul(V[(int64_t)(j0 + jj) * ldv + i], s_h[jj]));
        }
        __syncthreads();
    }
    if (in) w[i] = t;
    if constexpr (DOTS) {
        // the next batch's rows load while the current batch is summed
        double2 a[kDotG], an[kDotG];
        load_rows(a, V, ldv, 0, k, i, in);
        for (int j0 = 0; j0 < k; j0 += kDotG) {
            if (j0 + kDotG < k) load_rows(an, V, ldv, j0 + kDotG, k, i, in);
            chunk_dots(a, t, sp, j0, k, next, nch, c);
#pragma unroll
            for (int g = 0; g < kDotG; ++g) a[g] = an[g];
        }
    } else {
        const double nn = wsum_all(in ? t.x * t.x + t.y * t.y : 0.0);
        if (lane == 0) sp[wv].x = nn;
        __syncthreads();
        if (threadIdx.x == 0) npart[c] = (sp[0].x + sp[1].x) + (sp[2].x + sp[3].x);
    }
}

// Publication of a step's Hessenberg column by one workgroup (every thread
// of it calls this): pin[0 .. k2) = hcol[0 .. k2), pin[k2].x = h, and last
// *tag = seq, after a system-scope fence of every store before it, so a
// host that sees the tag reads a complete column (pin and tag host-mapped).
__device__ inline void publish_column(const double2 *hcol, int k2, double h, double2 *pin,
                                      unsigned long long *tag, unsigned long long seq) {
    for (int t = threadIdx.x; t < k2; t += blockDim.x) pin[t] = hcol[t];
    if (threadIdx.x == 0) pin[k2] = {h, 0.0};
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(tag, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// |w| from the chunks' parts of |w|^2, the same sum in every wavefront
__device__ inline double norm_from_parts(const double *npart, int64_t nch) {
    double a = 0;
    for (int64_t c = threadIdx.x % kW; c < nch; c += kW) a += npart[c];
    return sqrt(wsum_all(a));
}

// dst = src / h with h = sqrt(sum_c npart[c]) (0 -> dst = 0); with pin,
// workgroup 0 publishes the step's column (publish_column).
__global__ __launch_bounds__(kChunkN) void k_cgs_scale(double2 *dst, const double2 *src, const double *npart,
                                                      int64_t nch, int64_t n, const double2 *hcol, int k2,
                                                      double2 *pin, unsigned long long *tag,
                                                      unsigned long long seq) {
    const double h = norm_from_parts(npart, nch), inv = h > 0 ? 1.0 / h : 0.0;
    const int64_t i = blockIdx.x * (int64_t)kChunkN + threadIdx.x;
    if (i < n) dst[i] = {inv * src[i].x, inv * src[i].y};
    if (blockIdx.x == 0 && pin) publish_column(hcol, k2, h, pin, tag, seq);
}

// The normalisation that ends an Arnoldi step fused with the block-Jacobi
// product that starts the next: V_k = w / |w| and z = P^-1 V_k, one
// wavefront per row of a diagonal block as in k_mbj_apply; the row's sum
// is formed from w and scaled once (z = (P^-1 w) / |w|).  One extra
// workgroup, the first, publishes the finished step's column meanwhile.
template <typename TM>
__global__ __launch_bounds__(256) void k_mbj_scale_apply(int64_t n2, int B, int nb, const TM *Minv,
                                                         const double2 *w, const double *npart, int64_t nch,
                                                         double2 *vk, double2 *z, const double2 *hcol, int k2,
                                                         double2 *pin, unsigned long long *tag,
                                                         unsigned long long seq) {
    if (blockIdx.x == 0) {   // the extra first workgroup publishes
        publish_column(hcol, k2, norm_from_parts(npart, nch), pin, tag, seq);
        return;
    }
    const int64_t wid = ((blockIdx.x - 1) * (int64_t)blockDim.x + threadIdx.x) / kW;
    const int lane = threadIdx.x % kW;
    const int64_t ld = 2 * B;
    const int64_t m = wid / ld, r = wid % ld;
    const int64_t b = m < nb ? min((int64_t)B, n2 - m * B) : 0;
    const int64_t n = 2 * b;
    const bool ok = r < n;   // uniform over the wavefront
    // the loads of the norm's parts and of the row are issued together
    double a = 0;
    for (int64_t c = lane; c < nch; c += kW) a += npart[c];
    double re = 0, im = 0;
    if (ok) {
        const TM *row = Minv + m * ld * ld + r * ld;
        for (int64_t q = lane; q < n; q += kW) {
            const int64_t g = (q < b ? 0 : n2) + m * B + (q % b);
            const double2 e = ld_c(row + q), x = w[g];
            re += e.x * x.x - e.y * x.y;
            im += e.x * x.y + e.y * x.x;
        }
    }
    const double h = sqrt(wsum_all(a)), inv = h > 0 ? 1.0 / h : 0.0;   // as norm_from_parts
    re = wsum_all(re);
    im = wsum_all(im);
    if (ok && lane == 0) {
        const int64_t go = (r < b ? 0 : n2) + m * B + (r % b);
        const double2 x = w[go];
        z[go] = {inv * re, inv * im};
        vk[go] = {inv * x.x, inv * x.y};
    }
}

// r[n] = b[n] - sum_j W[j][n] y[j] (r may be b)
__global__ void k_resid_products(double2 *r, const double2 *b, const double2 *W, int64_t ldw, int k,
                                 const double2 *y, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 s = b[i];
    for (int j = 0; j < k; ++j) s = csub(s, cmul(W[(int64_t)j * ldw + i], y[j]));
    r[i] = s;
}

// out[n] = sum_j V[j][n] y[j]
__global__ void k_combine_basis(double2 *out, const double2 *V, int64_t ldv, int k, const double2 *y,
                                int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 s = {0, 0};
    for (int j = 0; j < k; ++j) s = cadd(s, cmul(V[(int64_t)j * ldv + i], y[j]));
    out[i] = s;
}

__global__ __launch_bounds__(1024) void k_norm2(const double2 *v, int64_t n, double *out) {
    __shared__ double s[16];
    double a = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) a += v[i].x * v[i].x + v[i].y * v[i].y;
    a = wave_sum(a);
    if (threadIdx.x % kW == 0) s[threadIdx.x / kW] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < (int)(blockDim.x / kW); ++i) t += s[i];
        *out = sqrt(t);
    }
}

__global__ void k_scale_copy(double2 *dst, const double2 *src, double2 a, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = cmul(a, src[i]);
}

__global__ void k_axpy(double2 *y, const double2 *x, double2 a, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = cadd(y[i], cmul(a, x[i]));
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

int vec_combine(double2 *out, const double2 *V, int64_t ldv, int k, const double2 *y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_combine_basis, dim3(nblk(n)), dim3(256), 0, s, out, V, ldv, k, y, n);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}
int vec_resid_products(double2 *r, const double2 *b, const double2 *W, int64_t ldw, int k, const double2 *y,
                       int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_resid_products, dim3(nblk(n)), dim3(256), 0, s, r, b, W, ldw, k, y, n);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}
int vec_norm2(const double2 *v, int64_t n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, s, v, n, out);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}
int vec_scale_copy(double2 *dst, const double2 *src, double2 a, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_copy, dim3(nblk(n)), dim3(256), 0, s, dst, src, a, n);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}
int64_t arnoldi_chunks(int64_t n) { return (n + kChunkN - 1) / kChunkN; }
int arnoldi_cgs2(const double2 *win, double2 *w, double2 *V, int64_t ldv, int k, int64_t n, double2 *part,
                 double *npart, double2 *hcol, bool finish, double2 *pin, unsigned long long *tag,
                 unsigned long long seq, hipStream_t s) {
    if (k < 1 || n < 1) return MBEM_EINVAL;
    const int64_t nch = arnoldi_chunks(n);
    double2 *part2 = part + (int64_t)k * nch;
    hipLaunchKernelGGL(k_cgs_dots, dim3((unsigned)((nch + 7) / 8 * 8), (unsigned)((k + kDotG - 1) / kDotG)),
                       dim3(kChunkN), 0, s, V, ldv, k, win, n, part, nch);
    MBEM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cgs_update<true>, dim3((unsigned)nch), dim3(kChunkN), 0, s, win, w, V, ldv, k, part, nch,
                       hcol, n, part2, nullptr);
    MBEM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cgs_update<false>, dim3((unsigned)nch), dim3(kChunkN), 0, s, (const double2 *)w, w, V, ldv,
                       k, part2, nch, hcol + k, n, nullptr, npart);
    MBEM_HIP(hipGetLastError());
    if (finish) MBEM_TRY(arnoldi_finish(w, V, ldv, k, n, npart, hcol, pin, tag, seq, s));
    return MBEM_OK;
}
int arnoldi_finish(const double2 *w, double2 *V, int64_t ldv, int k, int64_t n, const double *npart,
                   const double2 *hcol, double2 *pin, unsigned long long *tag, unsigned long long seq,
                   hipStream_t s) {
    const int64_t nch = arnoldi_chunks(n);
    hipLaunchKernelGGL(k_cgs_scale, dim3((unsigned)nch), dim3(kChunkN), 0, s, V + (int64_t)k * ldv, w, npart,
                       nch, n, hcol, 2 * k, pin, tag, seq);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}
bool mbj_present(const mbem_op *op) { return op->d_minv && op->nb > 0; }
int mbj_scale_apply_run(const mbem_op *op, const double2 *w, const double *npart, int64_t n, double2 *vk,
                        double2 *z, const double2 *hcol, int k, double2 *pin, unsigned long long *tag,
                        unsigned long long seq, hipStream_t s, bool trans, bool lowp) {
    if (!mbj_present(op) || n != 2 * op->n2 || !pin || !tag) return MBEM_EINVAL;
    const int64_t rows = (int64_t)op->nb * 2 * op->B;
    const dim3 grid((unsigned)((rows * kW + 255) / 256 + 1));
    const float2 *m32 = lowp ? (trans ? op->d_minv_t32 : op->d_minv32) : nullptr;
    if (m32)
        hipLaunchKernelGGL(k_mbj_scale_apply<float2>, grid, dim3(256), 0, s, op->n2, op->B, op->nb, m32, w, npart,
                           arnoldi_chunks(n), vk, z, hcol, 2 * k, pin, tag, seq);
    else
        hipLaunchKernelGGL(k_mbj_scale_apply<double2>, grid, dim3(256), 0, s, op->n2, op->B, op->nb,
                           (const double2 *)(trans ? op->d_minv_t : op->d_minv), w, npart, arnoldi_chunks(n), vk,
                           z, hcol, 2 * k, pin, tag, seq);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}
int vec_axpy(double2 *y, const double2 *x, double2 a, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(nblk(n)), dim3(256), 0, s, y, x, a, n);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

}  // namespace mbem

// ------------------------------------------------ allocation-free product --
// mbem_matvec_noalloc: the product of mbem_matvec with its partial sums
// (4 n2 complex values: K1 x_j, K1 x_m, K2e x_m, K2m x_j) in a file-scope
// device array instead of a per-call allocation.  Each device holds its own
// copy of the array; its address is looked up once per device, with that
// device current, and the kernels receive that address (the array's name in
// host code is not a device address).
namespace mbem {
constexpr int64_t kScratchN2 = 65536;                 // largest n2 = 2 n_nodes (4 MiB)
static __device__ __align__(256) double2 scratch[4 * kScratchN2];
namespace {
constexpr int kScratchDevices = 64;
void *g_scratch[kScratchDevices] = {};
std::mutex g_scratch_mu;

int scratch_of(int device, double2 **out) {
    if (device < 0 || device >= kScratchDevices) {
        set_error("device ordinal beyond the library's scratch table");
        return MBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("scratch address: ") + hipGetErrorString(e));
            return MBEM_EDEVICE;
        }
        g_scratch[device] = p;
    }
    *out = (double2 *)g_scratch[device];
    return MBEM_OK;
}
}  // namespace

}  // namespace mbem

extern "C" int mbem_matvec_noalloc(mbem_ctx *ctx, const mbem_op *op, const mbem_c128 *x, int32_t nrhs,
                                   mbem_c128 *y) {
    using namespace mbem;
    if (!ctx || !op || !x || !y || nrhs < 1) { set_error("bad argument"); return MBEM_EINVAL; }
    if (op->n2 > kScratchN2) {
        set_error("mbem_matvec_noalloc: 2 n_nodes = " + std::to_string(op->n2) + " exceeds its scratch limit of " +
                  std::to_string(kScratchN2));
        return MBEM_EINVAL;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) { set_error("hipSetDevice failed"); return MBEM_EDEVICE; }
    double2 *tmp = nullptr;
    MBEM_TRY(scratch_of(ctx->device, &tmp));
    const int64_t N = 2 * op->n2;
    for (int r = 0; r < nrhs; ++r)
        MBEM_TRY(matvec_run(op, (const double2 *)x + r * N, (double2 *)y + r * N, tmp, ctx->stream));
    return MBEM_OK;
}

