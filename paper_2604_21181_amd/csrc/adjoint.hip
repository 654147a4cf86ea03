// Adjoint of the discrete system for gradients of sigma_ext (extension of
// Sec. 6): the transposed product Z^T lambda (no conjugation: the gradient
// of a holomorphic quantity), the transposed block-Jacobi preconditioner,
// and the far-field functional g with g^T x = e . F(r).
#include <algorithm>
#include <type_traits>

#include "mbem_internal.h"
#include "near_store.h"
#include "p2_device.h"

namespace mbem {

// ----------------------------------------------- far-field functional ---
// e . F(r) with F = (i k / 4 pi) r x sum_q e^{-i k r.y} (W j x r - W j_m)
// equals (i k / 4 pi) sum_q e^{-i k r.y} [W j . (e - r (r.e)) - W j_m . (e x r)],
// so with j = sum_i x_j[i,b] N_i t_b and j_m likewise:
//   g_j[i,b] = (i k / 4 pi) sum_q e^{..} W N_i t_b . e_perp
//   g_m[i,b] = -(i k / 4 pi) sum_q e^{..} W N_i t_b . (e x r)
// One thread per quadrature point, added into g with atomics (each node
// receives a few dozen contributions).
__global__ void k_ff_functional(int64_t nt, int64_t n2, const double *__restrict__ qp,
                                const int32_t *__restrict__ tri, const double *__restrict__ frames, int frame,
                                dvec3 r, cx<double> e0, cx<double> e1, cx<double> e2, double ka,
                                double2 *__restrict__ g) {
    const int64_t nq = nt * kQP;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const int64_t el = i / kQP;
    const int q = (int)(i % kQP);
    const dvec3 y = {qp[QX * nq + i], qp[(QX + 1) * nq + i], qp[(QX + 2) * nq + i]};
    const dvec3 t0[2] = {{qp[QT1 * nq + i], qp[(QT1 + 1) * nq + i], qp[(QT1 + 2) * nq + i]},
                         {qp[QT2 * nq + i], qp[(QT2 + 1) * nq + i], qp[(QT2 + 2) * nq + i]}};
    const dvec3 n = {qp[QN * nq + i], qp[(QN + 1) * nq + i], qp[(QN + 2) * nq + i]};
    const double W = qp[QW * nq + i];
    double sn, cs;
    sincos(-ka * dot(r, y), &sn, &cs);
    const double c4 = ka / (4.0 * 3.14159265358979323846);
    const cx<double> pre = cx<double>{0.0, c4} * cx<double>{cs, sn};   // (i k / 4 pi) e^{-i k r.y}
    const cx<double> E[3] = {e0, e1, e2};
    const cx<double> re = r.x * e0 + r.y * e1 + r.z * e2;
    const cx<double> ep[3] = {E[0] - r.x * re, E[1] - r.y * re, E[2] - r.z * re};
    const cx<double> ex[3] = {r.z * E[1] - r.y * E[2], r.x * E[2] - r.z * E[0], r.y * E[0] - r.x * E[1]};
    double xi, eta, w, N[6], d1[6], d2[6];
    rule7(q, xi, eta, w);
    p2_shape(xi, eta, N, d1, d2);
    for (int b = 0; b < 2; ++b) {
        for (int k = 0; k < 6; ++k) {
            const int64_t node = tri[6 * el + k];
            const dvec3 t = frame == 0 ? t0[b] : project_tangent(nodal_tangent(frames, node, b), n);
            const cx<double> tj = t.x * ep[0] + t.y * ep[1] + t.z * ep[2];
            const cx<double> tm = t.x * ex[0] + t.y * ex[1] + t.z * ex[2];
            const cx<double> vj = pre * tj, vm = pre * tm;
            const int64_t row = 2 * node + b;
            const double f = W * N[k];
            unsafeAtomicAdd(&g[row].x, f * vj.re);
            unsafeAtomicAdd(&g[row].y, f * vj.im);
            unsafeAtomicAdd(&g[n2 + row].x, -f * vm.re);
            unsafeAtomicAdd(&g[n2 + row].y, -f * vm.im);
        }
    }
}

int ff_functional_run(const mbem_mesh *m, const mbem_params *p, const double *rhat, const double2 *e,
                      double2 *g, hipStream_t s) {
    const int64_t n2 = 2 * m->nn;
    MBEM_HIP(hipMemsetAsync(g, 0, sizeof(double2) * 2 * n2, s));
    const int64_t nq = m->nt * kQP;
    hipLaunchKernelGGL(k_ff_functional, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, m->nt, n2, m->d_qp,
                       m->d_tri, m->d_frames, p->frame, dvec3{rhat[0], rhat[1], rhat[2]}, cx<double>{e[0].x, e[0].y},
                       cx<double>{e[1].x, e[1].y}, cx<double>{e[2].x, e[2].y}, p->k0, g);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

// ---------------------------------------------------- Z^T product ---
// Partial sums of K^T v over row chunks: one thread per column, reading
// rows of the stored blocks (contiguous across the wavefront).
//   slot 0: K1^T l1, slot 1: K1^T l2, slot 2: K2eps^T l1, slot 3: K2mu^T l2
// Rows per chunk: 256 for the complex128 blocks (a quarter of the partial
// sums to write and add; the adjoint solve to 1e-8 on the 1280-triangle
// sphere 9.33 -> 8.42 ms), 64 for complex64, whose shorter loads need the
// four times larger grid (256 rows: 6.41 -> 7.05 ms)
template <typename TS> constexpr int rows_per_chunk() { return std::is_same<TS, double2>::value ? 256 : 64; }
constexpr int kRowsPerChunkMin = 64;
template <typename TS>
__global__ __launch_bounds__(256) void k_gemvt_part(int64_t n2, const TS *K1, const TS *K2e, const TS *K2m,
                                                    const double2 *l1, const double2 *l2, double2 *part) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    const int which = blockIdx.z;
    if (j >= n2) return;
    constexpr int kRows = rows_per_chunk<TS>();
    const int64_t r0 = chunk * kRows, r1 = min(n2, r0 + kRows);
    const TS *K = which == 0 ? K1 : (which == 1 ? K2e : K2m);
    double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
    for (int64_t i = r0; i < r1; ++i) {
        const TS kv = K[i * n2 + j];
        const double kr = (double)kv.x, ki = (double)kv.y;
        const double2 u = which == 2 ? l2[i] : l1[i];
        a0r += kr * u.x - ki * u.y;
        a0i += kr * u.y + ki * u.x;
        if (which == 0) {
            const double2 v = l2[i];
            a1r += kr * v.x - ki * v.y;
            a1i += kr * v.y + ki * v.x;
        }
    }
    const int64_t nch = gridDim.y;
    double2 *o = part + chunk * 4 * n2;
    (void)nch;
    if (which == 0) { o[j] = {a0r, a0i}; o[n2 + j] = {a1r, a1i}; }
    else o[(1 + which) * n2 + j] = {a0r, a0i};
}

struct TCoef { double2 iw, ce, cm; };
__device__ inline double2 zm(double2 a, double2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// y = Z^T lambda from the summed partials and the mass matrix (symmetric as
// a matrix of unknowns, so M^T l = M l):
//   y_j = (i/w) K1^T l1 + K2mu^T l2 + c_mu M l2
//   y_m = K2eps^T l1 + c_eps M l1 - (i/w) K1^T l2
// A workgroup takes 64 rows; its four wavefronts sum every fourth chunk of
// partials and the four sums are added in a fixed order through LDS.
constexpr int kCombRows = 64;
__global__ __launch_bounds__(256) void k_combine_t(int64_t n2, int nch, const double2 *__restrict__ part,
                                                   const int32_t *__restrict__ mptr,
                                                   const int32_t *__restrict__ mcol,
                                                   const double *__restrict__ mval,
                                                   const double2 *__restrict__ l1,
                                                   const double2 *__restrict__ l2, TCoef c, NearView nv,
                                                   double2 *__restrict__ y) {
    __shared__ double2 s_t[4][4][kCombRows];   // [group][slot][row]
    const int lr = threadIdx.x % kCombRows, grp = threadIdx.x / kCombRows;
    const int64_t r = blockIdx.x * (int64_t)kCombRows + lr;
    double2 t[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    if (r < n2)
        for (int ch = grp; ch < nch; ch += 4)
            for (int k = 0; k < 4; ++k) {
                const double2 v = part[((int64_t)ch * 4 + k) * n2 + r];
                t[k].x += v.x; t[k].y += v.y;
            }
    for (int k = 0; k < 4; ++k) s_t[grp][k][lr] = t[k];
    __syncthreads();
    if (grp != 0 || r >= n2) return;
    for (int k = 0; k < 4; ++k) {
        t[k] = s_t[0][k][lr];
        for (int g = 1; g < 4; ++g) { t[k].x += s_t[g][k][lr].x; t[k].y += s_t[g][k][lr].y; }
    }
    const int64_t i = r / 2;
    const int al = (int)(r % 2);
    if (nv.bits) {
        // the near store, transposed: output row 2 i + al (column of Z)
        // takes V(k, i)[4 op + 2 a + al] of every stored pair (k, i) times l
        // at 2 k + a; the pattern is symmetric, so row i lists every k
        for (int32_t s = nv.rptr[i]; s < nv.rptr[i + 1]; ++s) {
            const int64_t k = nv.col[s];
            const int64_t sk = near_slot(nv, k, i);
            if (sk < 0) continue;
            const double2 *V = nv.val + 12 * sk + al;
            const double2 a0 = l1[2 * k], a1 = l1[2 * k + 1], b0 = l2[2 * k], b1 = l2[2 * k + 1];
            const double2 p0 = zm(V[0], a0), p1 = zm(V[2], a1), q0 = zm(V[0], b0), q1 = zm(V[2], b1);
            const double2 e0 = zm(V[4], a0), e1 = zm(V[6], a1), m0 = zm(V[8], b0), m1 = zm(V[10], b1);
            t[0].x += p0.x + p1.x; t[0].y += p0.y + p1.y;
            t[1].x += q0.x + q1.x; t[1].y += q0.y + q1.y;
            t[2].x += e0.x + e1.x; t[2].y += e0.y + e1.y;
            t[3].x += m0.x + m1.x; t[3].y += m0.y + m1.y;
        }
    }
    double2 M1 = {0, 0}, M2 = {0, 0};
    for (int32_t s = mptr[i]; s < mptr[i + 1]; ++s) {
        const int64_t col = 2 * (int64_t)mcol[s];
        const double v0 = mval[4 * s + 2 * al], v1 = mval[4 * s + 2 * al + 1];
        M1.x += v0 * l1[col].x + v1 * l1[col + 1].x; M1.y += v0 * l1[col].y + v1 * l1[col + 1].y;
        M2.x += v0 * l2[col].x + v1 * l2[col + 1].x; M2.y += v0 * l2[col].y + v1 * l2[col + 1].y;
    }
    const double2 a = zm(c.iw, t[0]), b = zm(c.iw, t[1]), cm = zm(c.cm, M2), ce = zm(c.ce, M1);
    y[r] = {a.x + t[3].x + cm.x, a.y + t[3].y + cm.y};
    y[n2 + r] = {t[2].x + ce.x - b.x, t[2].y + ce.y - b.y};
}

int matvec_t_run(const mbem_op *op, const double2 *x, double2 *y, double2 *part, hipStream_t s) {
    const int64_t n2 = op->n2;
    const int rows = op->prec == MBEM_FP64 ? rows_per_chunk<double2>() : rows_per_chunk<float2>();
    const int nch = (int)((n2 + rows - 1) / rows);
    const dim3 grid((unsigned)((n2 + 255) / 256), (unsigned)nch, 3);
    if (op->prec == MBEM_FP64)
        hipLaunchKernelGGL((k_gemvt_part<double2>), grid, dim3(256), 0, s, n2, (const double2 *)op->K[0],
                           (const double2 *)op->K[1], (const double2 *)op->K[2], x, x + n2, part);
    else
        hipLaunchKernelGGL((k_gemvt_part<float2>), grid, dim3(256), 0, s, n2, (const float2 *)op->K[0],
                           (const float2 *)op->K[1], (const float2 *)op->K[2], x, x + n2, part);
    MBEM_HIP(hipGetLastError());
    const mbem_mesh *m = op->mesh;
    hipLaunchKernelGGL(k_combine_t, dim3((unsigned)((n2 + kCombRows - 1) / kCombRows)), dim3(256), 0, s, n2, nch,
                       part, m->d_mptr,
                       m->d_mcol, op->d_mval, x, x + n2, TCoef{op->iw, op->ce, op->cm}, op->near_view(), y);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

int64_t matvec_t_work(const mbem_op *op) {
    const int64_t nch = (op->n2 + kRowsPerChunkMin - 1) / kRowsPerChunkMin;   // enough for either
    return nch * 4 * op->n2;
}

// ------------------------------------- transposed preconditioner ---
__global__ void k_transpose_blocks(int64_t nb, int64_t ld, const double2 *A, double2 *At) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nb * ld * ld) return;
    const int64_t m = id / (ld * ld), t = id % (ld * ld), r = t / ld, c = t % ld;
    At[m * ld * ld + c * ld + r] = A[id];
}

int mbj_transpose_run(mbem_op *op, hipStream_t s) {
    if (!op->d_minv || op->nb == 0 || op->d_minv_t) return MBEM_OK;
    const int64_t ld = 2 * (int64_t)op->B, n = (int64_t)op->nb * ld * ld;
    MBEM_HIP(hipMalloc((void **)&op->d_minv_t, sizeof(double2) * n));
    hipLaunchKernelGGL(k_transpose_blocks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (int64_t)op->nb, ld,
                       (const double2 *)op->d_minv, op->d_minv_t);
    MBEM_HIP(hipGetLastError());
    if (op->prec == MBEM_MIXED) MBEM_TRY(mbj_copy_c64(op->d_minv_t, &op->d_minv_t32, n, s));
    return MBEM_OK;
}

// out = sum_i a_i b_i (no conjugation); one workgroup
__global__ __launch_bounds__(1024) void k_dotu(const double2 *a, const double2 *b, int64_t n, double2 *out) {
    __shared__ double sr[16], si[16];
    double re = 0.0, im = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 u = a[i], v = b[i];
        re += u.x * v.x - u.y * v.y;
        im += u.x * v.y + u.y * v.x;
    }
    for (int o = 32; o > 0; o >>= 1) { re += __shfl_down(re, o, 64); im += __shfl_down(im, o, 64); }
    if (threadIdx.x % 64 == 0) { sr[threadIdx.x / 64] = re; si[threadIdx.x / 64] = im; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 t = {0.0, 0.0};
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) { t.x += sr[w]; t.y += si[w]; }
        *out = t;
    }
}

int dotu_run(const double2 *a, const double2 *b, int64_t n, double2 *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dotu, dim3(1), dim3(1024), 0, s, a, b, n, out);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

}  // namespace mbem
