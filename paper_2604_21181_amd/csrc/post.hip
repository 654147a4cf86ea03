// Excitation and post-processing: plane-wave right-hand sides (eqs. rhs_E,
// rhs_H), far field of the equivalent currents and the absorbed power.
#include "mbem_internal.h"
#include "p2_device.h"

namespace mbem {

constexpr int kW2 = 64;

__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = kW2 / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kW2);
    return v;
}

__device__ inline cx<double> cexpi(double ph) {
    double s, c;
    sincos(ph, &s, &c);
    return {c, s};
}

// Basis tangent of local node kk, component bb, at point i of the 7-point
// table: the interpolated frame (frame 0) or the projected nodal tangent.
__device__ inline dvec3 basis_at(int frame, const double *__restrict__ qp, int64_t nq, int64_t i,
                                 const double *__restrict__ frames, int64_t node, int bb) {
    if (frame == 0) {
        const int c = bb ? QT2 : QT1;
        return {qp[c * nq + i], qp[(c + 1) * nq + i], qp[(c + 2) * nq + i]};
    }
    const dvec3 n = {qp[QN * nq + i], qp[(QN + 1) * nq + i], qp[(QN + 2) * nq + i]};
    return project_tangent(nodal_tangent(frames, node, bb), n);
}

// One thread per (quadrature point, right-hand side):
//   b_E[2i+a] += -eps_a W N_i s_a.E,  b_H[2i+a] += mu_a W N_i s_a.H
// with s_a the rotated test vector of node i (frame 0: of the point).
__global__ void k_rhs(int64_t nt, int64_t n2, int nrhs, const double *__restrict__ qp,
                      const int32_t *__restrict__ tri, const double *__restrict__ frames, int frame,
                      const double *__restrict__ khat, const double2 *__restrict__ pol, double ka,
                      double2 *__restrict__ b) {
    const int64_t nq = nt * kQP;
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nq * nrhs) return;
    const int64_t i = id % nq;
    const int r = (int)(id / nq);
    const int64_t e = i / kQP;
    const int q = (int)(i % kQP);
    const dvec3 x = {qp[QX * nq + i], qp[(QX + 1) * nq + i], qp[(QX + 2) * nq + i]};
    const dvec3 s0[2] = {{qp[QS1 * nq + i], qp[(QS1 + 1) * nq + i], qp[(QS1 + 2) * nq + i]},
                         {qp[QS2 * nq + i], qp[(QS2 + 1) * nq + i], qp[(QS2 + 2) * nq + i]}};
    const dvec3 n = {qp[QN * nq + i], qp[(QN + 1) * nq + i], qp[(QN + 2) * nq + i]};
    const double W = qp[QW * nq + i];
    const dvec3 k = {khat[3 * r], khat[3 * r + 1], khat[3 * r + 2]};
    const cx<double> ph = cexpi(ka * dot(k, x));
    const cx<double> E[3] = {ph * cx<double>{pol[3 * r].x, pol[3 * r].y},
                             ph * cx<double>{pol[3 * r + 1].x, pol[3 * r + 1].y},
                             ph * cx<double>{pol[3 * r + 2].x, pol[3 * r + 2].y}};
    // H = khat x E
    const cx<double> H[3] = {k.y * E[2] - k.z * E[1], k.z * E[0] - k.x * E[2], k.x * E[1] - k.y * E[0]};
    double xi, eta, w, N[6], d1[6], d2[6];
    rule7(q, xi, eta, w);
    p2_shape(xi, eta, N, d1, d2);
    double2 *bc = b + (int64_t)r * 2 * n2;
    for (int a = 0; a < 2; ++a) {
        for (int kk = 0; kk < 6; ++kk) {
            const int64_t node = tri[6 * e + kk];
            const dvec3 s = frame == 0 ? s0[a] : cross(nodal_tangent(frames, node, a), n);
            const cx<double> sE = s.x * E[0] + s.y * E[1] + s.z * E[2];
            const cx<double> sH = s.x * H[0] + s.y * H[1] + s.z * H[2];
            const int64_t row = 2 * node + a;
            const double f = W * N[kk];
            unsafeAtomicAdd(&bc[row].x, -f * sE.re);
            unsafeAtomicAdd(&bc[row].y, -f * sE.im);
            unsafeAtomicAdd(&bc[n2 + row].x, f * sH.re);
            unsafeAtomicAdd(&bc[n2 + row].y, f * sH.im);
        }
    }
}

int rhs_run(const mbem_mesh *m, const mbem_params *p, const double *khat, const double2 *pol,
            int nrhs, double2 *b, hipStream_t s) {
    const int64_t n2 = 2 * m->nn;
    MBEM_HIP(hipMemsetAsync(b, 0, sizeof(double2) * 2 * n2 * nrhs, s));
    const int64_t n = m->nt * kQP * nrhs;
    hipLaunchKernelGGL(k_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, m->nt, n2, nrhs,
                       m->d_qp, m->d_tri, m->d_frames, p->frame, khat, pol, p->k0, b);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

// Surface currents W j, W j_m at every quadrature point of one solution:
// cur[i][0..5] = W j (3 complex), cur[i][6..11] = W j_m.
__global__ void k_currents(int64_t nt, int64_t n2, const double *__restrict__ qp,
                           const int32_t *__restrict__ tri, const double *__restrict__ frames, int frame,
                           const double2 *__restrict__ x, double *__restrict__ cur) {
    const int64_t nq = nt * kQP;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const int64_t e = i / kQP;
    const int q = (int)(i % kQP);
    const double W = qp[QW * nq + i];
    double xi, eta, w, N[6], d1[6], d2[6];
    rule7(q, xi, eta, w);
    p2_shape(xi, eta, N, d1, d2);
    cx<double> J[3] = {{0, 0}, {0, 0}, {0, 0}}, Jm[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int kk = 0; kk < 6; ++kk) {
        const int64_t node = tri[6 * e + kk];
        for (int bb = 0; bb < 2; ++bb) {
            const double2 cj = x[2 * node + bb], cm = x[n2 + 2 * node + bb];
            const dvec3 t = basis_at(frame, qp, nq, i, frames, node, bb);
            const double c[3] = {t.x, t.y, t.z};
            for (int d = 0; d < 3; ++d) {
                const double f = W * N[kk] * c[d];
                J[d] = J[d] + cx<double>{f * cj.x, f * cj.y};
                Jm[d] = Jm[d] + cx<double>{f * cm.x, f * cm.y};
            }
        }
    }
    double *o = cur + 12 * i;
    for (int d = 0; d < 3; ++d) {
        o[2 * d] = J[d].re; o[2 * d + 1] = J[d].im;
        o[6 + 2 * d] = Jm[d].re; o[6 + 2 * d + 1] = Jm[d].im;
    }
}

// F(r) = (i k / 4 pi) r x sum_q e^{-i k r.y_q} (W j x r - W j_m); one
// workgroup per direction.
__global__ __launch_bounds__(256) void k_farfield(int64_t nq, const double *__restrict__ qp,
                                                  const double *__restrict__ cur,
                                                  const double *__restrict__ rhat, double ka,
                                                  double2 *__restrict__ F) {
    __shared__ double s[4][6];
    const int64_t d = blockIdx.x;
    const dvec3 r = {rhat[3 * d], rhat[3 * d + 1], rhat[3 * d + 2]};
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = threadIdx.x; i < nq; i += blockDim.x) {
        const dvec3 y = {qp[QX * nq + i], qp[(QX + 1) * nq + i], qp[(QX + 2) * nq + i]};
        const cx<double> ph = cexpi(-ka * dot(r, y));
        const double *c = cur + 12 * i;
        const cx<double> J[3] = {{c[0], c[1]}, {c[2], c[3]}, {c[4], c[5]}};
        const cx<double> Jm[3] = {{c[6], c[7]}, {c[8], c[9]}, {c[10], c[11]}};
        // j x r - j_m
        const cx<double> v[3] = {r.z * J[1] - r.y * J[2] - Jm[0], r.x * J[2] - r.z * J[0] - Jm[1],
                                 r.y * J[0] - r.x * J[1] - Jm[2]};
        for (int k = 0; k < 3; ++k) {
            const cx<double> t = ph * v[k];
            acc[2 * k] += t.re;
            acc[2 * k + 1] += t.im;
        }
    }
    for (int k = 0; k < 6; ++k) acc[k] = wsum(acc[k]);
    if (threadIdx.x % kW2 == 0)
        for (int k = 0; k < 6; ++k) s[threadIdx.x / kW2][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        cx<double> a[3];
        for (int k = 0; k < 3; ++k)
            a[k] = {s[0][2 * k] + s[1][2 * k] + s[2][2 * k] + s[3][2 * k],
                    s[0][2 * k + 1] + s[1][2 * k + 1] + s[2][2 * k + 1] + s[3][2 * k + 1]};
        // r x a, times i k / (4 pi)
        const cx<double> c[3] = {r.y * a[2] - r.z * a[1], r.z * a[0] - r.x * a[2], r.x * a[1] - r.y * a[0]};
        const double f = ka * 0.079577471545947667884;
        for (int k = 0; k < 3; ++k) F[3 * d + k] = {-f * c[k].im, f * c[k].re};
    }
}

int farfield_run(const mbem_mesh *m, const mbem_params *p, const double2 *x, int nrhs,
                 const double *rhat, int64_t ndir, double2 *F, hipStream_t s) {
    const int64_t nq = m->nt * kQP, n2 = 2 * m->nn;
    double *cur = nullptr;
    MBEM_HIP(hipMallocAsync((void **)&cur, sizeof(double) * 12 * nq, s));
    for (int r = 0; r < nrhs; ++r) {
        hipLaunchKernelGGL(k_currents, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, m->nt, n2,
                           m->d_qp, m->d_tri, m->d_frames, p->frame, x + (int64_t)r * 2 * n2, cur);
        MBEM_HIP(hipGetLastError());
        if (ndir > 0) {
            hipLaunchKernelGGL(k_farfield, dim3((unsigned)ndir), dim3(256), 0, s, nq, m->d_qp, cur, rhat,
                               p->k0, F + (int64_t)r * ndir * 3);
            MBEM_HIP(hipGetLastError());
        }
    }
    MBEM_HIP(hipFreeAsync(cur, s));
    return MBEM_OK;
}

// sum_q Re n.(W j_m x conj(j)) with j from the unweighted coefficients.
__global__ __launch_bounds__(256) void k_absorbed(int64_t nt, int64_t n2, const double *__restrict__ qp,
                                                  const int32_t *__restrict__ tri,
                                                  const double *__restrict__ frames, int frame,
                                                  const double2 *__restrict__ x, double *out) {
    const int64_t nq = nt * kQP;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < nq) {
        const int64_t e = i / kQP;
        const int q = (int)(i % kQP);
        const dvec3 n = {qp[QN * nq + i], qp[(QN + 1) * nq + i], qp[(QN + 2) * nq + i]};
        double xi, eta, w, N[6], d1[6], d2[6];
        rule7(q, xi, eta, w);
        p2_shape(xi, eta, N, d1, d2);
        cx<double> J[3] = {{0, 0}, {0, 0}, {0, 0}}, Jm[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int kk = 0; kk < 6; ++kk) {
            const int64_t node = tri[6 * e + kk];
            for (int bb = 0; bb < 2; ++bb) {
                const double2 cj = x[2 * node + bb], cm = x[n2 + 2 * node + bb];
                const dvec3 t = basis_at(frame, qp, nq, i, frames, node, bb);
                const double c[3] = {t.x, t.y, t.z};
                for (int d = 0; d < 3; ++d) {
                    J[d] = J[d] + cx<double>{N[kk] * c[d] * cj.x, N[kk] * c[d] * cj.y};
                    Jm[d] = Jm[d] + cx<double>{N[kk] * c[d] * cm.x, N[kk] * c[d] * cm.y};
                }
            }
        }
        // j_m x conj(j)
        const cx<double> Jc[3] = {{J[0].re, -J[0].im}, {J[1].re, -J[1].im}, {J[2].re, -J[2].im}};
        const cx<double> c[3] = {Jm[1] * Jc[2] - Jm[2] * Jc[1], Jm[2] * Jc[0] - Jm[0] * Jc[2],
                                 Jm[0] * Jc[1] - Jm[1] * Jc[0]};
        v = qp[QW * nq + i] * (n.x * c[0].re + n.y * c[1].re + n.z * c[2].re);
    }
    v = wsum(v);
    if (threadIdx.x % kW2 == 0) unsafeAtomicAdd(out, v);
}

int absorbed_run(const mbem_mesh *m, const mbem_params *p, const double2 *x, double *out_dev, hipStream_t s) {
    const int64_t nq = m->nt * kQP;
    MBEM_HIP(hipMemsetAsync(out_dev, 0, sizeof(double), s));
    hipLaunchKernelGGL(k_absorbed, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, m->nt, 2 * m->nn,
                       m->d_qp, m->d_tri, m->d_frames, p->frame, x, out_dev);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

// sum_d w_d |F_d|^2 over ndir directions (3 complex components each)
__global__ __launch_bounds__(256) void k_wnorm(int64_t ndir, const double2 *F, const double *w, double *out) {
    const int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double v = 0;
    if (d < ndir)
        for (int k = 0; k < 3; ++k) v += w[d] * (F[3 * d + k].x * F[3 * d + k].x + F[3 * d + k].y * F[3 * d + k].y);
    v = wsum(v);
    if (threadIdx.x % kW2 == 0) unsafeAtomicAdd(out, v);
}

int weighted_norm_run(int64_t ndir, const double2 *F, const double *w, double *out, hipStream_t s) {
    MBEM_HIP(hipMemsetAsync(out, 0, sizeof(double), s));
    hipLaunchKernelGGL(k_wnorm, dim3((unsigned)((ndir + 255) / 256)), dim3(256), 0, s, ndir, F, w, out);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

}  // namespace mbem
