// Geometry tables on the device (Sec. 3): metric-weighted nodal normals and
// tangent triads, and the continuous orthonormal frame at the regular
// quadrature points of every curved P2 triangle.
#include "mbem_internal.h"
#include "p2_device.h"

namespace mbem {

// Nodal normal of Sec. 3.1: sum over incident triangles of
// U = (a1 x a2) / (|a1|^2 |a2|^2) with a1, a2 the covariant tangents along
// the edges leaving the node (vertex nodes), or along the edge and into
// the triangle at the edge midpoint (mid-edge nodes); then the tangent
// triad of Sec. 3.2 from the adaptive reference axis.
__global__ void k_nodal_frames(int64_t nn, const double *__restrict__ xyz,
                               const int32_t *__restrict__ tri,
                               const int32_t *__restrict__ inc_ptr,
                               const int32_t *__restrict__ inc,
                               double *__restrict__ frames) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= nn) return;
    dvec3 acc = {0.0, 0.0, 0.0};
    for (int32_t s = inc_ptr[v]; s < inc_ptr[v + 1]; ++s) {
        int32_t e = inc[s] >> 3, k = inc[s] & 7;
        const int32_t *t = tri + 6 * e;
        dvec3 a1, a2;
        if (k < 3) {
            // v is vertex k; next / previous vertices in the element's order
            int kn = (k + 1) % 3, kp = (k + 2) % 3;
            dvec3 X0 = load3(xyz, t[k]), Xn = load3(xyz, t[kn]), Xp = load3(xyz, t[kp]);
            dvec3 Mn = load3(xyz, t[3 + k]), Mp = load3(xyz, t[3 + kp]);
            a1 = -3.0 * X0 + 4.0 * Mn - Xn;    // d/dxi at the vertex
            a2 = -3.0 * X0 + 4.0 * Mp - Xp;    // d/deta at the vertex
        } else {
            // mid node of edge a -> a+1, evaluated at the edge midpoint
            int a = k - 3, b = (a + 1) % 3, c = (a + 2) % 3;
            dvec3 Xa = load3(xyz, t[a]), Xb = load3(xyz, t[b]), Xc = load3(xyz, t[c]);
            dvec3 Mab = load3(xyz, t[3 + a]), Mbc = load3(xyz, t[3 + b]), Mca = load3(xyz, t[3 + c]);
            a1 = Xb - Xa;
            a2 = 2.0 * (Mbc + Mca - Mab) - Xa - Xc;
        }
        dvec3 c = cross(a1, a2);
        acc = acc + (1.0 / (dot(a1, a1) * dot(a2, a2))) * c;
    }
    dvec3 n = (1.0 / sqrt(dot(acc, acc))) * acc;
    dvec3 ref = fabs(n.z) > 0.9 ? dvec3{1.0, 0.0, 0.0} : dvec3{0.0, 0.0, 1.0};
    dvec3 t1 = cross(ref, n);
    t1 = (1.0 / sqrt(dot(t1, t1))) * t1;
    dvec3 t2 = cross(n, t1);
    double *o = frames + 9 * v;
    o[0] = n.x;  o[1] = n.y;  o[2] = n.z;
    o[3] = t1.x; o[4] = t1.y; o[5] = t1.z;
    o[6] = t2.x; o[7] = t2.y; o[8] = t2.z;
}

// Quadrature-point table: position, weight * Jacobian, exact normal, the
// Gram-Schmidt frame t1, t2 (Sec. 3.3) and the rotated test vectors
// s_alpha = t_alpha x n (Sec. 4.1), at the 7 regular points of every
// triangle; written in FP64 and FP32 (structure of arrays).
template <int NQ>
__global__ void k_qp_table(int64_t nt, const double *__restrict__ xyz,
                           const int32_t *__restrict__ tri,
                           const double *__restrict__ frames,
                           double *__restrict__ qp, float *__restrict__ qp32) {
    int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t nq = nt * NQ;
    if (id >= nq) return;
    int64_t e = id / NQ;
    int q = (int)(id % NQ);
    double xi, eta, w;
    if constexpr (NQ == 12) rule12(q, xi, eta, w);
    else rule7(q, xi, eta, w);
    P2Point P;
    p2_point(xyz, frames, tri + 6 * e, xi, eta, P);
    double vals[kQPF] = {P.x.x, P.x.y, P.x.z, w * P.J,
                         P.n.x, P.n.y, P.n.z, P.t1.x, P.t1.y, P.t1.z,
                         P.t2.x, P.t2.y, P.t2.z, P.s1.x, P.s1.y, P.s1.z,
                         P.s2.x, P.s2.y, P.s2.z};
#pragma unroll
    for (int f = 0; f < kQPF; ++f) {
        qp[f * nq + id] = vals[f];
        qp32[f * nq + id] = (float)vals[f];
    }
}

// Centroid and bounding radius of every triangle (for the near/far split).
__global__ void k_elem_info(int64_t nt, const double *__restrict__ xyz,
                            const int32_t *__restrict__ tri,
                            double *__restrict__ info) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nt) return;
    const int32_t *t = tri + 6 * e;
    dvec3 c = (1.0 / 3.0) * (load3(xyz, t[0]) + load3(xyz, t[1]) + load3(xyz, t[2]));
    double r = 0.0;
    for (int k = 0; k < 6; ++k) {
        dvec3 d = load3(xyz, t[k]) - c;
        r = fmax(r, sqrt(dot(d, d)));
    }
    // a P2 edge bulges at most 1/8 of its control deviation; 1.25 covers it
    info[4 * e + 0] = c.x;
    info[4 * e + 1] = c.y;
    info[4 * e + 2] = c.z;
    info[4 * e + 3] = 1.25 * r;
}

int geom_build(const mbem_mesh *m, hipStream_t s, bool with12) {
    const int bs = 256;
    hipLaunchKernelGGL(k_nodal_frames, dim3((unsigned)((m->nn + bs - 1) / bs)), dim3(bs), 0, s,
                       m->nn, m->d_xyz, m->d_tri, m->d_inc_ptr, m->d_inc, m->d_frames);
    MBEM_HIP(hipGetLastError());
    int64_t nq = m->nt * kQP;
    hipLaunchKernelGGL(k_qp_table<kQP>, dim3((unsigned)((nq + bs - 1) / bs)), dim3(bs), 0, s,
                       m->nt, m->d_xyz, m->d_tri, m->d_frames, m->d_qp, m->d_qp32);
    MBEM_HIP(hipGetLastError());
    if (with12) {
        nq = m->nt * kQP12;
        hipLaunchKernelGGL(k_qp_table<kQP12>, dim3((unsigned)((nq + bs - 1) / bs)), dim3(bs), 0, s,
                           m->nt, m->d_xyz, m->d_tri, m->d_frames, m->d_qp12, m->d_qp12_32);
        MBEM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_elem_info, dim3((unsigned)((m->nt + bs - 1) / bs)), dim3(bs), 0, s,
                       m->nt, m->d_xyz, m->d_tri, m->d_elem);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

}  // namespace mbem
