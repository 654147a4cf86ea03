// Twelve weighted kernel values of the Galerkin fill at a test point
// (x, n, t_a, s_a) and a trial point (y, t_b) (eqs. kappa1_alphabeta,
// kappa2_alpha_beta):
//   kappa1_ab = (D0 - dg)(s_a.t_b) + df (s_a.R)(R.t_b)
//   kappa2_ab = G_chi [(t_a.t_b)(n.R) - (t_a.R)(n.t_b)],  R = (x - y)/|x - y|
// output order c = 4 op + 2 a + b, op: K1, K2^eps, K2^mu.  The scalars are
// those of the full kernels (kappa12), of their derivative in eps_i
// (kappa12<.., true>), of the singular parts kappa^s (kappa12_sing) or of
// the remainders kappa - kappa^s (kappa12_rem, which accepts x = y: the
// direction R is then taken as 0, so the terms along it drop out).
#pragma once

#include "p2_device.h"

namespace mbem {

template <typename T>
__device__ __forceinline__ void kappa_combine(const KScal<T> &s, vec3<T> Rh, vec3<T> n,
                                              const vec3<T> ta[2], const vec3<T> sa[2],
                                              const vec3<T> tb[2], T ww, cx<T> out[12]) {
    const cx<T> A = s.D0 - s.dg;
    const T nR = dot(n, Rh);
    T tRy[2], ntb[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) { tRy[b] = dot(tb[b], Rh); ntb[b] = dot(n, tb[b]); }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const T sR = dot(sa[a], Rh), tR = dot(ta[a], Rh);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const T st = dot(sa[a], tb[b]);
            const T g2 = dot(ta[a], tb[b]) * nR - tR * ntb[b];
            const cx<T> k1 = st * A + (sR * tRy[b]) * s.df;
            out[0 + 2 * a + b] = ww * k1;
            out[4 + 2 * a + b] = (ww * g2) * s.Ge;
            out[8 + 2 * a + b] = (ww * g2) * s.Gm;
        }
    }
}

template <typename T, bool DK = false>
__device__ __forceinline__ void kappa12(const KernelConst &K, vec3<T> x, vec3<T> n,
                                        const vec3<T> ta[2], const vec3<T> sa[2],
                                        vec3<T> y, const vec3<T> tb[2], T ww,
                                        cx<T> out[12]) {
    vec3<T> Rv = x - y;
    const T R = sqrt(dot(Rv, Rv));
    const vec3<T> Rh = ((T)1 / R) * Rv;
    KScal<T> s;
    if constexpr (DK) s = kernel_scalars_deps(K, R);
    else s = kernel_scalars<T>(K, R);
    kappa_combine<T>(s, Rh, n, ta, sa, tb, ww, out);
}

__device__ __forceinline__ void kappa12_sing(const KernelConst &K, dvec3 x, dvec3 n, const dvec3 ta[2],
                                             const dvec3 sa[2], dvec3 y, const dvec3 tb[2], double ww,
                                             cx<double> out[12]) {
    const dvec3 Rv = x - y;
    const double R = sqrt(dot(Rv, Rv));
    kappa_combine<double>(kernel_scalars_sing(K, R), (1.0 / R) * Rv, n, ta, sa, tb, ww, out);
}

__device__ __forceinline__ void kappa12_rem(const KernelConst &K, const KernelConst &Kr, dvec3 x, dvec3 n,
                                            const dvec3 ta[2], const dvec3 sa[2], dvec3 y,
                                            const dvec3 tb[2], double ww, cx<double> out[12]) {
    const dvec3 Rv = x - y;
    const double R = sqrt(dot(Rv, Rv));
    const dvec3 Rh = R > 0.0 ? (1.0 / R) * Rv : dvec3{0.0, 0.0, 0.0};
    kappa_combine<double>(kernel_scalars_rem(K, Kr, R), Rh, n, ta, sa, tb, ww, out);
}

}  // namespace mbem
