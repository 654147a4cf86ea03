// Device helpers: small vectors, complex arithmetic, the P2 isoparametric
// element with its continuous frame (Sec. 3), and the kernel-difference
// evaluator (Sec. 2.3, 4.1, 4.2) in FP64 or FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mbem {

// ------------------------------------------------------------ vectors --
template <typename T>
struct vec3 {
    T x, y, z;
};
using dvec3 = vec3<double>;

template <typename T>
__device__ __host__ inline vec3<T> operator+(vec3<T> a, vec3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__device__ __host__ inline vec3<T> operator-(vec3<T> a, vec3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ __host__ inline vec3<T> operator*(T s, vec3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T>
__device__ __host__ inline vec3<T> operator-(vec3<T> a) { return {-a.x, -a.y, -a.z}; }
template <typename T>
__device__ __host__ inline T dot(vec3<T> a, vec3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __host__ inline vec3<T> cross(vec3<T> a, vec3<T> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline dvec3 load3(const double *p, int64_t i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }

// ------------------------------------------------------------ complex --
template <typename T>
struct cx {
    T re, im;
};
template <typename T>
__device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }

// -------------------------------------------------- 7-point rule (Radon) --
// Degree-5 rule on {xi, eta >= 0, xi + eta <= 1}, weights summing to 1/2:
// centroid, and two orbits of three points at distances a, b from the edges.
__device__ inline void rule7(int q, double &xi, double &eta, double &w) {
    const double r15 = sqrt(15.0);
    const double a = (6.0 - r15) / 21.0, b = (6.0 + r15) / 21.0;
    if (q == 0) { xi = 1.0 / 3.0; eta = 1.0 / 3.0; w = 9.0 / 80.0; return; }
    const double s = (q <= 3) ? a : b;
    w = (q <= 3) ? (155.0 - r15) / 2400.0 : (155.0 + r15) / 2400.0;
    const int r = (q - 1) % 3;
    xi = (r == 1) ? 1.0 - 2.0 * s : s;
    eta = (r == 2) ? 1.0 - 2.0 * s : s;
}

// The 12-point degree-6 symmetric rule (the regular rule of the paper's own
// scheme): two three-point orbits (a, a, 1 - 2a) and one six-point orbit
// (b, c, 1 - b - c) in barycentric coordinates (L0, L1, L2) = (1 - xi - eta,
// xi, eta); its seven parameters solve the moment equations of the
// S3-invariant polynomials of degree <= 6.  Weights sum to 1/2.
__host__ __device__ constexpr double r12_bary(int q, int k) {
    if (q < 6) {
        const double a = q < 3 ? 0.06308901449150309 : 0.24928674517091215;
        return k == q % 3 ? 1.0 - 2.0 * a : a;
    }
    const double v[3] = {0.053145049844817806, 0.3103524510337839,
                         1.0 - 0.053145049844817806 - 0.3103524510337839};
    // orbit point m: L[perm(m)[d]] = v[d] for the six permutations
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int m = q - 6;
    for (int d = 0; d < 3; ++d)
        if (perm[m][d] == k) return v[d];
    return 0.0;
}
__host__ __device__ constexpr double r12_weight(int q) {
    return 0.5 * (q < 3 ? 0.05084490637020728 : (q < 6 ? 0.11678627572637695 : 0.08285107561837454));
}
__device__ inline void rule12(int q, double &xi, double &eta, double &w) {
    xi = r12_bary(q, 1);
    eta = r12_bary(q, 2);
    w = r12_weight(q);
}

// ------------------------------------------------------- P2 element ---
// Shape functions in barycentric form: vertex l(2l-1), mid-edge 4 l l'.
__device__ inline void p2_shape(double xi, double eta, double N[6], double Nxi[6],
                                double Neta[6]) {
    const double L0 = 1.0 - xi - eta, L1 = xi, L2 = eta;
    N[0] = L0 * (2.0 * L0 - 1.0);
    N[1] = L1 * (2.0 * L1 - 1.0);
    N[2] = L2 * (2.0 * L2 - 1.0);
    N[3] = 4.0 * L0 * L1;
    N[4] = 4.0 * L1 * L2;
    N[5] = 4.0 * L2 * L0;
    // chain rule with dL/dxi = (-1, 1, 0), dL/deta = (-1, 0, 1)
    const double g0 = 4.0 * L0 - 1.0, g1 = 4.0 * L1 - 1.0, g2 = 4.0 * L2 - 1.0;
    Nxi[0] = -g0; Nxi[1] = g1;  Nxi[2] = 0.0;
    Nxi[3] = 4.0 * (L0 - L1); Nxi[4] = 4.0 * L2; Nxi[5] = -4.0 * L2;
    Neta[0] = -g0; Neta[1] = 0.0; Neta[2] = g2;
    Neta[3] = -4.0 * L1; Neta[4] = 4.0 * L1; Neta[5] = 4.0 * (L0 - L2);
}

struct P2Point {
    dvec3 x, n, t1, t2, s1, s2;
    double J;
    double N[6];
};

// Position, exact unit normal a1 x a2 / |a1 x a2|, and the continuous
// frame: nodal tangents interpolated with the shape functions, projected
// on the tangent plane and Gram-Schmidt orthonormalised (Sec. 3.3);
// s_alpha = t_alpha x n (Sec. 4.1).
__device__ inline void p2_point(const double *__restrict__ xyz,
                                const double *__restrict__ frames,
                                const int32_t *t, double xi, double eta,
                                P2Point &P) {
    double Nxi[6], Neta[6];
    p2_shape(xi, eta, P.N, Nxi, Neta);
    dvec3 x = {0, 0, 0}, a1 = {0, 0, 0}, a2 = {0, 0, 0};
    dvec3 u1 = {0, 0, 0}, u2 = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int64_t v = t[k];
        const dvec3 X = load3(xyz, v);
        x = x + P.N[k] * X;
        a1 = a1 + Nxi[k] * X;
        a2 = a2 + Neta[k] * X;
        const double *f = frames + 9 * v;
        u1 = u1 + P.N[k] * dvec3{f[3], f[4], f[5]};
        u2 = u2 + P.N[k] * dvec3{f[6], f[7], f[8]};
    }
    const dvec3 c = cross(a1, a2);
    P.J = sqrt(dot(c, c));
    const dvec3 n = (1.0 / P.J) * c;
    P.x = x;
    P.n = n;
    u1 = u1 - dot(n, u1) * n;
    u2 = u2 - dot(n, u2) * n;
    P.t1 = (1.0 / sqrt(dot(u1, u1))) * u1;
    u2 = u2 - dot(P.t1, u2) * P.t1;
    P.t2 = (1.0 / sqrt(dot(u2, u2))) * u2;
    P.s1 = cross(P.t1, n);
    P.s2 = cross(P.t2, n);
}

// Node-attached tangents (frame 1): the basis function of node v, component
// b, is N_v(y) P(y) t_b,v with t_b,v the node's own triad tangent and
// P(y) = I - n n^T the tangent-plane projector at y; its rotated test vector
// is P t_b,v x n = t_b,v x n.  Frame 0 uses the interpolated frame t_b(y) of
// p2_point for every node.
__device__ inline dvec3 nodal_tangent(const double *__restrict__ frames, int64_t v, int b) {
    const double *f = frames + 9 * v + 3 + 3 * b;
    return {f[0], f[1], f[2]};
}
__device__ inline dvec3 project_tangent(dvec3 t, dvec3 n) { return t - dot(t, n) * n; }

// ------------------------------------------------- kernel differences --
constexpr int kSeriesTerms = 16;   // Taylor terms n = 0..16
constexpr double kSeriesRho = 0.5; // series below max|k| R = 1/2

// Material constants and the frequency-dependent Taylor coefficients,
// precomputed on the host once per fill (Sec. 6.1).  With
// c_n(k) = (i k)^n / n!:
//   cD[n] = k_a^2 c_n(k_a) - k_i^2 c_n(k_i)          D0 = sum cD R^n / (4 pi R)
//   cF[n] = (n-1)(n-3)(c_n(k_a) - c_n(k_i))           df = sum cF R^n / (4 pi R^3)
//   cG[n] = -(n-1)(c_n(k_a) - c_n(k_i))               dg = sum cG R^n / (4 pi R^3)
//   cE[n] = (n-1)(eps_a c_n(k_a) - eps_i c_n(k_i))    G_eps = sum cE R^n / (4 pi R^2)
//   cM[n] = (n-1)(mu_a c_n(k_a) - mu_i c_n(k_i))      G_mu  = sum cM R^n / (4 pi R^2)
struct KernelConst {
    double ka_re, ka_im, ki_re, ki_im;
    double eps_a_re, eps_a_im, eps_i_re, eps_i_im;
    double mu_a_re, mu_a_im, mu_i_re, mu_i_im;
    double kmax;
    double cD[2 * (kSeriesTerms + 1)], cF[2 * (kSeriesTerms + 1)],
        cG[2 * (kSeriesTerms + 1)], cE[2 * (kSeriesTerms + 1)],
        cM[2 * (kSeriesTerms + 1)];
};

template <typename T>
struct KScal {
    cx<T> D0, df, dg, Ge, Gm;
};

template <typename T>
__device__ __forceinline__ cx<T> horner(const double *c, T R) {
    cx<T> s = {(T)c[2 * kSeriesTerms], (T)c[2 * kSeriesTerms + 1]};
#pragma unroll
    for (int n = kSeriesTerms - 1; n >= 0; --n) s = cx<T>{s.re * R + (T)c[2 * n], s.im * R + (T)c[2 * n + 1]};
    return s;
}

// sin and cos of the phases k R of the kernels (|x| far below 2^20).
// Cody and Waite's reduction x = n pi/2 + r, |r| <= pi/4, with pi/2 split
// into three floating-point parts (each product n P_i is exact inside the
// fused multiply-add), then the Taylor series of sin r and cos r, truncated
// where the next term is below the unit roundoff on |r| <= pi/4 (FP64:
// r^15 and r^16; FP32: r^9 and r^10), and the quadrant n mod 4.
template <typename T>
__device__ __forceinline__ void quadrant(int q, T sr, T cr, T *s, T *c) {
    const T ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
    *s = (q & 2) ? -ss : ss;
    *c = ((q + 1) & 2) ? -cc : cc;
}
__device__ __forceinline__ void sincos_t(double x, double *s, double *c) {
    const double n = rint(x * 0.63661977236758134308);
    double r = fma(-n, 0x1.921fb54442d18p+0, x);
    r = fma(-n, 0x1.1a62633145c07p-54, r);
    r = fma(-n, -0x1.f1976b7ed8fbcp-110, r);
    const double u = r * r;
    double ps = -1.0 / 1307674368000.0;                 // -1/15!
    ps = fma(ps, u, 1.0 / 6227020800.0);                // 1/13!
    ps = fma(ps, u, -1.0 / 39916800.0);                 // -1/11!
    ps = fma(ps, u, 1.0 / 362880.0);
    ps = fma(ps, u, -1.0 / 5040.0);
    ps = fma(ps, u, 1.0 / 120.0);
    ps = fma(ps, u, -1.0 / 6.0);
    const double sr = fma(r * u, ps, r);
    double pc = 1.0 / 20922789888000.0;                 // 1/16!
    pc = fma(pc, u, -1.0 / 87178291200.0);              // -1/14!
    pc = fma(pc, u, 1.0 / 479001600.0);                 // 1/12!
    pc = fma(pc, u, -1.0 / 3628800.0);
    pc = fma(pc, u, 1.0 / 40320.0);
    pc = fma(pc, u, -1.0 / 720.0);
    pc = fma(pc, u, 1.0 / 24.0);
    pc = fma(pc, u, -0.5);
    const double cr = fma(u, pc, 1.0);
    quadrant((int)n, sr, cr, s, c);
}
__device__ __forceinline__ void sincos_t(float x, float *s, float *c) {
    const float n = rintf(x * 0.636619772f);
    float r = fmaf(-n, 0x1.921fb6p+0f, x);
    r = fmaf(-n, -0x1.777a5cp-25f, r);
    r = fmaf(-n, -0x1.ee59dap-50f, r);
    const float u = r * r;
    float ps = 1.0f / 362880.0f;
    ps = fmaf(ps, u, -1.0f / 5040.0f);
    ps = fmaf(ps, u, 1.0f / 120.0f);
    ps = fmaf(ps, u, -1.0f / 6.0f);
    const float sr = fmaf(r * u, ps, r);
    float pc = -1.0f / 3628800.0f;
    pc = fmaf(pc, u, 1.0f / 40320.0f);
    pc = fmaf(pc, u, -1.0f / 720.0f);
    pc = fmaf(pc, u, 1.0f / 24.0f);
    pc = fmaf(pc, u, -0.5f);
    const float cr = fmaf(u, pc, 1.0f);
    quadrant((int)n, sr, cr, s, c);
}
__device__ inline double exp_t(double x) { return exp(x); }
__device__ inline float exp_t(float x) { return expf(x); }

// Scalar parts of D0 = k_a^2 phi_a - k_i^2 phi_i, H_diff = df RR^T - dg I
// (eq. Hdiff_exact) and grad Phi_chi = G_chi Rhat at distance R.
template <typename T>
__device__ __forceinline__ KScal<T> kernel_scalars_closed(const KernelConst &K, T R);

template <typename T>
__device__ __forceinline__ KScal<T> kernel_scalars(const KernelConst &K, T R) {
    const T inv4pi = (T)0.079577471545947667884;   // 1 / (4 pi)
    KScal<T> o;
    if ((T)K.kmax * R < (T)kSeriesRho) {
        const T r1 = inv4pi / R, r2 = r1 / R, r3 = r2 / R;
        o.D0 = r1 * horner<T>(K.cD, R);
        o.df = r3 * horner<T>(K.cF, R);
        o.dg = r3 * horner<T>(K.cG, R);
        o.Ge = r2 * horner<T>(K.cE, R);
        o.Gm = r2 * horner<T>(K.cM, R);
        return o;
    }
    return kernel_scalars_closed<T>(K, R);
}

// The closed forms alone (every R > 0).
template <typename T>
__device__ __forceinline__ KScal<T> kernel_scalars_closed(const KernelConst &K, T R) {
    const T inv4pi = (T)0.079577471545947667884;
    KScal<T> o;
    const T r1 = inv4pi / R, r3 = r1 / (R * R);
    cx<T> k[2] = {{(T)K.ka_re, (T)K.ka_im}, {(T)K.ki_re, (T)K.ki_im}};
    cx<T> phi[2], f[2], g[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const cx<T> ikR = {-k[s].im * R, k[s].re * R};
        T sn, cs;
        sincos_t(k[s].re * R, &sn, &cs);
        const T am = k[s].im == (T)0 ? (T)1 : exp_t(-k[s].im * R);
        const cx<T> e = {am * cs, am * sn};
        const cx<T> k2R2 = (R * R) * (k[s] * k[s]);
        phi[s] = r1 * e;
        f[s] = r3 * (e * cx<T>{(T)3 - (T)3 * ikR.re - k2R2.re, -(T)3 * ikR.im - k2R2.im});
        g[s] = r3 * (e * cx<T>{(T)1 - ikR.re, -ikR.im});
    }
    o.D0 = (k[0] * k[0]) * phi[0] - (k[1] * k[1]) * phi[1];
    o.df = f[0] - f[1];
    o.dg = g[0] - g[1];
    // phi'(R) = -R g(R)
    const cx<T> ea = {(T)K.eps_a_re, (T)K.eps_a_im}, ei = {(T)K.eps_i_re, (T)K.eps_i_im};
    const cx<T> ma = {(T)K.mu_a_re, (T)K.mu_a_im}, mi = {(T)K.mu_i_re, (T)K.mu_i_im};
    o.Ge = (-R) * (ea * g[0] - ei * g[1]);
    o.Gm = (-R) * (ma * g[0] - mi * g[1]);
    return o;
}

// Singular parts of the scalars (kappa^s of the paper's scheme, Sec. 4.1
// and 4.2): the terms of negative order in R of the expansions,
//   D0^s = (k_a^2 - k_i^2)/(4 pi R), df^s = dg^s = (k_a^2 - k_i^2)/(8 pi R),
//   G_chi^s = -(chi_a - chi_i)/(4 pi R^2).
__device__ __forceinline__ KScal<double> kernel_scalars_sing(const KernelConst &K, double R) {
    const double inv4pi = 0.079577471545947667884;
    const cx<double> ka = {K.ka_re, K.ka_im}, ki = {K.ki_re, K.ki_im};
    const cx<double> dk2 = ka * ka - ki * ki;
    const double r1 = inv4pi / R, r2 = r1 / R;
    KScal<double> o;
    o.D0 = r1 * dk2;
    o.df = (0.5 * r1) * dk2;
    o.dg = o.df;
    o.Ge = (-r2) * cx<double>{K.eps_a_re - K.eps_i_re, K.eps_a_im - K.eps_i_im};
    o.Gm = (-r2) * cx<double>{K.mu_a_re - K.mu_i_re, K.mu_a_im - K.mu_i_im};
    return o;
}

// Remainders kernel - kernel^s.  Below max|k| R = 1/2 (and at R = 0): the
// expansions without their singular terms, whose coefficients the host
// shifts into Kr so that only non-negative powers of R remain (D0 by one
// power, df and dg by three, G by two; truncated after n = 6); otherwise the
// closed forms minus the singular parts.
__device__ __forceinline__ KScal<double> kernel_scalars_rem(const KernelConst &K, const KernelConst &Kr,
                                                           double R) {
    const double inv4pi = 0.079577471545947667884;
    KScal<double> o;
    if (R > 0.0 && K.kmax * R >= kSeriesRho) {
        const KScal<double> c = kernel_scalars_closed<double>(K, R), s = kernel_scalars_sing(K, R);
        o.D0 = c.D0 - s.D0;
        o.df = c.df - s.df;
        o.dg = c.dg - s.dg;
        o.Ge = c.Ge - s.Ge;
        o.Gm = c.Gm - s.Gm;
        return o;
    }
    o.D0 = inv4pi * horner<double>(Kr.cD, R);
    o.df = inv4pi * horner<double>(Kr.cF, R);
    o.dg = inv4pi * horner<double>(Kr.cG, R);
    o.Ge = inv4pi * horner<double>(Kr.cE, R);
    o.Gm = inv4pi * horner<double>(Kr.cM, R);
    return o;
}

// Derivatives of the same scalars with respect to the interior permittivity
// eps_i at fixed k_0 and mu_i (k_i = k_0 sqrt(eps_i mu_i), dk_i/deps_i =
// k_i / (2 eps_i)), for the adjoint gradient.  With e = e^{i k_i R}:
//   d phi_i/dk = i R phi_i,  d f_i/dk = e k (1 - i k R) / (4 pi R),
//   d g_i/dk = e k / (4 pi R);
//   dD0 = -k phi_i (2 + i k R) dk,  ddf = -d f_i/dk dk,  ddg = -d g_i/dk dk,
//   dG_eps = R (g_i + eps_i d g_i/dk dk),  dG_mu = R mu_i d g_i/dk dk.
// Below max|k| R = 1/2 the host supplies the term-by-term derivative of the
// Taylor coefficients instead (same Horner evaluation as kernel_scalars).
// KernelConst.ka_re/ka_im hold dk_i/deps_i in this mode.
__device__ __forceinline__ KScal<double> kernel_scalars_deps(const KernelConst &K, double R) {
    const double inv4pi = 0.079577471545947667884;
    KScal<double> o;
    if (K.kmax * R < kSeriesRho) {
        const double r1 = inv4pi / R, r2 = r1 / R, r3 = r2 / R;
        o.D0 = r1 * horner<double>(K.cD, R);
        o.df = r3 * horner<double>(K.cF, R);
        o.dg = r3 * horner<double>(K.cG, R);
        o.Ge = r2 * horner<double>(K.cE, R);
        o.Gm = r2 * horner<double>(K.cM, R);
        return o;
    }
    const double r1 = inv4pi / R;
    const cx<double> k = {K.ki_re, K.ki_im}, dk = {K.ka_re, K.ka_im};
    double sn, cs;
    sincos_t(k.re * R, &sn, &cs);
    const double am = exp(-k.im * R);
    const cx<double> e = {am * cs, am * sn};
    const cx<double> phi = r1 * e;
    const cx<double> ikR = {-k.im * R, k.re * R};
    const cx<double> ek = r1 * (e * k);                       // e k / (4 pi R)
    const cx<double> dfk = ek * cx<double>{1.0 - ikR.re, -ikR.im};
    const cx<double> g = (r1 / (R * R)) * (e * cx<double>{1.0 - ikR.re, -ikR.im});
    o.D0 = ((-1.0) * (k * phi) * cx<double>{2.0 + ikR.re, ikR.im}) * dk;
    o.df = (-1.0) * (dfk * dk);
    o.dg = (-1.0) * (ek * dk);
    const cx<double> ei = {K.eps_i_re, K.eps_i_im}, mi = {K.mu_i_re, K.mu_i_im};
    o.Ge = R * (g + ei * (ek * dk));
    o.Gm = R * (mi * (ek * dk));
    return o;
}

}  // namespace mbem
