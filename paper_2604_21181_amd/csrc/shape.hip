// Shape gradient of sigma_ext by the adjoint method (extension of Sec. 6).
//
// With the solution x of Z x = b and lambda of Z^T lambda = g (g the
// far-field functional, sigma = (4 pi / k) Im g^T x), the derivative of
// sigma with respect to any geometric parameter is (4 pi / k) times that of
//     Phi = Im( g^T x + lambda^T b - lambda^T Z x )      (x, lambda frozen).
// Every term of Phi is a sum over quadrature points (right-hand side, far
// field, mass) or point pairs (dense blocks, Sec. 4) of an expression in
// the point's position, weight W = w J, normal n and frame t1, t2 (Sec. 3),
// with the current coefficients interpolated by the shape functions:
//   test point:  p_1 = L0 t1 + L1 t2,  p_2 = L2 t1 + L3 t2  (from lambda),
//                u_a = p_a x n  (= sum_alpha L s_alpha),
//   trial point: v_j = X0 t1 + X1 t2,  v_m = X2 t1 + X3 t2  (from x).
// The point-pair integrand of lambda^T Z x (eqs. kappa1/kappa2 summed over
// alpha, beta with these weights) is
//   F = (i/w) [A (u1.vj - u2.vm) + df ((u1.R)(R.vj) - (u2.R)(R.vm))]
//     + G_eps [(p1.vm)(n.R) - (p1.R)(n.vm)] + G_mu [(p2.vj)(n.R) - (p2.R)(n.vj)]
// with A = D0 - dg.  Reverse mode: adjoints of the point quantities are
// accumulated per quadrature point (regular rule) or per singular pair
// (Sauter-Schwab points), carried back through the P2 map and the
// Gram-Schmidt frame to node positions and nodal tangents, and through the
// nodal triads and metric-weighted normals to node positions.  The pair
// classes and the choice of reference vector are held fixed.
// Node-attached tangents (NODAL): the point vectors are p = m - (m.n) n with
// m = sum_k N_k sum_b c_kb t_b,k; their adjoints are kept as vectors and
// carried back through that projection to the normal and to the nodal
// tangents, which then go through the nodal triads as above.
#include <cmath>

#include "mbem_internal.h"
#include "p2_device.h"
#include "ssq_map.h"

namespace mbem {

using cxd = cx<double>;

// ------------------------------------------------------- complex vectors --
struct cv3 {
    cxd x, y, z;
};
__device__ inline cv3 operator+(cv3 a, cv3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline cv3 operator-(cv3 a, cv3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline cv3 operator*(cxd s, cv3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline cv3 operator*(cxd s, dvec3 a) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline cv3 operator*(double s, cv3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline cxd cdot(cv3 a, dvec3 b) { return b.x * a.x + b.y * a.y + b.z * a.z; }
__device__ inline cxd cdot(cv3 a, cv3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline cv3 ccross(dvec3 a, cv3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline cv3 ccross(cv3 a, dvec3 b) {
    return {b.z * a.y - b.y * a.z, b.x * a.z - b.z * a.x, b.y * a.x - b.x * a.y};
}
__device__ inline cv3 ccross(cv3 a, cv3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline dvec3 im3(cv3 a) { return {a.x.im, a.y.im, a.z.im}; }
__device__ inline cxd cscale(double s, cxd a) { return {s * a.re, s * a.im}; }

// ------------------------------ kernel differences and their R-derivatives --
struct KScalD {
    cxd A, Ap, df, dfp, Ge, Gep, Gm, Gmp;   // A = D0 - dg; p = d/dR
};

__device__ inline void horner_d(const double *c, double R, cxd &S, cxd &Sp) {
    S = {c[2 * kSeriesTerms], c[2 * kSeriesTerms + 1]};
    Sp = {0.0, 0.0};
    for (int n = kSeriesTerms - 1; n >= 0; --n) {
        Sp = cxd{Sp.re * R + S.re, Sp.im * R + S.im};
        S = cxd{S.re * R + c[2 * n], S.im * R + c[2 * n + 1]};
    }
}

// Same branches as kernel_scalars: Taylor series below max|k| R = 1/2,
// closed forms above, with
//   phi' = phi (i k - 1/R),  f' = e k^2 (1 - i k R) / (4 pi R^2) - 3 f / R,
//   g' = e k^2 / (4 pi R^2) - 3 g / R.
__device__ KScalD kernel_scalars_dr(const KernelConst &K, double R) {
    const double inv4pi = 0.079577471545947667884;
    KScalD o;
    const double r1 = inv4pi / R, r2 = r1 / R, r3 = r2 / R;
    if (K.kmax * R < kSeriesRho) {
        cxd SD, SDp, SF, SFp, SG, SGp, SE, SEp, SM, SMp;
        horner_d(K.cD, R, SD, SDp);
        horner_d(K.cF, R, SF, SFp);
        horner_d(K.cG, R, SG, SGp);
        horner_d(K.cE, R, SE, SEp);
        horner_d(K.cM, R, SM, SMp);
        const cxd D0 = r1 * SD, D0p = cscale(-1.0 / R, D0) + r1 * SDp;
        o.df = r3 * SF;
        o.dfp = cscale(-3.0 / R, o.df) + r3 * SFp;
        const cxd dg = r3 * SG, dgp = cscale(-3.0 / R, dg) + r3 * SGp;
        o.Ge = r2 * SE;
        o.Gep = cscale(-2.0 / R, o.Ge) + r2 * SEp;
        o.Gm = r2 * SM;
        o.Gmp = cscale(-2.0 / R, o.Gm) + r2 * SMp;
        o.A = D0 - dg;
        o.Ap = D0p - dgp;
        return o;
    }
    const cxd k[2] = {{K.ka_re, K.ka_im}, {K.ki_re, K.ki_im}};
    const cxd ch[2] = {{K.eps_a_re, K.eps_a_im}, {K.eps_i_re, K.eps_i_im}};
    const cxd cm[2] = {{K.mu_a_re, K.mu_a_im}, {K.mu_i_re, K.mu_i_im}};
    cxd D0 = {0, 0}, D0p = {0, 0}, dg = {0, 0}, dgp = {0, 0}, Eg = {0, 0}, Egp = {0, 0}, Mg = {0, 0}, Mgp = {0, 0};
    o.df = {0, 0};
    o.dfp = {0, 0};
    for (int s = 0; s < 2; ++s) {
        const double sg = s == 0 ? 1.0 : -1.0;
        double sn, cs;
        sincos_t(k[s].re * R, &sn, &cs);
        const double am = exp(-k[s].im * R);
        const cxd e = {am * cs, am * sn};
        const cxd ikR = {-k[s].im * R, k[s].re * R};
        const cxd k2 = k[s] * k[s];
        const cxd phi = r1 * e;
        const cxd phip = phi * cxd{-k[s].im - 1.0 / R, k[s].re};
        const cxd one_m = {1.0 - ikR.re, -ikR.im};
        const cxd f = r3 * (e * cxd{3.0 - 3.0 * ikR.re - (k2.re * R * R), -3.0 * ikR.im - k2.im * R * R});
        const cxd fp = r2 * (e * (k2 * one_m)) - cscale(3.0 / R, f);
        const cxd g = r3 * (e * one_m);
        const cxd gp = r2 * (e * k2) - cscale(3.0 / R, g);
        D0 = D0 + cscale(sg, k2 * phi);
        D0p = D0p + cscale(sg, k2 * phip);
        o.df = o.df + cscale(sg, f);
        o.dfp = o.dfp + cscale(sg, fp);
        dg = dg + cscale(sg, g);
        dgp = dgp + cscale(sg, gp);
        Eg = Eg + cscale(sg, ch[s] * g);
        Egp = Egp + cscale(sg, ch[s] * gp);
        Mg = Mg + cscale(sg, cm[s] * g);
        Mgp = Mgp + cscale(sg, cm[s] * gp);
    }
    // G_chi = -R (chi_a g_a - chi_i g_i)
    o.Ge = cscale(-R, Eg);
    o.Gep = cscale(-1.0, Eg) + cscale(-R, Egp);
    o.Gm = cscale(-R, Mg);
    o.Gmp = cscale(-1.0, Mg) + cscale(-R, Mgp);
    o.A = D0 - dg;
    o.Ap = D0p - dgp;
    return o;
}

// ------------------------------------------------- point-pair adjoint ---
struct TPt {
    dvec3 x, n, t1, t2;
    double W;
    cxd L[4];
};
struct SPt {
    dvec3 y, t1, t2;
    double W;
    cxd X[4];
};
// NODAL (node-attached tangents): the adjoints of the point's vectors p1, p2
// (test) and vj, vm (trial) themselves, complex and not yet reduced to Im,
// in place of those of the point frame.
struct TGrad {
    dvec3 x, n, t1, t2;
    double W;
    cv3 p1, p2;
};
struct SGrad {
    dvec3 y, t1, t2;
    double W;
    cv3 vj, vm;
};
__device__ inline cv3 czero3() { return {{0, 0}, {0, 0}, {0, 0}}; }
__device__ inline void zero(TGrad &g) {
    g.x = g.n = g.t1 = g.t2 = {0, 0, 0};
    g.W = 0.0;
    g.p1 = g.p2 = czero3();
}
__device__ inline void zero(SGrad &g) {
    g.y = g.t1 = g.t2 = {0, 0, 0};
    g.W = 0.0;
    g.vj = g.vm = czero3();
}

// Node-attached field of the coefficients c (node v, component b at
// c[2 v + b]) at a point with shape functions N: m = sum_k N_k sum_b c_kb t_b,k
// (the nodal tangents, not yet projected on the point's tangent plane).
__device__ inline cv3 nodal_field(const double *__restrict__ frames, const int32_t *t, const double N[6],
                                  const double2 *__restrict__ c) {
    cv3 m = czero3();
    for (int k = 0; k < 6; ++k) {
        const int64_t v = t[k];
        for (int b = 0; b < 2; ++b) {
            const double2 cf = c[2 * v + b];
            m = m + cxd{N[k] * cf.x, N[k] * cf.y} * nodal_tangent(frames, v, b);
        }
    }
    return m;
}

// Reverse of p = m - (m.n) n for the adjoint G of p (Im(G.p) is the
// quantity): adds the normal's part to bn and returns the adjoint of m.
__device__ inline cv3 proj_reverse(cv3 G, cv3 m, dvec3 n, dvec3 &bn) {
    const cxd mn = cdot(m, n), Gn = cdot(G, n);
    bn = bn - im3(Gn * m + mn * G);
    return G - Gn * n;
}

// Node-tangent adjoints of one point: Im(N_k sum_f c_f[kb] G_f) for the
// fields f built from the coefficient vectors c_f (nf of them).
template <int NF>
__device__ inline void nodal_tangent_adjoint(const int32_t *t, const double N[6], const double2 *const c[NF],
                                             const cv3 G[NF], dvec3 gT1[6], dvec3 gT2[6]) {
    for (int k = 0; k < 6; ++k) {
        const int64_t v = t[k];
        cv3 g[2] = {czero3(), czero3()};
        for (int f = 0; f < NF; ++f)
            for (int b = 0; b < 2; ++b) {
                const double2 cf = c[f][2 * v + b];
                g[b] = g[b] + cxd{N[k] * cf.x, N[k] * cf.y} * G[f];
            }
        gT1[k] = im3(g[0]);
        gT2[k] = im3(g[1]);
    }
}

// Adds d Im(c) / d(point quantities) for c = -wfac W_x W_y F.
template <bool WT, bool WS, bool NODAL = false>
__device__ void pair_adjoint(const KernelConst &K, cxd iw, const TPt &P, const SPt &Q, double wfac, TGrad &gt,
                             SGrad &gs) {
    const dvec3 Rv = P.x - Q.y;
    const double R = sqrt(dot(Rv, Rv));
    const dvec3 Rh = (1.0 / R) * Rv;
    const KScalD s = kernel_scalars_dr(K, R);
    const cv3 p1 = P.L[0] * P.t1 + P.L[1] * P.t2, p2 = P.L[2] * P.t1 + P.L[3] * P.t2;
    const cv3 u1 = ccross(p1, P.n), u2 = ccross(p2, P.n);
    const cv3 vj = Q.X[0] * Q.t1 + Q.X[1] * Q.t2, vm = Q.X[2] * Q.t1 + Q.X[3] * Q.t2;
    const double nR = dot(P.n, Rh);
    const cxd uv1 = cdot(u1, vj), uR1 = cdot(u1, Rh), Rv1 = cdot(vj, Rh);
    const cxd uv2 = cdot(u2, vm), uR2 = cdot(u2, Rh), Rv2 = cdot(vm, Rh);
    const cxd pv1 = cdot(p1, vm), pR1 = cdot(p1, Rh), nv1 = cdot(vm, P.n);
    const cxd pv2 = cdot(p2, vj), pR2 = cdot(p2, Rh), nv2 = cdot(vj, P.n);
    const cxd k1 = s.A * (uv1 - uv2) + s.df * (uR1 * Rv1 - uR2 * Rv2);
    const cxd e2 = pv1 * cxd{nR, 0.0} - pR1 * nv1, m2 = pv2 * cxd{nR, 0.0} - pR2 * nv2;
    const cxd F = iw * k1 + s.Ge * e2 + s.Gm * m2;
    // complex gradients of F
    const cv3 g_u1 = iw * (s.A * vj + (s.df * Rv1) * Rh);
    const cv3 g_u2 = cxd{-iw.re, -iw.im} * (s.A * vm + (s.df * Rv2) * Rh);
    const cv3 g_Rh = iw * (s.df * (uR1 * vj + Rv1 * u1 - uR2 * vm - Rv2 * u2)) +
                     s.Ge * (pv1 * P.n - nv1 * p1) + s.Gm * (pv2 * P.n - nv2 * p2);
    const cxd g_R = iw * (s.Ap * (uv1 - uv2) + s.dfp * (uR1 * Rv1 - uR2 * Rv2)) + s.Gep * e2 + s.Gmp * m2;
    const cxd gRh_Rh = cdot(g_Rh, Rh);
    const cv3 g_Rv = (1.0 / R) * (g_Rh - gRh_Rh * Rh) + g_R * Rh;
    const double c = -wfac * P.W * Q.W;
    if (WT) {
        const cv3 g_p1 = s.Ge * (cxd{nR, 0.0} * vm - nv1 * Rh) + ccross(P.n, g_u1);
        const cv3 g_p2 = s.Gm * (cxd{nR, 0.0} * vj - nv2 * Rh) + ccross(P.n, g_u2);
        const cv3 g_n = s.Ge * (pv1 * Rh - pR1 * vm) + s.Gm * (pv2 * Rh - pR2 * vj) + ccross(g_u1, p1) +
                        ccross(g_u2, p2);
        gt.x = gt.x + c * im3(g_Rv);
        gt.n = gt.n + c * im3(g_n);
        if constexpr (NODAL) {
            gt.p1 = gt.p1 + c * g_p1;
            gt.p2 = gt.p2 + c * g_p2;
        } else {
            const cv3 g_t1 = P.L[0] * g_p1 + P.L[2] * g_p2, g_t2 = P.L[1] * g_p1 + P.L[3] * g_p2;
            gt.t1 = gt.t1 + c * im3(g_t1);
            gt.t2 = gt.t2 + c * im3(g_t2);
        }
        gt.W += -wfac * Q.W * F.im;
    }
    if (WS) {
        const cv3 g_vj = iw * (s.A * u1 + (s.df * uR1) * Rh) + s.Gm * (cxd{nR, 0.0} * p2 - pR2 * P.n);
        const cv3 g_vm = cxd{-iw.re, -iw.im} * (s.A * u2 + (s.df * uR2) * Rh) +
                         s.Ge * (cxd{nR, 0.0} * p1 - pR1 * P.n);
        gs.y = gs.y - c * im3(g_Rv);
        if constexpr (NODAL) {
            gs.vj = gs.vj + c * g_vj;
            gs.vm = gs.vm + c * g_vm;
        } else {
            const cv3 g_t1 = Q.X[0] * g_vj + Q.X[2] * g_vm, g_t2 = Q.X[1] * g_vj + Q.X[3] * g_vm;
            gs.t1 = gs.t1 + c * im3(g_t1);
            gs.t2 = gs.t2 + c * im3(g_t2);
        }
        gs.W += -wfac * P.W * F.im;
    }
}

// --------------------------------------------------- per-point fields ---
// fields[i][0..7]: L0..L3 (lambda), [8..15]: X0..X3 (x) at regular point i.
// NODAL: the components in the point frame of the node-attached fields,
// L = (m1.t1, m1.t2, m2.t1, m2.t2) with m1, m2 the fields of lambda's two
// currents, X likewise from x, so that L0 t1 + L1 t2 = P m1 exactly.
template <bool NODAL>
__global__ void k_qp_fields(int64_t nt, int64_t n2, const int32_t *__restrict__ tri,
                            const double *__restrict__ qp, const double *__restrict__ frames,
                            const double2 *__restrict__ lam, const double2 *__restrict__ x,
                            double *__restrict__ fields) {
    const int64_t nq = nt * kQP;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const int64_t e = i / kQP;
    double xi, eta, w, N[6], d1[6], d2[6];
    rule7((int)(i % kQP), xi, eta, w);
    p2_shape(xi, eta, N, d1, d2);
    if constexpr (NODAL) {
        const dvec3 t1 = {qp[QT1 * nq + i], qp[(QT1 + 1) * nq + i], qp[(QT1 + 2) * nq + i]};
        const dvec3 t2 = {qp[QT2 * nq + i], qp[(QT2 + 1) * nq + i], qp[(QT2 + 2) * nq + i]};
        const double2 *c[4] = {lam, lam + n2, x, x + n2};
        for (int f = 0; f < 4; ++f) {
            const cv3 m = nodal_field(frames, tri + 6 * e, N, c[f]);
            const cxd a = cdot(m, t1), b = cdot(m, t2);
            fields[16 * i + 4 * f] = a.re;
            fields[16 * i + 4 * f + 1] = a.im;
            fields[16 * i + 4 * f + 2] = b.re;
            fields[16 * i + 4 * f + 3] = b.im;
        }
        return;
    }
    double acc[16];
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;
    for (int k = 0; k < 6; ++k) {
        const int64_t nd = tri[6 * e + k];
        const double2 v[8] = {lam[2 * nd], lam[2 * nd + 1], lam[n2 + 2 * nd], lam[n2 + 2 * nd + 1],
                              x[2 * nd], x[2 * nd + 1], x[n2 + 2 * nd], x[n2 + 2 * nd + 1]};
        for (int c = 0; c < 8; ++c) { acc[2 * c] += N[k] * v[c].x; acc[2 * c + 1] += N[k] * v[c].y; }
    }
    for (int c = 0; c < 16; ++c) fields[16 * i + c] = acc[c];
}

__device__ inline void load_tpt(const double *qp, const double *fields, int64_t nq, int64_t i, TPt &P) {
    P.x = {qp[QX * nq + i], qp[(QX + 1) * nq + i], qp[(QX + 2) * nq + i]};
    P.W = qp[QW * nq + i];
    P.n = {qp[QN * nq + i], qp[(QN + 1) * nq + i], qp[(QN + 2) * nq + i]};
    P.t1 = {qp[QT1 * nq + i], qp[(QT1 + 1) * nq + i], qp[(QT1 + 2) * nq + i]};
    P.t2 = {qp[QT2 * nq + i], qp[(QT2 + 1) * nq + i], qp[(QT2 + 2) * nq + i]};
    const double *f = fields + 16 * i;
    for (int c = 0; c < 4; ++c) P.L[c] = {f[2 * c], f[2 * c + 1]};
}
__device__ inline void load_spt(const double *qp, const double *fields, int64_t nq, int64_t i, SPt &Q) {
    Q.y = {qp[QX * nq + i], qp[(QX + 1) * nq + i], qp[(QX + 2) * nq + i]};
    Q.W = qp[QW * nq + i];
    Q.t1 = {qp[QT1 * nq + i], qp[(QT1 + 1) * nq + i], qp[(QT1 + 2) * nq + i]};
    Q.t2 = {qp[QT2 * nq + i], qp[(QT2 + 1) * nq + i], qp[(QT2 + 2) * nq + i]};
    const double *f = fields + 16 * i + 8;
    for (int c = 0; c < 4; ++c) Q.X[c] = {f[2 * c], f[2 * c + 1]};
}

__device__ inline bool share_vertex(const int32_t *te, const int32_t *tf) {
    bool s = false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s = s || te[a] == tf[b];
    return s;
}

// --------------------------------------------------- regular pairs ---
// Point adjoint table qb[i][13]: x(3), W(1), n(3), t1(3), t2(3).
// NODAL, qb[i][31]: x(3), W(1), n(3), then the complex adjoints (re, im per
// component) of p1, p2 (test side) and vj, vm (trial side).
constexpr int kQB = 13;
constexpr int kQBN = 31;
template <bool NODAL> constexpr int qb_stride() { return NODAL ? kQBN : kQB; }
constexpr int kGroups = 36;   // 36 x 7 = 252 threads

__device__ inline void put_cv3(double *o, cv3 v) {
    o[0] = v.x.re; o[1] = v.x.im; o[2] = v.y.re; o[3] = v.y.im; o[4] = v.z.re; o[5] = v.z.im;
}
__device__ inline cv3 get_cv3(const double *o) { return {{o[0], o[1]}, {o[2], o[3]}, {o[4], o[5]}}; }

// TEST = true: workgroup per test triangle e, its 7 points accumulate over
// every regular trial point; TEST = false: the same with roles exchanged.
template <bool TEST, bool NODAL>
__global__ __launch_bounds__(256) void k_shape_regular(int64_t nt, const double *__restrict__ qp,
                                                       const double *__restrict__ fields,
                                                       const int32_t *__restrict__ tri, const KernelConst *Kp,
                                                       cxd iw, double *__restrict__ qb) {
    constexpr int kS = qb_stride<NODAL>();
    __shared__ double s_red[kGroups][kQP][kS];
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int64_t nq = nt * kQP;
    const int q = tid % kQP, grp = tid / kQP;
    const bool active = grp < kGroups;
    const KernelConst &K = *Kp;
    TGrad gt;
    SGrad gs;
    zero(gt);
    zero(gs);
    const int32_t *te = tri + 6 * e;
    if (active) {
        TPt P;
        SPt Q;
        if (TEST) load_tpt(qp, fields, nq, e * kQP + q, P);
        else load_spt(qp, fields, nq, e * kQP + q, Q);
        for (int64_t idx = grp; idx < nq; idx += kGroups) {
            const int64_t f = idx / kQP;
            if (share_vertex(te, tri + 6 * f)) continue;
            if (TEST) {
                load_spt(qp, fields, nq, idx, Q);
                pair_adjoint<true, false, NODAL>(K, iw, P, Q, 1.0, gt, gs);
            } else {
                load_tpt(qp, fields, nq, idx, P);
                pair_adjoint<false, true, NODAL>(K, iw, P, Q, 1.0, gt, gs);
            }
        }
        double v[kS];
        for (int c = 0; c < kS; ++c) v[c] = 0.0;
        if (TEST) {
            v[0] = gt.x.x; v[1] = gt.x.y; v[2] = gt.x.z; v[3] = gt.W;
            v[4] = gt.n.x; v[5] = gt.n.y; v[6] = gt.n.z;
            if constexpr (NODAL) {
                put_cv3(v + 7, gt.p1);
                put_cv3(v + 13, gt.p2);
            } else {
                v[7] = gt.t1.x; v[8] = gt.t1.y; v[9] = gt.t1.z; v[10] = gt.t2.x; v[11] = gt.t2.y; v[12] = gt.t2.z;
            }
        } else {
            v[0] = gs.y.x; v[1] = gs.y.y; v[2] = gs.y.z; v[3] = gs.W;
            if constexpr (NODAL) {
                put_cv3(v + 19, gs.vj);
                put_cv3(v + 25, gs.vm);
            } else {
                v[7] = gs.t1.x; v[8] = gs.t1.y; v[9] = gs.t1.z; v[10] = gs.t2.x; v[11] = gs.t2.y; v[12] = gs.t2.z;
            }
        }
        for (int c = 0; c < kS; ++c) s_red[grp][q][c] = v[c];
    }
    __syncthreads();
    if (tid < kQP * kS) {
        const int qq = tid / kS, c = tid % kS;
        double acc = 0.0;
        for (int g = 0; g < kGroups; ++g) acc += s_red[g][qq][c];
        qb[(e * kQP + qq) * kS + c] += acc;
    }
}

// ------------------------------------------------ single-point terms ---
// + Im(g^T x)    far field functional, g^T x = sum_q pre W [j.e_perp - j_m.(e x r)]
// + Im(lambda^T b)  right-hand side, sum_q W [-u1.E + u2.H]
// - Im(lambda^T M-part x)  mass, sum_q W [c_eps (L0 X2 + L1 X3) + c_mu (L2 X0 + L3 X1)]
struct SingleArgs {
    dvec3 khat;
    cxd pol[3], ec[3];    // incident polarisation, conj(pol)
    double ka;
    cxd ce, cm;
};

template <bool NODAL>
__global__ __launch_bounds__(256) void k_shape_single(int64_t nt, const double *__restrict__ qp, const double *__restrict__ fields,
                               SingleArgs a, double *__restrict__ qb) {
    const int64_t nq = nt * kQP;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    TPt P;
    SPt Q;
    load_tpt(qp, fields, nq, i, P);
    load_spt(qp, fields, nq, i, Q);
    const dvec3 r = a.khat, y = P.x, n = P.n;
    const double W = P.W;
    dvec3 gx = {0, 0, 0}, gn = {0, 0, 0}, gt1 = {0, 0, 0}, gt2 = {0, 0, 0};
    double gW = 0.0;
    // NODAL: complex adjoints of the point's vectors p1, p2, vj, vm
    cv3 gp1 = czero3(), gp2 = czero3(), gvj = czero3(), gvm = czero3();
    // far field
    {
        double sn, cs;
        sincos(-a.ka * dot(r, y), &sn, &cs);
        const cxd pre = cxd{0.0, a.ka * 0.079577471545947667884} * cxd{cs, sn};
        const cv3 e = {a.ec[0], a.ec[1], a.ec[2]};
        const cxd re = cdot(e, r);
        const cv3 ep = e - re * r;
        const cv3 ex = ccross(e, r);
        const cv3 j = Q.X[0] * P.t1 + Q.X[1] * P.t2, jm = Q.X[2] * P.t1 + Q.X[3] * P.t2;
        const cxd G1 = cdot(j, ep) - cdot(jm, ex);
        const cxd T = pre * cxd{W * G1.re, W * G1.im};
        gx = gx + im3(cxd{0.0, -a.ka} * T * r);
        gW += (pre * G1).im;
        if constexpr (NODAL) {
            gvj = gvj + (cxd{W, 0} * pre) * ep;
            gvm = gvm - (cxd{W, 0} * pre) * ex;
        } else {
            gt1 = gt1 + im3((cxd{W, 0} * pre) * (Q.X[0] * ep - Q.X[2] * ex));
            gt2 = gt2 + im3((cxd{W, 0} * pre) * (Q.X[1] * ep - Q.X[3] * ex));
        }
    }
    // right-hand side
    {
        double sn, cs;
        sincos(a.ka * dot(a.khat, y), &sn, &cs);
        const cxd ph = {cs, sn};
        const cv3 E = {ph * a.pol[0], ph * a.pol[1], ph * a.pol[2]};
        const cv3 H = ccross(a.khat, E);
        const cv3 p1 = P.L[0] * P.t1 + P.L[1] * P.t2, p2 = P.L[2] * P.t1 + P.L[3] * P.t2;
        const cv3 u1 = ccross(p1, n), u2 = ccross(p2, n);
        const cxd V = cdot(u2, H) - cdot(u1, E);
        gW += V.im;
        gx = gx + im3((cxd{0.0, a.ka} * cxd{W * V.re, W * V.im}) * a.khat);
        const cv3 g_u1 = cxd{-W, 0.0} * E, g_u2 = cxd{W, 0.0} * H;
        const cv3 g_p1 = ccross(n, g_u1), g_p2 = ccross(n, g_u2);
        gn = gn + im3(ccross(g_u1, p1) + ccross(g_u2, p2));
        if constexpr (NODAL) {
            gp1 = gp1 + g_p1;
            gp2 = gp2 + g_p2;
        } else {
            gt1 = gt1 + im3(P.L[0] * g_p1 + P.L[2] * g_p2);
            gt2 = gt2 + im3(P.L[1] * g_p1 + P.L[3] * g_p2);
        }
    }
    // mass (p1 . vm = L0 X2 + L1 X3: both are expansions on the same
    // orthonormal pair)
    {
        const cxd m = a.ce * (P.L[0] * Q.X[2] + P.L[1] * Q.X[3]) + a.cm * (P.L[2] * Q.X[0] + P.L[3] * Q.X[1]);
        gW -= m.im;
        if constexpr (NODAL) {
            const cv3 p1 = P.L[0] * P.t1 + P.L[1] * P.t2, p2 = P.L[2] * P.t1 + P.L[3] * P.t2;
            const cv3 vj = Q.X[0] * P.t1 + Q.X[1] * P.t2, vm = Q.X[2] * P.t1 + Q.X[3] * P.t2;
            const cxd we = cxd{-W, 0} * a.ce, wm = cxd{-W, 0} * a.cm;
            gp1 = gp1 + we * vm;
            gvm = gvm + we * p1;
            gp2 = gp2 + wm * vj;
            gvj = gvj + wm * p2;
        }
    }
    constexpr int kS = qb_stride<NODAL>();
    double v[kS];
    v[0] = gx.x; v[1] = gx.y; v[2] = gx.z; v[3] = gW; v[4] = gn.x; v[5] = gn.y; v[6] = gn.z;
    if constexpr (NODAL) {
        put_cv3(v + 7, gp1);
        put_cv3(v + 13, gp2);
        put_cv3(v + 19, gvj);
        put_cv3(v + 25, gvm);
    } else {
        v[7] = gt1.x; v[8] = gt1.y; v[9] = gt1.z; v[10] = gt2.x; v[11] = gt2.y; v[12] = gt2.z;
    }
    double *o = qb + i * kS;
    for (int c = 0; c < kS; ++c) o[c] += v[c];
}

// ------------------------------------------ P2 point: forward + reverse ---
struct P2Fwd {
    dvec3 x, a1, a2, c, n, u1, u2, w1, w2, w3, t1, t2;
    double J, l1, l3;     // |w1|, |w3|
    double N[6], Nxi[6], Neta[6];
};

__device__ inline void p2_forward(const double *__restrict__ xyz, const double *__restrict__ frames,
                                  const int32_t *t, double xi, double eta, P2Fwd &P) {
    p2_shape(xi, eta, P.N, P.Nxi, P.Neta);
    P.x = {0, 0, 0}; P.a1 = {0, 0, 0}; P.a2 = {0, 0, 0}; P.u1 = {0, 0, 0}; P.u2 = {0, 0, 0};
    for (int k = 0; k < 6; ++k) {
        const int64_t v = t[k];
        const dvec3 X = load3(xyz, v);
        P.x = P.x + P.N[k] * X;
        P.a1 = P.a1 + P.Nxi[k] * X;
        P.a2 = P.a2 + P.Neta[k] * X;
        const double *f = frames + 9 * v;
        P.u1 = P.u1 + P.N[k] * dvec3{f[3], f[4], f[5]};
        P.u2 = P.u2 + P.N[k] * dvec3{f[6], f[7], f[8]};
    }
    P.c = cross(P.a1, P.a2);
    P.J = sqrt(dot(P.c, P.c));
    P.n = (1.0 / P.J) * P.c;
    P.w1 = P.u1 - dot(P.n, P.u1) * P.n;
    P.l1 = sqrt(dot(P.w1, P.w1));
    P.t1 = (1.0 / P.l1) * P.w1;
    P.w2 = P.u2 - dot(P.n, P.u2) * P.n;
    P.w3 = P.w2 - dot(P.t1, P.w2) * P.t1;
    P.l3 = sqrt(dot(P.w3, P.w3));
    P.t2 = (1.0 / P.l3) * P.w3;
}

// Adjoints of (x, J, n, t1, t2) -> node positions (gX) and nodal tangents
// (gT1, gT2) of the 6 nodes of the triangle.
__device__ inline void p2_reverse(const P2Fwd &P, dvec3 bx, double bJ, dvec3 bn, dvec3 bt1, dvec3 bt2, dvec3 gX[6],
                                  dvec3 gT1[6], dvec3 gT2[6]) {
    // t2 = w3 / |w3|
    const dvec3 bw3 = (1.0 / P.l3) * (bt2 - dot(bt2, P.t2) * P.t2);
    // w3 = w2 - (t1.w2) t1
    const double s = dot(P.t1, P.w2), bs = dot(bw3, P.t1);
    const dvec3 bw2 = bw3 - bs * P.t1;
    bt1 = bt1 - bs * P.w2 - s * bw3;
    // w2 = u2 - (n.u2) n
    const double nu2 = dot(P.n, P.u2), bwn2 = dot(bw2, P.n);
    const dvec3 bu2 = bw2 - bwn2 * P.n;
    bn = bn - bwn2 * P.u2 - nu2 * bw2;
    // t1 = w1 / |w1|
    const dvec3 bw1 = (1.0 / P.l1) * (bt1 - dot(bt1, P.t1) * P.t1);
    // w1 = u1 - (n.u1) n
    const double nu1 = dot(P.n, P.u1), bwn1 = dot(bw1, P.n);
    const dvec3 bu1 = bw1 - bwn1 * P.n;
    bn = bn - bwn1 * P.u1 - nu1 * bw1;
    // n = c / J, J = |c|
    const dvec3 bc = (1.0 / P.J) * (bn - dot(bn, P.n) * P.n) + bJ * P.n;
    // c = a1 x a2
    const dvec3 ba1 = cross(P.a2, bc), ba2 = cross(bc, P.a1);
    for (int k = 0; k < 6; ++k) {
        gX[k] = P.N[k] * bx + P.Nxi[k] * ba1 + P.Neta[k] * ba2;
        gT1[k] = P.N[k] * bu1;
        gT2[k] = P.N[k] * bu2;
    }
}

__device__ inline void atomic_add3(double *p, dvec3 v) {
    unsafeAtomicAdd(p, v.x);
    unsafeAtomicAdd(p + 1, v.y);
    unsafeAtomicAdd(p + 2, v.z);
}

// Regular points: back through the P2 map and frame of their triangle.
// nodeb[v][9]: position (3), nodal t1 (3), nodal t2 (3) adjoints.
// NODAL: back through the projections p = m - (m.n) n of the four
// node-attached fields to the normal and the nodal tangents; the point
// frame does not enter.
template <bool NODAL>
__global__ __launch_bounds__(256) void k_qp_backprop(int64_t nt, int64_t n2, const double *__restrict__ xyz,
                              const double *__restrict__ frames, const int32_t *__restrict__ tri,
                              const double2 *__restrict__ lam, const double2 *__restrict__ x,
                              const double *__restrict__ qb, double *__restrict__ nodeb) {
    const int64_t nq = nt * kQP;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const int64_t e = i / kQP;
    double xi, eta, w;
    rule7((int)(i % kQP), xi, eta, w);
    P2Fwd P;
    p2_forward(xyz, frames, tri + 6 * e, xi, eta, P);
    constexpr int kS = qb_stride<NODAL>();
    const double *b = qb + i * kS;
    dvec3 gX[6], gT1[6], gT2[6];
    if constexpr (NODAL) {
        const int32_t *t = tri + 6 * e;
        const double2 *c[4] = {lam, lam + n2, x, x + n2};
        dvec3 bn = {b[4], b[5], b[6]};
        cv3 gm[4];
        for (int f = 0; f < 4; ++f)
            gm[f] = proj_reverse(get_cv3(b + 7 + 6 * f), nodal_field(frames, t, P.N, c[f]), P.n, bn);
        p2_reverse(P, {b[0], b[1], b[2]}, w * b[3], bn, {0, 0, 0}, {0, 0, 0}, gX, gT1, gT2);
        nodal_tangent_adjoint<4>(t, P.N, c, gm, gT1, gT2);
    } else {
        p2_reverse(P, {b[0], b[1], b[2]}, w * b[3], {b[4], b[5], b[6]}, {b[7], b[8], b[9]}, {b[10], b[11], b[12]},
                   gX, gT1, gT2);
    }
    for (int k = 0; k < 6; ++k) {
        double *o = nodeb + 9 * (int64_t)tri[6 * e + k];
        atomic_add3(o, gX[k]);
        atomic_add3(o + 3, gT1[k]);
        atomic_add3(o + 6, gT2[k]);
    }
}

// ------------------------------------------------- singular pairs ---
// One wavefront per coincident / common-edge / common-vertex pair, the
// Sauter-Schwab points of the fill, one point per lane and batch.  After
// each batch the 6 x 9 test-node adjoints of every lane go through LDS and
// lane c < 54 adds column c over the 64 points (then the same for the trial
// nodes), so each lane keeps two running sums and the workgroup 28 KB of LDS.
struct ShapeSsqArgs {
    int64_t n2, npairs;
    const int32_t *pairs, *tri;
    const double *xyz, *frames;
    const double2 *lam, *x;
    int order;
    double glx[kMaxSSQ], glw[kMaxSSQ];
    const KernelConst *K;
    cxd iw;
    double *nodeb;
};

template <bool NODAL>
__global__ __launch_bounds__(64) void k_shape_ssq(ShapeSsqArgs a) {
    constexpr int kCols = 54, kStride = 55;
    __shared__ double s_buf[64 * kStride];
    const int lane = threadIdx.x;
    const int64_t pid = blockIdx.x;
    const int32_t e = a.pairs[4 * pid], f = a.pairs[4 * pid + 1];
    const int cls = a.pairs[4 * pid + 2], code = a.pairs[4 * pid + 3];
    const int n = a.order, n4 = n * n * n * n;
    const int nreg = cls == 3 ? 6 : (cls == 2 ? 5 : 2);
    const int npts = nreg * n4;
    const int32_t *te = a.tri + 6 * e, *tf = a.tri + 6 * f;
    const KernelConst &K = *a.K;
    double accT = 0.0, accS = 0.0;       // column `lane` of the test / trial adjoints
    double *row = s_buf + lane * kStride;
    for (int base = 0; base < npts; base += 64) {
        const int idx = base + lane;
        const bool on = idx < npts;
        P2Fwd X, Y;
        TGrad gt;
        SGrad gs;
        zero(gt);
        zero(gs);
        if (on) {
            const int r = idx / n4;
            int g = idx % n4;
            const int i3 = g % n; g /= n;
            const int i2 = g % n; g /= n;
            const int i1 = g % n; g /= n;
            const int i0 = g;
            double s1, t1, s2, t2;
            const double jac = ss_region(cls, r, a.glx[i0], a.glx[i1], a.glx[i2], a.glx[i3], s1, t1, s2, t2);
            const double wg = jac * a.glw[i0] * a.glw[i1] * a.glw[i2] * a.glw[i3];
            double xe, ye, xf, yf;
            ss_local(code & 63, s1, t1, xe, ye);
            ss_local(code >> 6, s2, t2, xf, yf);
            p2_forward(a.xyz, a.frames, te, xe, ye, X);
            p2_forward(a.xyz, a.frames, tf, xf, yf, Y);
            TPt P;
            SPt Q;
            P.x = X.x; P.n = X.n; P.t1 = X.t1; P.t2 = X.t2; P.W = X.J;
            Q.y = Y.x; Q.t1 = Y.t1; Q.t2 = Y.t2; Q.W = Y.J;
            if constexpr (NODAL) {
                // components of the node-attached fields in the point frames
                const double2 *cl[2] = {a.lam, a.lam + a.n2}, *cx_[2] = {a.x, a.x + a.n2};
                for (int f = 0; f < 2; ++f) {
                    const cv3 m = nodal_field(a.frames, te, X.N, cl[f]), v = nodal_field(a.frames, tf, Y.N, cx_[f]);
                    P.L[2 * f] = cdot(m, X.t1);
                    P.L[2 * f + 1] = cdot(m, X.t2);
                    Q.X[2 * f] = cdot(v, Y.t1);
                    Q.X[2 * f + 1] = cdot(v, Y.t2);
                }
            } else {
                for (int c = 0; c < 4; ++c) { P.L[c] = {0, 0}; Q.X[c] = {0, 0}; }
                for (int k = 0; k < 6; ++k) {
                    const int64_t ne = te[k], nf = tf[k];
                    const double2 l[4] = {a.lam[2 * ne], a.lam[2 * ne + 1], a.lam[a.n2 + 2 * ne],
                                          a.lam[a.n2 + 2 * ne + 1]};
                    const double2 u[4] = {a.x[2 * nf], a.x[2 * nf + 1], a.x[a.n2 + 2 * nf], a.x[a.n2 + 2 * nf + 1]};
                    for (int c = 0; c < 4; ++c) {
                        P.L[c] = P.L[c] + cxd{X.N[k] * l[c].x, X.N[k] * l[c].y};
                        Q.X[c] = Q.X[c] + cxd{Y.N[k] * u[c].x, Y.N[k] * u[c].y};
                    }
                }
            }
            pair_adjoint<true, true, NODAL>(K, a.iw, P, Q, wg, gt, gs);
        }
        // test side
        {
            dvec3 gX[6], gT1[6], gT2[6];
            if (on) {
                if constexpr (NODAL) {
                    const double2 *cl[2] = {a.lam, a.lam + a.n2};
                    dvec3 bn = gt.n;
                    const cv3 gm[2] = {proj_reverse(gt.p1, nodal_field(a.frames, te, X.N, cl[0]), X.n, bn),
                                       proj_reverse(gt.p2, nodal_field(a.frames, te, X.N, cl[1]), X.n, bn)};
                    p2_reverse(X, gt.x, gt.W, bn, {0, 0, 0}, {0, 0, 0}, gX, gT1, gT2);
                    nodal_tangent_adjoint<2>(te, X.N, cl, gm, gT1, gT2);
                } else {
                    p2_reverse(X, gt.x, gt.W, gt.n, gt.t1, gt.t2, gX, gT1, gT2);
                }
            }
            for (int k = 0; k < 6; ++k) {
                double *o = row + 9 * k;
                if (on) {
                    o[0] = gX[k].x; o[1] = gX[k].y; o[2] = gX[k].z;
                    o[3] = gT1[k].x; o[4] = gT1[k].y; o[5] = gT1[k].z;
                    o[6] = gT2[k].x; o[7] = gT2[k].y; o[8] = gT2[k].z;
                } else {
                    for (int c = 0; c < 9; ++c) o[c] = 0.0;
                }
            }
        }
        __syncthreads();
        if (lane < kCols)
            for (int l = 0; l < 64; ++l) accT += s_buf[l * kStride + lane];
        __syncthreads();
        // trial side
        {
            dvec3 gX[6], gT1[6], gT2[6];
            if (on) {
                if constexpr (NODAL) {
                    const double2 *cx_[2] = {a.x, a.x + a.n2};
                    dvec3 bn = {0, 0, 0};
                    const cv3 gm[2] = {proj_reverse(gs.vj, nodal_field(a.frames, tf, Y.N, cx_[0]), Y.n, bn),
                                       proj_reverse(gs.vm, nodal_field(a.frames, tf, Y.N, cx_[1]), Y.n, bn)};
                    p2_reverse(Y, gs.y, gs.W, bn, {0, 0, 0}, {0, 0, 0}, gX, gT1, gT2);
                    nodal_tangent_adjoint<2>(tf, Y.N, cx_, gm, gT1, gT2);
                } else {
                    p2_reverse(Y, gs.y, gs.W, {0, 0, 0}, gs.t1, gs.t2, gX, gT1, gT2);
                }
            }
            for (int k = 0; k < 6; ++k) {
                double *o = row + 9 * k;
                if (on) {
                    o[0] = gX[k].x; o[1] = gX[k].y; o[2] = gX[k].z;
                    o[3] = gT1[k].x; o[4] = gT1[k].y; o[5] = gT1[k].z;
                    o[6] = gT2[k].x; o[7] = gT2[k].y; o[8] = gT2[k].z;
                } else {
                    for (int c = 0; c < 9; ++c) o[c] = 0.0;
                }
            }
        }
        __syncthreads();
        if (lane < kCols)
            for (int l = 0; l < 64; ++l) accS += s_buf[l * kStride + lane];
        __syncthreads();
    }
    if (lane < kCols) {
        const int k = lane / 9, comp = lane % 9;
        unsafeAtomicAdd(&a.nodeb[9 * (int64_t)te[k] + comp], accT);
        unsafeAtomicAdd(&a.nodeb[9 * (int64_t)tf[k] + comp], accS);
    }
}

// -------------------------------------------------- nodal frames ---
// Tangents of triangle t at its local node k after the cyclic re-indexing
// that puts the node at the origin (vertex) or at (1/2, 0) (mid-edge node).
__device__ inline void node_tangents(int32_t k, const int32_t *t, const double *X, dvec3 &a1, dvec3 &a2) {
    if (k < 3) {
        const int kn = (k + 1) % 3, kp = (k + 2) % 3;
        a1 = -3.0 * load3(X, t[k]) + 4.0 * load3(X, t[3 + k]) - load3(X, t[kn]);
        a2 = -3.0 * load3(X, t[k]) + 4.0 * load3(X, t[3 + kp]) - load3(X, t[kp]);
    } else {
        const int aa = k - 3, b = (aa + 1) % 3, c = (aa + 2) % 3;
        a1 = load3(X, t[b]) - load3(X, t[aa]);
        a2 = 2.0 * (load3(X, t[3 + b]) + load3(X, t[3 + c]) - load3(X, t[3 + aa])) - load3(X, t[aa]) -
             load3(X, t[c]);
    }
}

// Back through t1 = (ref x n)/|ref x n|, t2 = n x t1 (reference vector held
// fixed), n = S/|S|, S = sum over incident triangles of (a1 x a2)/(g11 g22).
__global__ void k_frames_backprop(int64_t nn, const double *__restrict__ xyz, const int32_t *__restrict__ tri,
                                  const int32_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc,
                                  const double *__restrict__ nodeb_t, double *__restrict__ nodeb_x) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= nn) return;
    dvec3 S = {0, 0, 0};
    for (int32_t s = inc_ptr[v]; s < inc_ptr[v + 1]; ++s) {
        dvec3 a1, a2;
        node_tangents(inc[s] & 7, tri + 6 * (inc[s] >> 3), xyz, a1, a2);
        S = S + (1.0 / (dot(a1, a1) * dot(a2, a2))) * cross(a1, a2);
    }
    const double ls = sqrt(dot(S, S));
    const dvec3 n = (1.0 / ls) * S;
    const dvec3 ref = fabs(n.z) > 0.9 ? dvec3{1.0, 0.0, 0.0} : dvec3{0.0, 0.0, 1.0};
    const dvec3 wv = cross(ref, n);
    const double lw = sqrt(dot(wv, wv));
    const dvec3 t1 = (1.0 / lw) * wv;
    const double *b = nodeb_t + 9 * v;
    const dvec3 bt1 = {b[3], b[4], b[5]}, bt2 = {b[6], b[7], b[8]};
    // t2 = n x t1
    dvec3 bn = cross(t1, bt2);
    const dvec3 bt1s = bt1 + cross(bt2, n);
    // t1 = w / |w|, w = ref x n
    const dvec3 bw = (1.0 / lw) * (bt1s - dot(bt1s, t1) * t1);
    bn = bn + cross(bw, ref);
    // n = S / |S|
    const dvec3 bS = (1.0 / ls) * (bn - dot(bn, n) * n);
    for (int32_t s = inc_ptr[v]; s < inc_ptr[v + 1]; ++s) {
        const int32_t k = inc[s] & 7;
        const int32_t *t = tri + 6 * (inc[s] >> 3);
        dvec3 a1, a2;
        node_tangents(k, t, xyz, a1, a2);
        const double g11 = dot(a1, a1), g22 = dot(a2, a2), D = g11 * g22;
        const dvec3 c = cross(a1, a2);
        const dvec3 bc = (1.0 / D) * bS;
        const double q = dot(bS, c) / (D * D);
        const dvec3 ba1 = cross(a2, bc) - (2.0 * q * g22) * a1;
        const dvec3 ba2 = cross(bc, a1) - (2.0 * q * g11) * a2;
        if (k < 3) {
            const int kn = (k + 1) % 3, kp = (k + 2) % 3;
            atomic_add3(nodeb_x + 9 * (int64_t)t[k], -3.0 * (ba1 + ba2));
            atomic_add3(nodeb_x + 9 * (int64_t)t[3 + k], 4.0 * ba1);
            atomic_add3(nodeb_x + 9 * (int64_t)t[kn], -1.0 * ba1);
            atomic_add3(nodeb_x + 9 * (int64_t)t[3 + kp], 4.0 * ba2);
            atomic_add3(nodeb_x + 9 * (int64_t)t[kp], -1.0 * ba2);
        } else {
            const int aa = k - 3, bb = (aa + 1) % 3, cc = (aa + 2) % 3;
            atomic_add3(nodeb_x + 9 * (int64_t)t[bb], ba1);
            atomic_add3(nodeb_x + 9 * (int64_t)t[aa], -1.0 * (ba1 + ba2));
            atomic_add3(nodeb_x + 9 * (int64_t)t[3 + bb], 2.0 * ba2);
            atomic_add3(nodeb_x + 9 * (int64_t)t[3 + cc], 2.0 * ba2);
            atomic_add3(nodeb_x + 9 * (int64_t)t[3 + aa], -2.0 * ba2);
            atomic_add3(nodeb_x + 9 * (int64_t)t[cc], -1.0 * ba2);
        }
    }
}

// d sigma / d delta_v along the displacement direction of node v (dir[v],
// or the nodal normal when dir is null), and the full position gradient
__global__ void k_shape_out(int64_t nn, double scale, const double *__restrict__ frames,
                            const double *__restrict__ dir, const double *__restrict__ nodeb_x, double *dnode,
                            double *dx) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= nn) return;
    const double *b = nodeb_x + 9 * v, *nv = dir ? dir + 3 * v : frames + 9 * v;
    if (dnode) dnode[v] = scale * (b[0] * nv[0] + b[1] * nv[1] + b[2] * nv[2]);
    if (dx) for (int c = 0; c < 3; ++c) dx[3 * v + c] = scale * b[c];
}

// --------------------------------------------------------------- host ---
int shape_grad_run(const mbem_op *op, const mbem_params *p, const double2 *x, const double2 *lam,
                   const double *khat, const double2 *pol, const double *dir, double *dnode, double *dx,
                   hipStream_t s) {
    const mbem_mesh *m = op->mesh;
    const int64_t nt = m->nt, nq = nt * kQP, nn = m->nn;
    double *fields = nullptr, *qb = nullptr, *nodeb = nullptr, *nodeb_x = nullptr;
    auto cleanup = [&]() {
        if (fields) (void)hipFree(fields);
        if (qb) (void)hipFree(qb);
        if (nodeb) (void)hipFree(nodeb);
        if (nodeb_x) (void)hipFree(nodeb_x);
    };
    const bool nodal = op->p.frame == MBEM_FRAME_NODAL;
    const int kS = nodal ? kQBN : kQB;
    if (hipMalloc((void **)&fields, sizeof(double) * 16 * nq) != hipSuccess ||
        hipMalloc((void **)&qb, sizeof(double) * kS * nq) != hipSuccess ||
        hipMalloc((void **)&nodeb, sizeof(double) * 9 * nn) != hipSuccess ||
        hipMalloc((void **)&nodeb_x, sizeof(double) * 9 * nn) != hipSuccess) {
        cleanup();
        set_error("shape gradient workspace: out of memory");
        return MBEM_ENOMEM;
    }
    int st = MBEM_OK;
    auto launch_ok = [&]() {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) { set_error(std::string("shape gradient launch: ") + hipGetErrorString(e)); st = MBEM_EDEVICE; }
        return st == MBEM_OK;
    };
    (void)hipMemsetAsync(qb, 0, sizeof(double) * kS * nq, s);
    (void)hipMemsetAsync(nodeb, 0, sizeof(double) * 9 * nn, s);
    (void)hipMemsetAsync(nodeb_x, 0, sizeof(double) * 9 * nn, s);
    const unsigned gq = (unsigned)((nq + 255) / 256);
    const cxd iw = {op->iw.x, op->iw.y};
    if (nodal)
        hipLaunchKernelGGL(k_qp_fields<true>, dim3(gq), dim3(256), 0, s, nt, op->n2, m->d_tri, m->d_qp, m->d_frames,
                           lam, x, fields);
    else
        hipLaunchKernelGGL(k_qp_fields<false>, dim3(gq), dim3(256), 0, s, nt, op->n2, m->d_tri, m->d_qp,
                           m->d_frames, lam, x, fields);
    if (launch_ok()) {
        if (nodal)
            hipLaunchKernelGGL((k_shape_regular<true, true>), dim3((unsigned)nt), dim3(256), 0, s, nt, m->d_qp,
                               fields, m->d_tri, op->d_kconst, iw, qb);
        else
            hipLaunchKernelGGL((k_shape_regular<true, false>), dim3((unsigned)nt), dim3(256), 0, s, nt, m->d_qp,
                               fields, m->d_tri, op->d_kconst, iw, qb);
        launch_ok();
    }
    if (st == MBEM_OK) {
        if (nodal)
            hipLaunchKernelGGL((k_shape_regular<false, true>), dim3((unsigned)nt), dim3(256), 0, s, nt, m->d_qp,
                               fields, m->d_tri, op->d_kconst, iw, qb);
        else
            hipLaunchKernelGGL((k_shape_regular<false, false>), dim3((unsigned)nt), dim3(256), 0, s, nt, m->d_qp,
                               fields, m->d_tri, op->d_kconst, iw, qb);
        launch_ok();
    }
    if (st == MBEM_OK) {
        SingleArgs sa;
        sa.khat = {khat[0], khat[1], khat[2]};
        for (int c = 0; c < 3; ++c) { sa.pol[c] = {pol[c].x, pol[c].y}; sa.ec[c] = {pol[c].x, -pol[c].y}; }
        sa.ka = p->k0;
        sa.ce = {op->ce.x, op->ce.y};
        sa.cm = {op->cm.x, op->cm.y};
        if (nodal) hipLaunchKernelGGL(k_shape_single<true>, dim3(gq), dim3(256), 0, s, nt, m->d_qp, fields, sa, qb);
        else hipLaunchKernelGGL(k_shape_single<false>, dim3(gq), dim3(256), 0, s, nt, m->d_qp, fields, sa, qb);
        launch_ok();
    }
    if (st == MBEM_OK) {
        if (nodal)
            hipLaunchKernelGGL(k_qp_backprop<true>, dim3(gq), dim3(256), 0, s, nt, op->n2, m->d_xyz, m->d_frames,
                               m->d_tri, lam, x, qb, nodeb);
        else
            hipLaunchKernelGGL(k_qp_backprop<false>, dim3(gq), dim3(256), 0, s, nt, op->n2, m->d_xyz, m->d_frames,
                               m->d_tri, lam, x, qb, nodeb);
        launch_ok();
    }
    if (st == MBEM_OK && m->n_spairs > 0) {
        ShapeSsqArgs a;
        a.n2 = op->n2;
        a.npairs = m->n_spairs;
        a.pairs = m->d_spairs;
        a.tri = m->d_tri;
        a.xyz = m->d_xyz;
        a.frames = m->d_frames;
        a.lam = lam;
        a.x = x;
        a.order = op->p.ssq_order > 0 ? op->p.ssq_order : 4;
        double gx[kMaxSSQ], gw[kMaxSSQ];
        gauss_legendre(a.order, gx, gw);
        for (int i = 0; i < kMaxSSQ; ++i) {
            a.glx[i] = i < a.order ? 0.5 * (1.0 + gx[a.order - 1 - i]) : 0.0;
            a.glw[i] = i < a.order ? 0.5 * gw[a.order - 1 - i] : 0.0;
        }
        a.K = op->d_kconst;
        a.iw = iw;
        a.nodeb = nodeb;
        if (nodal) hipLaunchKernelGGL(k_shape_ssq<true>, dim3((unsigned)m->n_spairs), dim3(64), 0, s, a);
        else hipLaunchKernelGGL(k_shape_ssq<false>, dim3((unsigned)m->n_spairs), dim3(64), 0, s, a);
        launch_ok();
    }
    if (st == MBEM_OK) {
        // position adjoints so far, then the frame path adds to the copy
        (void)hipMemcpyAsync(nodeb_x, nodeb, sizeof(double) * 9 * nn, hipMemcpyDeviceToDevice, s);
        hipLaunchKernelGGL(k_frames_backprop, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, nn, m->d_xyz,
                           m->d_tri, m->d_inc_ptr, m->d_inc, (const double *)nodeb, nodeb_x);
        launch_ok();
    }
    if (st == MBEM_OK) {
        hipLaunchKernelGGL(k_shape_out, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, nn,
                           4.0 * 3.14159265358979323846 / p->k0, m->d_frames, dir, (const double *)nodeb_x, dnode,
                           dx);
        launch_ok();
    }
    if (hipStreamSynchronize(s) != hipSuccess && st == MBEM_OK) { set_error("shape gradient failed"); st = MBEM_EDEVICE; }
    cleanup();
    return st;
}

}  // namespace mbem
