/*
 * mbem oracle -- plain FP64 CPU reference of the nodal P2 Mueller Galerkin
 * discretisation (Y. Luo, "A High-Order Nodal Galerkin Formulation for the
 * Mueller Equation: Bypassing Divergence Conformity via Kernel Cancellation",
 * arXiv 2604.21181).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the product path never
 * calls it, and it shares no code, header or table with the HIP library.
 *
 * It is written to be checked against the paper by eye: every quantity is
 * computed the way the paper defines it, in double precision, one point and
 * one element pair at a time, with no blocking, fusion or reordering.
 * Nodes are in the caller's order; no spatial sorting happens here.
 *
 * Conventions (readings of the paper, all listed in the design notes):
 *  - exterior medium is vacuum: eps_a = mu_a = 1, omega = k_a = k0;
 *    k_i = k0 sqrt(eps_r mu_r) with Im k_i >= 0;
 *  - reference triangle {xi, eta >= 0, xi + eta <= 1}, barycentrics
 *    l0 = 1 - xi - eta, l1 = xi, l2 = eta, local nodes (v0 v1 v2 m01 m12 m20);
 *  - unknown index inside one current's block: 2 * node + alpha;
 *  - the 12 kernel values of one point pair are ordered
 *    c = 4 * op + 2 * alpha + beta, op = 0: K1, 1: K2^eps, 2: K2^mu;
 *  - tangential basis (phys[6]): frame 0 is the printed construction,
 *    N_j t_beta(y) with the interpolated Gram-Schmidt frame; frame 1 attaches
 *    each basis function to its node, N_j(y) P(y) t_beta,j.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------ */
/* quadrature rules                                                    */
/* ------------------------------------------------------------------ */

/* Radon's 7-point degree-5 rule on the reference triangle (area 1/2).   */
void or_rule7(double xi[7], double eta[7], double w[7]) {
    const double s15 = sqrt(15.0);
    const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
    const double wa = (155.0 - s15) / 2400.0, wb = (155.0 + s15) / 2400.0;
    double X[7] = {1.0 / 3.0, a, 1.0 - 2.0 * a, a, b, 1.0 - 2.0 * b, b};
    double Y[7] = {1.0 / 3.0, a, a, 1.0 - 2.0 * a, b, b, 1.0 - 2.0 * b};
    double W[7] = {9.0 / 80.0, wa, wa, wa, wb, wb, wb};
    for (int q = 0; q < 7; ++q) { xi[q] = X[q]; eta[q] = Y[q]; w[q] = W[q]; }
}

/* The 12-point degree-6 symmetric rule on the reference triangle (area
 * 1/2): two three-point orbits (a, a, 1 - 2a) and one six-point orbit
 * (b, c, 1 - b - c).  Its seven parameters solve the seven moment
 * equations of the S3-invariant polynomials e2^i e3^j, 2i + 3j <= 6
 * (Witherden and Vincent's 12-point rule for degree 6, whose points
 * Dunavant also lists); the values were refined by Newton's method on those
 * equations to double precision.  Order: orbit a1, orbit a2, then the six
 * permutations of (b, c, 1 - b - c).                                       */
void or_rule12(double xi[12], double eta[12], double w[12]) {
    const double a[2] = {0.06308901449150309, 0.24928674517091215};
    const double wa[2] = {0.05084490637020728, 0.11678627572637695};
    const double b = 0.053145049844817806, c = 0.3103524510337839;
    const double wb = 0.08285107561837454;
    int q = 0;
    for (int o = 0; o < 2; ++o)
        for (int k = 0; k < 3; ++k) {
            double l[3] = {a[o], a[o], a[o]};
            l[k] = 1.0 - 2.0 * a[o];
            xi[q] = l[1]; eta[q] = l[2]; w[q] = 0.5 * wa[o]; ++q;
        }
    const double v[3] = {b, c, 1.0 - b - c};
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k < 6; ++k) {
        double l[3];
        for (int d = 0; d < 3; ++d) l[perm[k][d]] = v[d];
        xi[q] = l[1]; eta[q] = l[2]; w[q] = 0.5 * wb; ++q;
    }
}

/* n-point Gauss-Legendre rule on [0,1], by Newton iteration on P_n.     */
int or_gauss_legendre01(int n, double *x, double *w) {
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* P2 isoparametric element (Sec. 3.1 and 3.3)                          */
/* ------------------------------------------------------------------ */

/* Shape functions N_k and their (xi, eta) derivatives.                  */
static void p2_shape(double xi, double eta, double N[6], double Nx[6],
                     double Ne[6]) {
    double l0 = 1.0 - xi - eta, l1 = xi, l2 = eta;
    /* d(l0,l1,l2)/dxi = (-1,1,0), d/deta = (-1,0,1) */
    N[0] = l0 * (2 * l0 - 1); N[1] = l1 * (2 * l1 - 1); N[2] = l2 * (2 * l2 - 1);
    N[3] = 4 * l0 * l1;       N[4] = 4 * l1 * l2;       N[5] = 4 * l2 * l0;
    Nx[0] = -(4 * l0 - 1); Nx[1] = 4 * l1 - 1; Nx[2] = 0.0;
    Nx[3] = 4 * (l0 - l1); Nx[4] = 4 * l2;     Nx[5] = -4 * l2;
    Ne[0] = -(4 * l0 - 1); Ne[1] = 0.0;        Ne[2] = 4 * l2 - 1;
    Ne[3] = -4 * l1;       Ne[4] = 4 * l1;     Ne[5] = 4 * (l0 - l2);
}

/* Position and covariant tangents a1 = dx/dxi, a2 = dx/deta.            */
static void p2_geom(const double X[6][3], double xi, double eta, double x[3],
                    double a1[3], double a2[3], double N[6]) {
    double Nx[6], Ne[6];
    p2_shape(xi, eta, N, Nx, Ne);
    for (int d = 0; d < 3; ++d) {
        x[d] = a1[d] = a2[d] = 0.0;
        for (int k = 0; k < 6; ++k) {
            x[d] += N[k] * X[k][d];
            a1[d] += Nx[k] * X[k][d];
            a2[d] += Ne[k] * X[k][d];
        }
    }
}

typedef struct {
    const double *xyz;   /* [n_nodes*3]           */
    const int64_t *tri;  /* [n_tris*6]            */
    int64_t nn, nt;
    double *nrm, *t1, *t2; /* nodal triads [n_nodes*3] each */
} or_mesh;

static void elem_coords(const or_mesh *m, int64_t e, double X[6][3]) {
    for (int k = 0; k < 6; ++k)
        for (int d = 0; d < 3; ++d) X[k][d] = m->xyz[3 * m->tri[6 * e + k] + d];
}

/*
 * Nodal frames.  Metric-weighted normal (Sec. 3.1, eqs. U_contribution and
 * the normalised sum over adjacent elements): each element adjacent to node
 * v contributes U = (a1 x a2)/(g11 g22) with a1, a2 taken along the element
 * edges that leave v (the element is cyclically re-indexed so that v is its
 * local vertex 0).  For a mid-edge node on edge (p -> q) the element is
 * re-indexed so that p is local vertex 0 and q local vertex 1, and a1, a2 are
 * taken at (1/2, 0).  Tangents by the adaptive reference axis (Sec. 3.2,
 * eqs. t1 and t2).
 */
void or_nodal_frames_impl(or_mesh *m) {
    double *acc = (double *)calloc((size_t)m->nn * 3, sizeof(double));
    for (int64_t e = 0; e < m->nt; ++e) {
        double X[6][3];
        elem_coords(m, e, X);
        for (int k = 0; k < 6; ++k) {
            int s = (k < 3) ? k : k - 3;          /* cyclic shift        */
            double R[6][3];
            for (int v = 0; v < 3; ++v)
                for (int d = 0; d < 3; ++d) {
                    R[v][d] = X[(v + s) % 3][d];
                    R[3 + v][d] = X[3 + (v + s) % 3][d];
                }
            double x[3], a1[3], a2[3], N[6], c[3];
            double xi = (k < 3) ? 0.0 : 0.5;
            p2_geom((const double(*)[3])R, xi, 0.0, x, a1, a2, N);
            cross3(a1, a2, c);
            double g = dot3(a1, a1) * dot3(a2, a2);
            int64_t node = m->tri[6 * e + k];
            for (int d = 0; d < 3; ++d) acc[3 * node + d] += c[d] / g;
        }
    }
    for (int64_t v = 0; v < m->nn; ++v) {
        double *n = m->nrm + 3 * v, *t1 = m->t1 + 3 * v, *t2 = m->t2 + 3 * v;
        double l = norm3(acc + 3 * v);
        for (int d = 0; d < 3; ++d) n[d] = acc[3 * v + d] / l;
        double ref[3] = {0, 0, 1};
        if (fabs(n[2]) > 0.9) { ref[0] = 1; ref[2] = 0; }
        cross3(ref, n, t1);
        double lt = norm3(t1);
        for (int d = 0; d < 3; ++d) t1[d] /= lt;
        cross3(n, t1, t2);
    }
    free(acc);
}

/* Everything a kernel evaluation needs at one surface point.           */
typedef struct {
    double x[3], J, n[3], t[2][3], s[2][3], N[6];
    int64_t elem;          /* element the point lies in            */
} or_point;

/*
 * Point data at (xi, eta) of element e: isoparametric position, exact
 * normal n = a1 x a2 / |a1 x a2|, interpolated nodal tangents projected on
 * the tangent plane and Gram-Schmidt orthonormalised (Sec. 3.3), and the
 * rotated test vectors s_alpha = t_alpha x n (Sec. 4.1).
 */
static void point_data(const or_mesh *m, int64_t e, double xi, double eta,
                       or_point *P) {
    double X[6][3], a1[3], a2[3], c[3];
    elem_coords(m, e, X);
    P->elem = e;
    p2_geom((const double(*)[3])X, xi, eta, P->x, a1, a2, P->N);
    cross3(a1, a2, c);
    P->J = norm3(c);
    for (int d = 0; d < 3; ++d) P->n[d] = c[d] / P->J;
    double tt[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int k = 0; k < 6; ++k) {
        int64_t node = m->tri[6 * e + k];
        for (int d = 0; d < 3; ++d) {
            tt[0][d] += P->N[k] * m->t1[3 * node + d];
            tt[1][d] += P->N[k] * m->t2[3 * node + d];
        }
    }
    double p1[3], p2[3];
    double d1 = dot3(P->n, tt[0]), d2 = dot3(P->n, tt[1]);
    for (int d = 0; d < 3; ++d) {
        p1[d] = tt[0][d] - d1 * P->n[d];
        p2[d] = tt[1][d] - d2 * P->n[d];
    }
    double l1 = norm3(p1);
    for (int d = 0; d < 3; ++d) P->t[0][d] = p1[d] / l1;
    double pr = dot3(P->t[0], p2), u[3];
    for (int d = 0; d < 3; ++d) u[d] = p2[d] - pr * P->t[0][d];
    double l2 = norm3(u);
    for (int d = 0; d < 3; ++d) P->t[1][d] = u[d] / l2;
    cross3(P->t[0], P->n, P->s[0]);
    cross3(P->t[1], P->n, P->s[1]);
}

/* ------------------------------------------------------------------ */
/* kernels (Sec. 2.3, 4.1, 4.2)                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    cplx ka, ki;           /* wavenumbers                         */
    cplx eps_a, eps_i, mu_a, mu_i;
    double omega;
    int nss;               /* Gauss points per SSQ dimension       */
    int mode;              /* 0 hybrid, 1 closed form, 2 series    */
    int variant;           /* 0: 7-point regular rule, Sauter-Schwab on the
                              full kernels, 16-term series;
                              1: the paper's variant: 12-point rule, Sauter-
                              Schwab on the singular parts only, the
                              remainder by the 12-point rule, series
                              truncated after n = 6                    */
    int nterms;            /* highest Taylor term n of the series  */
    int frame;             /* tangential basis: 0 the interpolated
                              Gram-Schmidt frame, N_j t_beta(y) (Sec. 3.3,
                              Sec. 4.1); 1 node-attached tangents,
                              N_j(y) P(y) t_beta,j with P(y) = I - n n^T
                              the tangent-plane projector at y          */
} or_phys;

#define OR_SERIES_RHO 0.5
#define OR_SERIES_TERMS 16

/*
 * Scalar parts of the kernel differences at distance R:
 *   D0 = k_a^2 phi_a - k_i^2 phi_i                       (eq. kappa1_alphabeta)
 *   H_diff = df RR^T - dg I,  df = f_ka - f_ki, dg = g_ka - g_ki  (eq. Hdiff_exact)
 *   grad_x Phi_chi = G_chi Rhat, G_chi = chi_a phi'_a - chi_i phi'_i (Sec. 4.2)
 * For max|k| R < 1/2 the Taylor series of Sec. 2.3 (eq. Hdiff_infinite and
 * the same expansion applied to phi and grad phi) is summed to n = 16, so
 * that the R^-3, R^-2 and R^-1 parts cancel exactly instead of numerically.
 */
static void kernel_scalars(const or_phys *ph, double R, cplx *D0, cplx *df,
                           cplx *dg, cplx *Ge, cplx *Gm) {
    double rho = fmax(cabs(ph->ka), cabs(ph->ki)) * R;
    int series = (ph->mode == 2) || (ph->mode == 0 && rho < OR_SERIES_RHO);
    if (!series) {
        cplx k[2] = {ph->ka, ph->ki};
        cplx phi[2], f[2], g[2], dphi[2];
        for (int s = 0; s < 2; ++s) {
            cplx ikR = I * k[s] * R;
            cplx e = cexp(ikR);
            phi[s] = e / (4 * OR_PI * R);
            f[s] = e / (4 * OR_PI * R * R * R) * (3.0 - 3.0 * ikR - k[s] * k[s] * R * R);
            g[s] = e / (4 * OR_PI * R * R * R) * (1.0 - ikR);
            dphi[s] = e * (ikR - 1.0) / (4 * OR_PI * R * R);
        }
        *D0 = ph->ka * ph->ka * phi[0] - ph->ki * ph->ki * phi[1];
        *df = f[0] - f[1];
        *dg = g[0] - g[1];
        *Ge = ph->eps_a * dphi[0] - ph->eps_i * dphi[1];
        *Gm = ph->mu_a * dphi[0] - ph->mu_i * dphi[1];
        return;
    }
    /* c_n(k) = (i k)^n / n! */
    cplx ca = 1.0, ci = 1.0;
    cplx sD = 0, sf = 0, sg = 0, se = 0, sm = 0;
    double Rp = 1.0 / R;            /* R^(n-1) at n = 0 */
    for (int n = 0; n <= ph->nterms; ++n) {
        if (n > 0) { ca *= I * ph->ka / n; ci *= I * ph->ki / n; }
        double Rn1 = Rp;            /* R^(n-1) */
        double Rn2 = Rp / R;        /* R^(n-2) */
        double Rn3 = Rp / (R * R);  /* R^(n-3) */
        sD += (ph->ka * ph->ka * ca - ph->ki * ph->ki * ci) * Rn1;
        if (n >= 2) {
            cplx d = ca - ci;
            sf += d * (double)((n - 1) * (n - 3)) * Rn3;
            sg -= d * (double)(n - 1) * Rn3;
        }
        se += (ph->eps_a * ca - ph->eps_i * ci) * (double)(n - 1) * Rn2;
        sm += (ph->mu_a * ca - ph->mu_i * ci) * (double)(n - 1) * Rn2;
        Rp *= R;
    }
    *D0 = sD / (4 * OR_PI); *df = sf / (4 * OR_PI); *dg = sg / (4 * OR_PI);
    *Ge = se / (4 * OR_PI); *Gm = sm / (4 * OR_PI);
}

/*
 * Singular parts of the scalars (the paper's kappa^s, eqs. kappa_S and the
 * singular part of grad Phi_chi): the terms of negative order in R of the
 * expansions, D0: n = 0, df and dg: n = 2, G_chi: n = 0.
 *   D0^s = (k_a^2 - k_i^2) / (4 pi R),  df^s = dg^s = (k_a^2 - k_i^2) / (8 pi R),
 *   G_chi^s = -(chi_a - chi_i) / (4 pi R^2)
 */
static void kernel_scalars_sing(const or_phys *ph, double R, cplx *D0, cplx *df,
                                cplx *dg, cplx *Ge, cplx *Gm) {
    cplx dk2 = ph->ka * ph->ka - ph->ki * ph->ki;
    *D0 = dk2 / (4 * OR_PI * R);
    *df = dk2 / (8 * OR_PI * R);
    *dg = *df;
    *Ge = -(ph->eps_a - ph->eps_i) / (4 * OR_PI * R * R);
    *Gm = -(ph->mu_a - ph->mu_i) / (4 * OR_PI * R * R);
}

/*
 * Regular remainders kernel - kernel^s.  For max|k| R < 1/2 (and at R = 0)
 * the expansions without their singular terms, truncated after n = nterms;
 * only non-negative powers of R remain, so R = 0 is an ordinary point.
 * Otherwise the closed forms minus the singular parts.
 */
static void kernel_scalars_rem(const or_phys *ph, double R, cplx *D0, cplx *df,
                               cplx *dg, cplx *Ge, cplx *Gm) {
    double rho = fmax(cabs(ph->ka), cabs(ph->ki)) * R;
    if (R > 0 && rho >= OR_SERIES_RHO) {
        or_phys q = *ph;
        q.mode = 1;
        cplx s[5];
        kernel_scalars(&q, R, D0, df, dg, Ge, Gm);
        kernel_scalars_sing(ph, R, &s[0], &s[1], &s[2], &s[3], &s[4]);
        *D0 -= s[0]; *df -= s[1]; *dg -= s[2]; *Ge -= s[3]; *Gm -= s[4];
        return;
    }
    cplx ca = 1.0, ci = 1.0;
    cplx sD = 0, sf = 0, sg = 0, se = 0, sm = 0;
    for (int n = 0; n <= ph->nterms; ++n) {
        if (n > 0) { ca *= I * ph->ka / n; ci *= I * ph->ki / n; }
        if (n >= 1) sD += (ph->ka * ph->ka * ca - ph->ki * ph->ki * ci) * pow(R, n - 1);
        if (n >= 3) {
            cplx d = ca - ci;
            if (n >= 4) sf += d * (double)((n - 1) * (n - 3)) * pow(R, n - 3);
            sg -= d * (double)(n - 1) * pow(R, n - 3);
        }
        if (n >= 2) {
            se += (ph->eps_a * ca - ph->eps_i * ci) * (double)(n - 1) * pow(R, n - 2);
            sm += (ph->mu_a * ca - ph->mu_i * ci) * (double)(n - 1) * pow(R, n - 2);
        }
    }
    *D0 = sD / (4 * OR_PI); *df = sf / (4 * OR_PI); *dg = sg / (4 * OR_PI);
    *Ge = se / (4 * OR_PI); *Gm = sm / (4 * OR_PI);
}

/*
 * The twelve scalar kernels at a test point X and a trial point Y from the
 * scalars and the unit vector Rh = (x - y)/|x - y|:
 *  kappa1_ab = D0 (s_a . t_b) + s_a . H_diff . t_b          (eq. kappa1_alphabeta)
 *  kappa2_ab = (t_a . t_b)(n . grad Phi) - (t_a . grad Phi)(n . t_b)
 *                                                          (eq. kappa2_alpha_beta)
 * with H_diff = df Rh Rh^T - dg I built as a full 3x3 matrix and grad Phi
 * = G Rh as a vector.
 */
static void kappa_combine(const or_point *X, const or_point *Y, const double Rh[3],
                          cplx D0, cplx df, cplx dg, cplx Ge, cplx Gm, cplx out[12]) {
    cplx H[3][3], gE[3], gM[3];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) H[a][b] = df * Rh[a] * Rh[b] - (a == b ? dg : 0.0);
        gE[a] = Ge * Rh[a];
        gM[a] = Gm * Rh[a];
    }
    for (int al = 0; al < 2; ++al)
        for (int be = 0; be < 2; ++be) {
            const double *sa = X->s[al], *ta = X->t[al], *tb = Y->t[be], *n = X->n;
            cplx Ht[3];
            for (int a = 0; a < 3; ++a)
                Ht[a] = H[a][0] * tb[0] + H[a][1] * tb[1] + H[a][2] * tb[2];
            cplx k1 = D0 * dot3(sa, tb) + (sa[0] * Ht[0] + sa[1] * Ht[1] + sa[2] * Ht[2]);
            cplx nGe = n[0] * gE[0] + n[1] * gE[1] + n[2] * gE[2];
            cplx tGe = ta[0] * gE[0] + ta[1] * gE[1] + ta[2] * gE[2];
            cplx nGm = n[0] * gM[0] + n[1] * gM[1] + n[2] * gM[2];
            cplx tGm = ta[0] * gM[0] + ta[1] * gM[1] + ta[2] * gM[2];
            double tt = dot3(ta, tb), nt = dot3(n, tb);
            out[0 + 2 * al + be] = k1;
            out[4 + 2 * al + be] = tt * nGe - tGe * nt;
            out[8 + 2 * al + be] = tt * nGm - tGm * nt;
        }
}

/* which = 0: the full kernels; 1: their singular parts; 2: the remainders.
 * At coincident points (R = 0, only the remainders can be asked for there)
 * the direction Rh is undefined; it multiplies df, which vanishes, and
 * G_chi, whose contribution is taken as its average over directions, 0.   */
static void kappa_eval(const or_phys *ph, const or_point *X, const or_point *Y,
                       int which, cplx out[12]) {
    double Rv[3], R, Rh[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) Rv[d] = X->x[d] - Y->x[d];
    R = norm3(Rv);
    if (R > 0)
        for (int d = 0; d < 3; ++d) Rh[d] = Rv[d] / R;
    cplx D0, df, dg, Ge, Gm;
    if (which == 0) kernel_scalars(ph, R, &D0, &df, &dg, &Ge, &Gm);
    else if (which == 1) kernel_scalars_sing(ph, R, &D0, &df, &dg, &Ge, &Gm);
    else kernel_scalars_rem(ph, R, &D0, &df, &dg, &Ge, &Gm);
    kappa_combine(X, Y, Rh, D0, df, dg, Ge, Gm, out);
}

/* ------------------------------------------------------------------ */
/* element-pair integration                                             */
/* ------------------------------------------------------------------ */

/* Pair class by shared vertex nodes (Sec. 4.2, the three singular classes).
 * 3: coincident, 2: common edge, 1: common vertex, 0: regular.           */
static int pair_class(const or_mesh *m, int64_t e, int64_t f, int sh_e[3],
                      int sh_f[3]) {
    int n = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (m->tri[6 * e + a] == m->tri[6 * f + b]) {
                sh_e[n] = a; sh_f[n] = b; ++n;
            }
    return n;
}

/*
 * Accumulate the point pair (X, Y) into blk[i][j][c]; `which` selects the
 * full kernels, their singular parts or the remainders.
 * frame 0: blk[i][j][c] += w N_i(x) N_j(y) kappa_c(x,y).
 * frame 1: the basis vector of node k at a point is P t_beta,k, whose
 * components in the point's orthonormal frame are R_k[beta][gamma] =
 * t_beta,k . t_gamma (the normal part drops out); the rotated test vector
 * t_alpha,i x n has the same components on (s_1, s_2).  The kernels are
 * linear in the test and in the trial vector, so
 *   blk[i][j][op,a,b] += w N_i N_j sum_{g,d} R_i[a][g] kappa_{op,g,d} R_j[b][d].
 */
static void accumulate_k(const or_mesh *m, const or_phys *ph, const or_point *X,
                         const or_point *Y, double w, int which, cplx blk[6][6][12]) {
    cplx k[12];
    kappa_eval(ph, X, Y, which, k);
    double ww = w * X->J * Y->J;
    if (ph->frame == 0) {
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double s = ww * X->N[i] * Y->N[j];
                for (int c = 0; c < 12; ++c) blk[i][j][c] += s * k[c];
            }
        return;
    }
    double RX[6][2][2], RY[6][2][2];
    for (int q = 0; q < 6; ++q) {
        int64_t vx = m->tri[6 * X->elem + q], vy = m->tri[6 * Y->elem + q];
        const double *tx[2] = {m->t1 + 3 * vx, m->t2 + 3 * vx};
        const double *ty[2] = {m->t1 + 3 * vy, m->t2 + 3 * vy};
        for (int a = 0; a < 2; ++a)
            for (int g = 0; g < 2; ++g) {
                RX[q][a][g] = dot3(tx[a], X->t[g]);
                RY[q][a][g] = dot3(ty[a], Y->t[g]);
            }
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = ww * X->N[i] * Y->N[j];
            for (int op = 0; op < 3; ++op)
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        cplx acc = 0;
                        for (int g = 0; g < 2; ++g)
                            for (int d = 0; d < 2; ++d)
                                acc += RX[i][a][g] * k[4 * op + 2 * g + d] * RY[j][b][d];
                        blk[i][j][4 * op + 2 * a + b] += s * acc;
                    }
        }
}

/*
 * Sauter-Schwab maps (the three singular classes of Sec. 4.2).  Reference
 * triangle Th = {0 <= t <= s <= 1}; common edge = {t = 0} in both
 * triangles with the same s, common vertex = (0,0).  Each map takes
 * (xi, e1, e2, e3) in [0,1]^4 to (s1,t1) in the test and (s2,t2) in the
 * trial triangle and returns its Jacobian.
 */
static double ss_map(int cls, int r, double x, double e1, double e2, double e3,
                     double *s1, double *t1, double *s2, double *t2) {
    if (cls == 3) {
        double w = x * x * x * e1 * e1 * e2;
        switch (r) {
        case 0: *s1 = x; *t1 = x * (1 - e1 + e1 * e2);
                *s2 = x * (1 - e1 * e2 * e3); *t2 = x * (1 - e1); break;
        case 1: *s1 = x * (1 - e1 * e2 * e3); *t1 = x * (1 - e1);
                *s2 = x; *t2 = x * (1 - e1 + e1 * e2); break;
        case 2: *s1 = x; *t1 = x * e1 * (1 - e2 + e2 * e3);
                *s2 = x * (1 - e1 * e2); *t2 = x * e1 * (1 - e2); break;
        case 3: *s1 = x * (1 - e1 * e2); *t1 = x * e1 * (1 - e2);
                *s2 = x; *t2 = x * e1 * (1 - e2 + e2 * e3); break;
        case 4: *s1 = x * (1 - e1 * e2 * e3); *t1 = x * e1 * (1 - e2 * e3);
                *s2 = x; *t2 = x * e1 * (1 - e2); break;
        default: *s1 = x; *t1 = x * e1 * (1 - e2);
                 *s2 = x * (1 - e1 * e2 * e3); *t2 = x * e1 * (1 - e2 * e3); break;
        }
        return w;
    }
    if (cls == 2) {
        switch (r) {
        case 0: *s1 = x; *t1 = x * e1 * e3;
                *s2 = x * (1 - e1 * e2); *t2 = x * e1 * (1 - e2);
                return x * x * x * e1 * e1;
        case 1: *s1 = x; *t1 = x * e1;
                *s2 = x * (1 - e1 * e2 * e3); *t2 = x * e1 * e2 * (1 - e3);
                return x * x * x * e1 * e1 * e2;
        case 2: *s1 = x * (1 - e1 * e2); *t1 = x * e1 * (1 - e2);
                *s2 = x; *t2 = x * e1 * e2 * e3;
                return x * x * x * e1 * e1 * e2;
        case 3: *s1 = x * (1 - e1 * e2 * e3); *t1 = x * e1 * e2 * (1 - e3);
                *s2 = x; *t2 = x * e1;
                return x * x * x * e1 * e1 * e2;
        default: *s1 = x * (1 - e1 * e2 * e3); *t1 = x * e1 * (1 - e2 * e3);
                 *s2 = x; *t2 = x * e1 * e2;
                 return x * x * x * e1 * e1 * e2;
        }
    }
    /* cls == 1 */
    if (r == 0) { *s1 = x; *t1 = x * e1; *s2 = x * e2; *t2 = x * e2 * e3; }
    else        { *s1 = x * e2; *t1 = x * e2 * e3; *s2 = x; *t2 = x * e1; }
    return x * x * x * e2;
}

static int ss_regions(int cls) { return cls == 3 ? 6 : (cls == 2 ? 5 : 2); }

/* (s,t) in Th -> (xi,eta) of the original element, given the order of its
 * local vertices in the re-indexed element (perm[k'] = original vertex).  */
static void ss_to_elem(const int perm[3], double s, double t, double *xi,
                       double *eta) {
    double lp[3] = {1.0 - s, s - t, t}, l[3];
    for (int k = 0; k < 3; ++k) l[perm[k]] = lp[k];
    *xi = l[1]; *eta = l[2];
}

/* Re-index both elements so that the shared vertices come first, in the
 * same order, in both.                                                   */
static void ss_perms(int cls, const int sh_e[3], const int sh_f[3], int pe[3],
                     int pf[3]) {
    if (cls == 3) { for (int k = 0; k < 3; ++k) pe[k] = pf[k] = k; return; }
    if (cls == 1) {
        for (int k = 0; k < 3; ++k) { pe[k] = (sh_e[0] + k) % 3; pf[k] = (sh_f[0] + k) % 3; }
        return;
    }
    /* common edge: order (A, B) so that A -> B is an edge of e in its own
     * counter-clockwise order */
    int a = 0, b = 1;
    if ((sh_e[0] + 1) % 3 != sh_e[1]) { a = 1; b = 0; }
    pe[0] = sh_e[a]; pe[1] = sh_e[b]; pe[2] = 3 - sh_e[a] - sh_e[b];
    pf[0] = sh_f[a]; pf[1] = sh_f[b]; pf[2] = 3 - sh_f[a] - sh_f[b];
}

/* 6x6x12 block of element pair (e test, f trial).                       */
static void pair_block(const or_mesh *m, const or_phys *ph, int64_t e,
                       int64_t f, cplx blk[6][6][12]) {
    memset(blk, 0, sizeof(cplx) * 6 * 6 * 12);
    int sh_e[3], sh_f[3];
    int cls = pair_class(m, e, f, sh_e, sh_f);
    if (ph->variant == 1) {
        /* 12-point rule: every regular pair with the closed-form kernels
         * (the truncated series is for singular pairs only), every singular
         * pair for the remainder kernel - kernel^s                          */
        double xi[12], eta[12], w[12];
        or_rule12(xi, eta, w);
        or_point X[12], Y[12];
        for (int q = 0; q < 12; ++q) {
            point_data(m, e, xi[q], eta[q], &X[q]);
            point_data(m, f, xi[q], eta[q], &Y[q]);
        }
        or_phys q = *ph;
        if (q.mode == 0) q.mode = 1;
        for (int p = 0; p < 12; ++p)
            for (int r = 0; r < 12; ++r)
                accumulate_k(m, &q, &X[p], &Y[r], w[p] * w[r], cls == 0 ? 0 : 2, blk);
        if (cls == 0) return;
    } else if (cls == 0) {
        double xi[7], eta[7], w[7];
        or_rule7(xi, eta, w);
        or_point X[7], Y[7];
        for (int q = 0; q < 7; ++q) {
            point_data(m, e, xi[q], eta[q], &X[q]);
            point_data(m, f, xi[q], eta[q], &Y[q]);
        }
        for (int p = 0; p < 7; ++p)
            for (int q = 0; q < 7; ++q) accumulate_k(m, ph, &X[p], &Y[q], w[p] * w[q], 0, blk);
        return;
    }
    int pe[3], pf[3];
    ss_perms(cls, sh_e, sh_f, pe, pf);
    int n = ph->nss;
    double g[64], gw[64];
    or_gauss_legendre01(n, g, gw);
    for (int r = 0; r < ss_regions(cls); ++r)
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                for (int c = 0; c < n; ++c)
                    for (int d = 0; d < n; ++d) {
                        double s1, t1, s2, t2, x1, y1, x2, y2;
                        double jac = ss_map(cls, r, g[a], g[b], g[c], g[d], &s1, &t1, &s2, &t2);
                        ss_to_elem(pe, s1, t1, &x1, &y1);
                        ss_to_elem(pf, s2, t2, &x2, &y2);
                        or_point X, Y;
                        point_data(m, e, x1, y1, &X);
                        point_data(m, f, x2, y2, &Y);
                        accumulate_k(m, ph, &X, &Y, jac * gw[a] * gw[b] * gw[c] * gw[d],
                                     ph->variant == 1 ? 1 : 0, blk);
                    }
}

/* ------------------------------------------------------------------ */
/* exported entry points (ctypes)                                       */
/* ------------------------------------------------------------------ */

/* phys[] = {k0, Re eps_r, Im eps_r, Re mu_r, Im mu_r, variant, frame}    */
static or_phys make_phys(const double *phys, int nss, int mode) {
    or_phys ph;
    cplx er = phys[1] + I * phys[2], mr = phys[3] + I * phys[4];
    ph.omega = phys[0];
    ph.eps_a = 1.0; ph.mu_a = 1.0; ph.eps_i = er; ph.mu_i = mr;
    ph.ka = phys[0];
    ph.ki = phys[0] * csqrt(er * mr);
    if (cimag(ph.ki) < 0) ph.ki = -ph.ki;
    ph.nss = nss; ph.mode = mode;
    ph.variant = (int)phys[5];
    ph.nterms = ph.variant == 1 ? 6 : OR_SERIES_TERMS;
    ph.frame = (int)phys[6];
    return ph;
}

static int mesh_init(or_mesh *m, const double *xyz, int64_t nn,
                     const int64_t *tri, int64_t nt) {
    m->xyz = xyz; m->tri = tri; m->nn = nn; m->nt = nt;
    m->nrm = (double *)malloc(sizeof(double) * 3 * nn);
    m->t1 = (double *)malloc(sizeof(double) * 3 * nn);
    m->t2 = (double *)malloc(sizeof(double) * 3 * nn);
    if (!m->nrm || !m->t1 || !m->t2) return -2;
    or_nodal_frames_impl(m);
    return 0;
}
static void mesh_free(or_mesh *m) { free(m->nrm); free(m->t1); free(m->t2); }

/* nodal triads: out[n_nodes*9] = (n, t1, t2) per node                    */
int or_nodal_frames(const double *xyz, int64_t nn, const int64_t *tri,
                    int64_t nt, double *out) {
    or_mesh m;
    if (mesh_init(&m, xyz, nn, tri, nt)) return -2;
    for (int64_t v = 0; v < nn; ++v)
        for (int d = 0; d < 3; ++d) {
            out[9 * v + d] = m.nrm[3 * v + d];
            out[9 * v + 3 + d] = m.t1[3 * v + d];
            out[9 * v + 6 + d] = m.t2[3 * v + d];
        }
    mesh_free(&m);
    return 0;
}

/* point data for npt (element, xi, eta) triples; out[npt*25] per point:
 * x(3) J(1) n(3) t1(3) t2(3) s1(3) s2(3) N(6)                            */
#define OR_PT_STRIDE 25
int or_point_data(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt,
                  int64_t npt, const int64_t *elem, const double *xi,
                  const double *eta, double *out) {
    or_mesh m;
    if (mesh_init(&m, xyz, nn, tri, nt)) return -2;
    for (int64_t p = 0; p < npt; ++p) {
        or_point P;
        point_data(&m, elem[p], xi[p], eta[p], &P);
        double *o = out + OR_PT_STRIDE * p;
        memcpy(o, P.x, 3 * sizeof(double)); o[3] = P.J;
        memcpy(o + 4, P.n, 3 * sizeof(double));
        memcpy(o + 7, P.t[0], 3 * sizeof(double));
        memcpy(o + 10, P.t[1], 3 * sizeof(double));
        memcpy(o + 13, P.s[0], 3 * sizeof(double));
        memcpy(o + 16, P.s[1], 3 * sizeof(double));
        memcpy(o + 19, P.N, 6 * sizeof(double));
    }
    mesh_free(&m);
    return 0;
}

/* kernel scalars at distances R[n]; out[n*10] = D0, df, dg, Ge, Gm (re,im);
 * mode 0 hybrid, 1 closed form, 2 series, 3 singular parts, 4 remainders */
int or_kernel_scalars(const double *phys, int mode, int64_t n, const double *R,
                      double *out) {
    or_phys ph = make_phys(phys, 4, mode);
    for (int64_t i = 0; i < n; ++i) {
        cplx v[5];
        if (mode == 3) kernel_scalars_sing(&ph, R[i], &v[0], &v[1], &v[2], &v[3], &v[4]);
        else if (mode == 4) kernel_scalars_rem(&ph, R[i], &v[0], &v[1], &v[2], &v[3], &v[4]);
        else kernel_scalars(&ph, R[i], &v[0], &v[1], &v[2], &v[3], &v[4]);
        for (int k = 0; k < 5; ++k) { out[10 * i + 2 * k] = creal(v[k]); out[10 * i + 2 * k + 1] = cimag(v[k]); }
    }
    return 0;
}

/* one 6x6x12 element-pair block (complex, interleaved re/im)             */
int or_pair_block(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt,
                  const double *phys, int nss, int mode, int64_t e, int64_t f,
                  double *out) {
    or_mesh m;
    if (mesh_init(&m, xyz, nn, tri, nt)) return -2;
    or_phys ph = make_phys(phys, nss, mode);
    cplx blk[6][6][12];
    pair_block(&m, &ph, e, f, blk);
    memcpy(out, blk, sizeof(blk));
    mesh_free(&m);
    return 0;
}

/* Sauter-Schwab rule on Th x Th for a flat integrand test: evaluates
 * sum_r sum_gauss jac * f at the (s1,t1,s2,t2) points.  Writes npoints*5
 * doubles (s1,t1,s2,t2,weight); returns the number of points.            */
int64_t or_ss_rule(int cls, int n, double *out) {
    double g[64], gw[64];
    if (or_gauss_legendre01(n, g, gw)) return -1;
    int64_t k = 0;
    for (int r = 0; r < ss_regions(cls); ++r)
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                for (int c = 0; c < n; ++c)
                    for (int d = 0; d < n; ++d) {
                        double s1, t1, s2, t2;
                        double jac = ss_map(cls, r, g[a], g[b], g[c], g[d], &s1, &t1, &s2, &t2);
                        if (out) {
                            double *o = out + 5 * k;
                            o[0] = s1; o[1] = t1; o[2] = s2; o[3] = t2;
                            o[4] = jac * gw[a] * gw[b] * gw[c] * gw[d];
                        }
                        ++k;
                    }
    return k;
}

/*
 * Dense operator blocks K1, K2^eps, K2^mu, each (2 nn) x (2 nn), row-major,
 * complex interleaved, entry [2 i + alpha][2 j + beta] = sum over element
 * pairs (e contains i, f contains j) of the pair block
 * (eqs. K1_matrix_entry and K2_matrix_entry).  OpenMP over test elements;
 * every thread adds the finished rows of its element under a lock.
 */
int or_fill(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt,
            const double *phys, int nss, int nthreads, double *K1d, double *K2ed,
            double *K2md) {
    or_mesh m;
    if (mesh_init(&m, xyz, nn, tri, nt)) return -2;
    or_phys ph = make_phys(phys, nss, 0);
    int64_t n2 = 2 * nn;
    cplx *K[3] = {(cplx *)K1d, (cplx *)K2ed, (cplx *)K2md};
    for (int o = 0; o < 3; ++o) memset(K[o], 0, sizeof(cplx) * n2 * n2);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        /* rows of the 6 nodes of one test element, all columns, 3 ops    */
        cplx *rows = (cplx *)malloc(sizeof(cplx) * 3 * 12 * n2);
#pragma omp for schedule(dynamic, 1)
        for (int64_t e = 0; e < nt; ++e) {
            memset(rows, 0, sizeof(cplx) * 3 * 12 * n2);
            for (int64_t f = 0; f < nt; ++f) {
                cplx blk[6][6][12];
                pair_block(&m, &ph, e, f, blk);
                for (int i = 0; i < 6; ++i)
                    for (int j = 0; j < 6; ++j) {
                        int64_t J = m.tri[6 * f + j];
                        for (int o = 0; o < 3; ++o)
                            for (int al = 0; al < 2; ++al)
                                for (int be = 0; be < 2; ++be)
                                    rows[(o * 12 + 2 * i + al) * n2 + 2 * J + be] +=
                                        blk[i][j][4 * o + 2 * al + be];
                    }
            }
#pragma omp critical(or_fill_add)
            {
                for (int i = 0; i < 6; ++i) {
                    int64_t Ii = m.tri[6 * e + i];
                    for (int o = 0; o < 3; ++o)
                        for (int al = 0; al < 2; ++al) {
                            cplx *dst = K[o] + (2 * Ii + al) * n2;
                            const cplx *src = rows + (o * 12 + 2 * i + al) * n2;
                            for (int64_t c = 0; c < n2; ++c) dst[c] += src[c];
                        }
                }
            }
        }
        free(rows);
    }
    mesh_free(&m);
    return 0;
}

/*
 * Selected node-pair entries, one at a time: for each (inode[s], jnode[s])
 * the 12 complex values [op][alpha][beta] summed over all element pairs
 * (e contains inode, f contains jnode).  out[s*24] interleaved re/im.
 */
int or_entries(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt,
               const double *phys, int nss, int nthreads, int64_t ns,
               const int64_t *inode, const int64_t *jnode, double *out) {
    or_mesh m;
    if (mesh_init(&m, xyz, nn, tri, nt)) return -2;
    or_phys ph = make_phys(phys, nss, 0);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ns; ++s) {
        cplx acc[12] = {0};
        int64_t Ei[64], Ej[64];
        int li[64], lj[64], ni = 0, nj = 0;
        for (int64_t e = 0; e < nt; ++e)
            for (int k = 0; k < 6; ++k) {
                if (tri[6 * e + k] == inode[s] && ni < 64) { Ei[ni] = e; li[ni++] = k; }
                if (tri[6 * e + k] == jnode[s] && nj < 64) { Ej[nj] = e; lj[nj++] = k; }
            }
        for (int a = 0; a < ni; ++a)
            for (int b = 0; b < nj; ++b) {
                cplx blk[6][6][12];
                pair_block(&m, &ph, Ei[a], Ej[b], blk);
                for (int c = 0; c < 12; ++c) acc[c] += blk[li[a]][lj[b]][c];
            }
        for (int c = 0; c < 12; ++c) { out[24 * s + 2 * c] = creal(acc[c]); out[24 * s + 2 * c + 1] = cimag(acc[c]); }
    }
    mesh_free(&m);
    return 0;
}
