/* The oracle's C core under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Built with gcc together with oracle/mbem_oracle.c (without OpenMP, so one
 * thread) by tests/test_sanitizers.py.  Reads a P2 mesh and the physical
 * parameters (int64 nn, int64 nt, double xyz[3 nn], int64 tri[6 nt],
 * double phys[7]), calls every entry point of the core once (quadrature
 * rules, Sauter-Schwab rules of the three classes, nodal frames, point
 * data, kernel scalars in every mode, one pair block, the dense fill and a
 * few node-pair entries), and writes the three dense blocks
 * (3 (2 nn)^2 complex) followed by the nodal frames (9 nn doubles) to the
 * output file.  Exit status 0 = every call returned success.            */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_rule7(double xi[7], double eta[7], double w[7]);
void or_rule12(double xi[12], double eta[12], double w[12]);
int or_gauss_legendre01(int n, double *x, double *w);
int or_nodal_frames(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt, double *out);
int or_point_data(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt, int64_t npt,
                  const int64_t *elem, const double *xi, const double *eta, double *out);
int or_kernel_scalars(const double *phys, int mode, int64_t n, const double *R, double *out);
int or_pair_block(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt, const double *phys,
                  int nss, int mode, int64_t e, int64_t f, double *out);
int64_t or_ss_rule(int cls, int n, double *out);
int or_fill(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt, const double *phys, int nss,
            int nthreads, double *K1d, double *K2ed, double *K2md);
int or_entries(const double *xyz, int64_t nn, const int64_t *tri, int64_t nt, const double *phys, int nss,
               int nthreads, int64_t ns, const int64_t *inode, const int64_t *jnode, double *out);

static int fail(const char *what) {
    fprintf(stderr, "oracle_driver: %s\n", what);
    return 1;
}

int main(int argc, char **argv) {
    if (argc != 3) return fail("usage: oracle_driver in.bin out.bin");
    FILE *f = fopen(argv[1], "rb");
    if (!f) return fail("cannot open input");
    int64_t nn = 0, nt = 0;
    if (fread(&nn, 8, 1, f) != 1 || fread(&nt, 8, 1, f) != 1 || nn < 4 || nt < 4) return fail("header");
    double *xyz = malloc(sizeof(double) * 3 * nn);
    int64_t *tri = malloc(sizeof(int64_t) * 6 * nt);
    double phys[7];
    if (fread(xyz, 8, 3 * nn, f) != (size_t)(3 * nn) || fread(tri, 8, 6 * nt, f) != (size_t)(6 * nt) ||
        fread(phys, 8, 7, f) != 7)
        return fail("body");
    fclose(f);

    double xi[12], eta[12], w[12], gx[16], gw[16];
    or_rule7(xi, eta, w);
    or_rule12(xi, eta, w);
    if (or_gauss_legendre01(16, gx, gw)) return fail("gauss_legendre01");
    for (int cls = 1; cls <= 3; ++cls) {   /* common vertex, common edge, coincident */
        double *pts = malloc(sizeof(double) * 5 * 6 * 4 * 4 * 4 * 4);
        if (or_ss_rule(cls, 4, pts) <= 0) return fail("ss_rule");
        free(pts);
    }
    double *frames = malloc(sizeof(double) * 9 * nn);
    if (or_nodal_frames(xyz, nn, tri, nt, frames)) return fail("nodal_frames");
    {
        int64_t elem[3] = {0, nt / 2, nt - 1};
        double pxi[3] = {0.2, 0.0, 0.5}, peta[3] = {0.3, 1.0, 0.5}, out[75];
        if (or_point_data(xyz, nn, tri, nt, 3, elem, pxi, peta, out)) return fail("point_data");
    }
    {
        double R[5] = {0.0, 1e-9, 1e-3, 0.3, 2.5}, out[50];
        for (int mode = 0; mode <= 4; ++mode)
            if (or_kernel_scalars(phys, mode, 5, R, out)) return fail("kernel_scalars");
    }
    {
        double *blk = malloc(sizeof(double) * 2 * 6 * 6 * 12);
        if (or_pair_block(xyz, nn, tri, nt, phys, 3, 0, 0, 0, blk) ||
            or_pair_block(xyz, nn, tri, nt, phys, 3, 0, 0, nt - 1, blk))
            return fail("pair_block");
        free(blk);
    }
    const int64_t n2 = 2 * nn;
    double *K = malloc(sizeof(double) * 3 * 2 * n2 * n2);
    if (or_fill(xyz, nn, tri, nt, phys, 3, 1, K, K + 2 * n2 * n2, K + 4 * n2 * n2)) return fail("fill");
    {
        int64_t in[4] = {0, 0, nn - 1, nn / 2}, jn[4] = {0, 1, 0, nn - 1};
        double out[96];
        if (or_entries(xyz, nn, tri, nt, phys, 3, 1, 4, in, jn, out)) return fail("entries");
    }

    FILE *o = fopen(argv[2], "wb");
    if (!o) return fail("cannot open output");
    fwrite(K, sizeof(double), 3 * 2 * n2 * n2, o);
    fwrite(frames, sizeof(double), 9 * nn, o);
    fclose(o);
    free(K);
    free(frames);
    free(xyz);
    free(tri);
    return 0;
}
