// Block low-rank (BLR) operator: far tiles of K1, K2^eps and K2^mu stored as
// products U V^T from adaptive cross approximation (ACA), near tiles dense.
// The paper stops at the dense operator and names fast far-field methods as
// future work (Sec. 7, Conclusion); this extends the solve to meshes whose dense blocks
// exceed one device's memory.  The operator is filled one band of rows (a
// run of whole row clusters) at a time into a scratch, compressed, and
// packed; the dense blocks never exist.
//
// Tiles are kept in the fixed order (op, row cluster t, column cluster s),
// so tile (op, t, s) is tiles[(op nc + t) nc + s] and the tiles of one band
// row are consecutive.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "mbem_internal.h"

namespace mbem {

constexpr int kAcaThreads = 256;
constexpr int kAcaWaves = kAcaThreads / 64;
constexpr int kMaxRank = 128;
constexpr int kMaxCluster = 2048;              // nodes per cluster
constexpr int kMaxTileRows = 2 * kMaxCluster;

struct BlrOp {
    int32_t L = 0, nc = 0;
    std::vector<int32_t> start;                // first node of each cluster, then nn
    int32_t *d_cl_of = nullptr;                // node -> cluster
    std::vector<BlrTile> tiles;                // host copy, order (op, t, s)
    BlrTile *d_tiles = nullptr;
    int32_t *d_lr = nullptr;                   // tiles with rank > 0
    int32_t n_lr = 0;
    double2 *d_w = nullptr;                    // V^T x of every low-rank tile
    double2 *d_z = nullptr;                    // row products of every tile
    int32_t *d_dense = nullptr;                // dense tiles
    int32_t n_dense = 0;
    std::vector<void *> store;                 // tile storage, one allocation per band
};

void blr_free(BlrOp *b) {
    if (!b) return;
    for (void *p : b->store)
        if (p) (void)hipFree(p);
    void *ps[] = {b->d_tiles, b->d_lr, b->d_w, b->d_cl_of, b->d_z, b->d_dense};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete b;
}

BlrView blr_view(const mbem_op *op) { return {op->blr->nc, op->blr->d_cl_of, op->blr->d_tiles}; }

// Leaves of the octree of the sorted Morton keys: the run [a, b) of nodes
// sharing the top 3 lev key bits is a cell; a cell of more than L nodes is
// split into the runs sharing 3 (lev + 1) bits, down to level 21, where a run
// still longer than L is cut into pieces of L.
static void octree_leaves(const std::vector<uint64_t> &key, int64_t a, int64_t b, int lev, int L,
                          std::vector<int32_t> &start) {
    if (b - a <= L) { start.push_back((int32_t)a); return; }
    if (lev == 21) {
        for (int64_t q = a; q < b; q += L) start.push_back((int32_t)q);
        return;
    }
    const int sh = 3 * (20 - lev);
    int64_t u = a;
    for (int64_t i = a + 1; i <= b; ++i)
        if (i == b || (key[i] >> sh) != (key[i - 1] >> sh)) {
            octree_leaves(key, u, i, lev + 1, L, start);
            u = i;
        }
}

// ------------------------------------------------------- reductions ---
__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// larger value wins, the lower index on equal values
__device__ inline void wave_argmax(double &v, int &i) {
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int oi = __shfl_xor(i, o, 64);
        if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
    }
}

// Every thread returns the workgroup's sum, combined in wave order.
__device__ inline double block_sum(double v, double *buf) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kAcaWaves; ++w) t += buf[w];
    __syncthreads();
    return t;
}

__device__ inline void block_argmax(double &v, int &i, double *bv, int *bi) {
    wave_argmax(v, i);
    if ((threadIdx.x & 63) == 0) { bv[threadIdx.x >> 6] = v; bi[threadIdx.x >> 6] = i; }
    __syncthreads();
    v = bv[0];
    i = bi[0];
    for (int w = 1; w < kAcaWaves; ++w)
        if (bv[w] > v || (bv[w] == v && bi[w] < i)) { v = bv[w]; i = bi[w]; }
    __syncthreads();
}

__device__ inline int block_min(int v, int *buf) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = buf[0];
    for (int w = 1; w < kAcaWaves; ++w) t = min(t, buf[w]);
    __syncthreads();
    return t;
}

__device__ inline double2 cmul2(double2 a, double2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// conj(a) b
__device__ inline double2 cdotc(double2 a, double2 b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }

// ------------------------------------------------------------ ACA ---
struct AcaTask {
    int32_t op, m, n, pad;
    int64_t org;         // offset of the tile's first entry in the band buffer
    int64_t u, v;        // scratch offsets of U [rmax][m] and V [rmax][n]
};

// Cross approximation with partial pivoting of one tile A (rows 0..m-1 of
// the band buffer, columns c0..c0+n-1), one workgroup per tile:
//   row pivot i (first 0), residual row r = A(i,:) - sum_l U_l(i) V_l,
//   column pivot j = argmax |r|, v_k = r / r(j), residual column u_k =
//   A(:,j) - sum_l V_l(j) U_l, next row pivot = argmax |u_k| over unused
//   rows; |S_k|_F^2 grows by 2 Re sum_l <u_l,u_k><v_l,v_k> + |u_k|^2 |v_k|^2
//   and the approximation stops when |u_k| |v_k| <= eps |S_k|_F.  A row
//   whose residual vanishes is marked used and the lowest unused row is
//   tried next.  rank_out: the number of terms, or -1 when rmax terms did
//   not reach eps.  Every pass adds a term or uses up a row, so the loop
//   ends after at most m + rmax passes.
__global__ __launch_bounds__(kAcaThreads) void k_aca(const AcaTask *tasks, const double2 *Z0,
                                                    const double2 *Z1, const double2 *Z2, int64_t ld,
                                                    double eps, int rmax, double2 *scr,
                                                    int32_t *rank_out) {
    __shared__ unsigned char s_used[kMaxTileRows];
    __shared__ double2 s_c[kMaxRank];                 // pivot entries of the earlier terms
    __shared__ double2 s_du[kMaxRank], s_dv[kMaxRank];
    __shared__ double s_bv[kAcaWaves];
    __shared__ int s_bi[kAcaWaves];
    const AcaTask T = tasks[blockIdx.x];
    const double2 *A = (T.op == 0 ? Z0 : (T.op == 1 ? Z1 : Z2)) + T.org;
    double2 *U = scr + T.u, *V = scr + T.v;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = T.m, n = T.n;
    for (int i = tid; i < m; i += kAcaThreads) s_used[i] = 0;
    __syncthreads();
    double s2 = 0.0;
    int piv = 0, k = 0, result = -1;
    for (int pass = 0; pass < m + rmax && k < rmax; ++pass) {
        // residual of row piv into V[k]
        for (int l = tid; l < k; l += kAcaThreads) s_c[l] = U[(int64_t)l * m + piv];
        __syncthreads();
        double2 *vk = V + (int64_t)k * n;
        double best = -1.0;
        int bj = n;
        for (int j = tid; j < n; j += kAcaThreads) {
            double2 r = A[(int64_t)piv * ld + j];
            for (int l = 0; l < k; ++l) {
                const double2 p = cmul2(s_c[l], V[(int64_t)l * n + j]);
                r.x -= p.x;
                r.y -= p.y;
            }
            vk[j] = r;
            const double a = r.x * r.x + r.y * r.y;
            if (a > best) { best = a; bj = j; }
        }
        block_argmax(best, bj, s_bv, s_bi);
        if (tid == 0) s_used[piv] = 1;
        __syncthreads();
        if (!(best > 0.0)) {
            int nxt = m;
            for (int i = tid; i < m; i += kAcaThreads)
                if (!s_used[i]) { nxt = i; break; }
            nxt = block_min(nxt, s_bi);
            if (nxt == m) { result = k; break; }
            piv = nxt;
            continue;
        }
        // v_k = r / r(j)
        const double2 d = vk[bj];
        const double dn = d.x * d.x + d.y * d.y;
        const double2 inv = {d.x / dn, -d.y / dn};
        double nv = 0.0;
        for (int j = tid; j < n; j += kAcaThreads) {
            const double2 r = cmul2(vk[j], inv);
            vk[j] = r;
            nv += r.x * r.x + r.y * r.y;
        }
        nv = block_sum(nv, s_bv);
        for (int l = wv; l < k; l += kAcaWaves) {
            double re = 0.0, im = 0.0;
            for (int j = lane; j < n; j += 64) {
                const double2 p = cdotc(V[(int64_t)l * n + j], vk[j]);
                re += p.x;
                im += p.y;
            }
            re = wave_sum(re);
            im = wave_sum(im);
            if (lane == 0) s_dv[l] = {re, im};
        }
        // residual of column bj into U[k]
        for (int l = tid; l < k; l += kAcaThreads) s_c[l] = V[(int64_t)l * n + bj];
        __syncthreads();
        double2 *uk = U + (int64_t)k * m;
        double nu = 0.0, bu = -1.0;
        int bi = m;
        for (int i = tid; i < m; i += kAcaThreads) {
            double2 r = A[(int64_t)i * ld + bj];
            for (int l = 0; l < k; ++l) {
                const double2 p = cmul2(s_c[l], U[(int64_t)l * m + i]);
                r.x -= p.x;
                r.y -= p.y;
            }
            uk[i] = r;
            const double a = r.x * r.x + r.y * r.y;
            nu += a;
            if (!s_used[i] && a > bu) { bu = a; bi = i; }
        }
        nu = block_sum(nu, s_bv);
        block_argmax(bu, bi, s_bv, s_bi);
        for (int l = wv; l < k; l += kAcaWaves) {
            double re = 0.0, im = 0.0;
            for (int i = lane; i < m; i += 64) {
                const double2 p = cdotc(U[(int64_t)l * m + i], uk[i]);
                re += p.x;
                im += p.y;
            }
            re = wave_sum(re);
            im = wave_sum(im);
            if (lane == 0) s_du[l] = {re, im};
        }
        __syncthreads();
        double cross = 0.0;
        for (int l = 0; l < k; ++l) cross += 2.0 * (s_du[l].x * s_dv[l].x - s_du[l].y * s_dv[l].y);
        s2 += cross + nu * nv;
        ++k;
        __syncthreads();   // s_c, s_du and s_dv are rewritten by the next pass
        if (sqrt(nu * nv) <= eps * sqrt(fmax(s2, 0.0))) { result = k; break; }
        if (bi == m) { result = k; break; }   // every row used
        piv = bi;
    }
    if (tid == 0) rank_out[blockIdx.x] = result;
}

// ------------------------------------------------------------ packing ---
struct PackTask {
    int32_t op, rank, m, n;  // rank < 0: dense copy of the band's tile
    int64_t org;             // offset of the tile's first entry in the band buffer
    int64_t u, v;            // scratch offsets (low-rank)
    double2 *a, *vt;         // destinations
};

__global__ __launch_bounds__(256) void k_blr_pack(const PackTask *tasks, const double2 *Z0, const double2 *Z1,
                                                  const double2 *Z2, int64_t ld, const double2 *scr) {
    const PackTask T = tasks[blockIdx.y];
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (T.rank < 0) {
        const double2 *A = (T.op == 0 ? Z0 : (T.op == 1 ? Z1 : Z2)) + T.org;
        const int64_t cnt = (int64_t)T.m * T.n;
        for (int64_t e = first; e < cnt; e += step) T.a[e] = A[(e / T.n) * ld + e % T.n];
        return;
    }
    const int64_t cu = (int64_t)T.m * T.rank, cv = (int64_t)T.rank * T.n;
    for (int64_t e = first; e < cu; e += step) T.a[e] = scr[T.u + e];    // U^T = scratch [k][m]
    for (int64_t e = first; e < cv; e += step) T.vt[e] = scr[T.v + e];   // V^T = scratch [k][n]
}

// ----------------------------------------------------------- products ---
// w = V^T x for every low-rank tile (K1: x_j then x_m; K2^eps: x_m;
// K2^mu: x_j), one wavefront per term.
__global__ __launch_bounds__(256) void k_blr_vt(const BlrTile *tiles, const int32_t *lr,
                                                const double2 *xj, const double2 *xm, double2 *w) {
    const BlrTile T = tiles[lr[blockIdx.x]];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool two = T.op == 0;
    const double2 *x0 = (T.op == 1 ? xm : xj) + T.c0, *x1 = xm + T.c0;
    for (int k = wv; k < T.rank; k += 4) {
        const double2 *row = T.vt + (int64_t)k * T.n;
        double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
        for (int j = lane; j < T.n; j += 64) {
            const double2 v = row[j];
            const double2 p = cmul2(v, x0[j]);
            a0r += p.x;
            a0i += p.y;
            if (two) {
                const double2 q = cmul2(v, x1[j]);
                a1r += q.x;
                a1i += q.y;
            }
        }
        a0r = wave_sum(a0r);
        a0i = wave_sum(a0i);
        if (two) { a1r = wave_sum(a1r); a1i = wave_sum(a1i); }
        if (lane == 0) {
            w[T.w + k] = {a0r, a0i};
            if (two) w[T.w + T.rank + k] = {a1r, a1i};
        }
    }
}

// Row products of every tile into its own slice of z (K1: x_j then x_m):
//   dense tiles: one wavefront per row, lanes along the columns;
//   low-rank tiles: U (m x rank) against the tile's V^T x, one lane per row;
// then one lane per (block, row) sums the slices of its band in column order
// (a fixed order: the product is reproducible).
__global__ __launch_bounds__(256) void k_blr_dense(const BlrTile *tiles, const int32_t *dense,
                                                   const double2 *xj, const double2 *xm, double2 *z) {
    const BlrTile T = tiles[dense[blockIdx.x]];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool two = T.op == 0;
    const double2 *y0 = (T.op == 1 ? xm : xj) + T.c0, *y1 = xm + T.c0;
    for (int i = wv; i < T.m; i += 4) {
        const double2 *a = T.a + (int64_t)i * T.n;
        double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
        for (int j = lane; j < T.n; j += 64) {
            const double2 v = a[j];
            const double2 p = cmul2(v, y0[j]);
            a0r += p.x;
            a0i += p.y;
            if (two) {
                const double2 q = cmul2(v, y1[j]);
                a1r += q.x;
                a1i += q.y;
            }
        }
        a0r = wave_sum(a0r);
        a0i = wave_sum(a0i);
        if (two) { a1r = wave_sum(a1r); a1i = wave_sum(a1i); }
        if (lane == 0) {
            z[T.z + i] = {a0r, a0i};
            if (two) z[T.z + T.m + i] = {a1r, a1i};
        }
    }
}

__global__ __launch_bounds__(256) void k_blr_u(const BlrTile *tiles, const int32_t *lr, const double2 *w,
                                               double2 *z) {
    __shared__ double2 s_w[2 * kMaxRank];
    const BlrTile T = tiles[lr[blockIdx.x]];
    const bool two = T.op == 0;
    const int nw = (two ? 2 : 1) * T.rank;
    for (int q = threadIdx.x; q < nw; q += blockDim.x) s_w[q] = w[T.w + q];
    __syncthreads();
    for (int i = threadIdx.x; i < T.m; i += blockDim.x) {
        double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
        for (int k = 0; k < T.rank; ++k) {
            const double2 v = T.a[(int64_t)k * T.m + i];
            const double2 p = cmul2(v, s_w[k]);
            a0r += p.x;
            a0i += p.y;
            if (two) {
                const double2 q = cmul2(v, s_w[T.rank + k]);
                a1r += q.x;
                a1i += q.y;
            }
        }
        z[T.z + i] = {a0r, a0i};
        if (two) z[T.z + T.m + i] = {a1r, a1i};
    }
}

__global__ __launch_bounds__(256) void k_blr_sum(int64_t n2, const int32_t *cl_of, int32_t nc,
                                                 const BlrTile *tiles, const double2 *z, double2 *t) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= 3 * n2) return;
    const int op = (int)(id / n2);
    const int64_t r = id % n2;
    const BlrTile *row = tiles + ((int64_t)op * nc + cl_of[r >> 1]) * nc;
    const int64_t lr = r - row[0].r0;
    double2 a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
    for (int sc = 0; sc < nc; ++sc) {
        const BlrTile &T = row[sc];
        if (T.rank == 0) continue;
        const double2 v = z[T.z + lr];
        a0.x += v.x;
        a0.y += v.y;
        if (op == 0) {
            const double2 u = z[T.z + T.m + lr];
            a1.x += u.x;
            a1.y += u.y;
        }
    }
    if (op == 0) { t[r] = a0; t[n2 + r] = a1; }
    else if (op == 1) t[2 * n2 + r] = a0;
    else t[3 * n2 + r] = a0;
}

// one workgroup per tile
__global__ __launch_bounds__(256) void k_blr_expand(const BlrTile *tiles, int64_t n2, double2 *K0, double2 *K1,
                                                    double2 *K2) {
    const BlrTile T = tiles[blockIdx.x];
    double2 *K = T.op == 0 ? K0 : (T.op == 1 ? K1 : K2);
    if (!K) return;
    const int64_t cnt = (int64_t)T.m * T.n;
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        const int64_t i = e / T.n, j = e % T.n;
        double2 z;
        if (T.rank < 0) z = T.a[e];
        else {
            z = {0.0, 0.0};
            for (int kk = 0; kk < T.rank; ++kk) {
                const double2 p = cmul2(T.a[(int64_t)kk * T.m + i], T.vt[(int64_t)kk * T.n + j]);
                z.x += p.x;
                z.y += p.y;
            }
        }
        K[(T.r0 + i) * n2 + T.c0 + j] = z;
    }
}

int blr_gemv_run(const mbem_op *op, const double2 *xj, const double2 *xm, double2 *t, hipStream_t s) {
    const BlrOp *b = op->blr;
    if (b->n_lr > 0) {
        hipLaunchKernelGGL(k_blr_vt, dim3((unsigned)b->n_lr), dim3(256), 0, s, b->d_tiles, b->d_lr, xj, xm, b->d_w);
        MBEM_HIP(hipGetLastError());
    }
    if (b->n_lr > 0) {
        hipLaunchKernelGGL(k_blr_u, dim3((unsigned)b->n_lr), dim3(256), 0, s, b->d_tiles, b->d_lr, b->d_w, b->d_z);
        MBEM_HIP(hipGetLastError());
    }
    if (b->n_dense > 0) {
        hipLaunchKernelGGL(k_blr_dense, dim3((unsigned)b->n_dense), dim3(256), 0, s, b->d_tiles, b->d_dense, xj, xm,
                           b->d_z);
        MBEM_HIP(hipGetLastError());
    }
    const int64_t rows = 3 * op->n2;
    hipLaunchKernelGGL(k_blr_sum, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, op->n2, b->d_cl_of, b->nc,
                       b->d_tiles, b->d_z, t);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

int blr_expand_run(const mbem_op *op, double2 *K0, double2 *K1, double2 *K2, hipStream_t s) {
    const BlrOp *b = op->blr;
    const int64_t n2 = op->n2;
    double2 *K[3] = {K0, K1, K2};
    for (int o = 0; o < 3; ++o)
        if (K[o]) MBEM_HIP(hipMemsetAsync(K[o], 0, sizeof(double2) * n2 * n2, s));
    const unsigned nt = (unsigned)b->tiles.size();
    hipLaunchKernelGGL(k_blr_expand, dim3(nt), dim3(256), 0, s, b->d_tiles, n2, K0, K1, K2);
    MBEM_HIP(hipGetLastError());
    MBEM_HIP(hipStreamSynchronize(s));
    return MBEM_OK;
}

// ------------------------------------------------------------- driver ---
namespace {

struct Events {
    hipEvent_t a = nullptr, b = nullptr, c = nullptr;
    Events() { (void)hipEventCreate(&a); (void)hipEventCreate(&b); (void)hipEventCreate(&c); }
    ~Events() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); }
    static double ms(hipEvent_t x, hipEvent_t y) {
        float t = 0.f;
        return hipEventElapsedTime(&t, x, y) == hipSuccess ? t : 0.0;
    }
};

// Device buffers of the assembly; freed on every exit.
struct Scratch {
    std::vector<void *> p;
    ~Scratch() {
        for (void *q : p)
            if (q) (void)hipFree(q);
    }
    template <typename T>
    int alloc(T **out, size_t n) {
        *out = nullptr;
        hipError_t e = hipMalloc((void **)out, sizeof(T) * std::max<size_t>(n, 1));
        if (e != hipSuccess) {
            set_error(std::string("block low-rank assembly: ") + hipGetErrorString(e));
            return MBEM_ENOMEM;
        }
        p.push_back(*out);
        return MBEM_OK;
    }
};

}  // namespace

int blr_fill_run(mbem_op *op, const mbem_blr_opts *o, mbem_blr_stats *bs, hipStream_t s) {
    const mbem_mesh *m = op->mesh;
    const int64_t nn = m->nn, nt = m->nt, n2 = op->n2;
    const int L = o->cluster;
    std::vector<int32_t> start;
    octree_leaves(m->node_key, 0, nn, 0, L, start);
    start.push_back((int32_t)nn);
    const int nc = (int)start.size() - 1;
    std::vector<int32_t> cl_of(nn);
    for (int c = 0; c < nc; ++c)
        for (int32_t v = start[c]; v < start[c + 1]; ++v) cl_of[v] = c;
    auto size_of = [&](int c) { return (int64_t)(start[c + 1] - start[c]); };
    // support boxes: every node of every element touching the cluster
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<double> lo(3 * (size_t)nc, inf), hi(3 * (size_t)nc, -inf);
    std::vector<std::vector<int32_t>> tri_bands(nt);   // clusters with a node of the triangle
    for (int64_t e = 0; e < nt; ++e) {
        std::vector<int32_t> &cs = tri_bands[e];
        for (int i = 0; i < 6; ++i) {
            const int32_t c = cl_of[m->tri[6 * e + i]];
            if (std::find(cs.begin(), cs.end(), c) == cs.end()) cs.push_back(c);
        }
        std::sort(cs.begin(), cs.end());
        for (int32_t c : cs)
            for (int i = 0; i < 6; ++i)
                for (int d = 0; d < 3; ++d) {
                    const double x = m->xyz[3 * (size_t)m->tri[6 * e + i] + d];
                    lo[3 * c + d] = std::min(lo[3 * c + d], x);
                    hi[3 * c + d] = std::max(hi[3 * c + d], x);
                }
    }
    std::vector<unsigned char> adm((size_t)nc * nc, 0);
    int n_adm = 0;
    for (int t = 0; t < nc; ++t)
        for (int sc = 0; sc < nc; ++sc) {
            if (t == sc) continue;
            double g2 = 0, dt = 0, ds = 0;
            for (int d = 0; d < 3; ++d) {
                const double gap = std::max(0.0, std::max(lo[3 * t + d] - hi[3 * sc + d], lo[3 * sc + d] - hi[3 * t + d]));
                g2 += gap * gap;
                dt += (hi[3 * t + d] - lo[3 * t + d]) * (hi[3 * t + d] - lo[3 * t + d]);
                ds += (hi[3 * sc + d] - lo[3 * sc + d]) * (hi[3 * sc + d] - lo[3 * sc + d]);
            }
            const double dist = std::sqrt(g2), diam = std::sqrt(std::max(dt, ds));
            if (dist > 0 && diam <= o->eta * dist) { adm[(size_t)t * nc + sc] = 1; ++n_adm; }
        }
    // Row bands: runs of whole clusters of up to `band` nodes (automatic:
    // three band buffers of about 16 GB), filled together so that the halo
    // and the number of launches shrink; every cluster's tiles are then
    // approximated from the band's rows.
    int64_t band_nodes = o->band > 0 ? o->band : (int64_t)(16e9 / (3.0 * 2.5 * 16.0 * (double)n2));
    band_nodes = std::max<int64_t>(band_nodes, L);
    if (o->band <= 0) band_nodes = std::min<int64_t>(band_nodes, 8192);
    std::vector<int32_t> bstart(1, 0);   // first cluster of each band, then nc
    for (int c = 0; c < nc; ++c)
        if (c > bstart.back() && (int64_t)start[c + 1] - start[bstart.back()] > band_nodes) bstart.push_back(c);
    bstart.push_back(nc);
    const int nb = (int)bstart.size() - 1;
    std::vector<int32_t> band_of(nc);
    for (int bb = 0; bb < nb; ++bb)
        for (int c = bstart[bb]; c < bstart[bb + 1]; ++c) band_of[c] = bb;
    // band lists: test triangles by colour class, singular pairs, halo nodes
    const int ntc = (int)m->tcol_off.size() - 1;
    std::vector<std::vector<int32_t>> tri_b(nt);   // bands with a node of the triangle
    for (int64_t e = 0; e < nt; ++e)
        for (int32_t c : tri_bands[e]) {
            const int32_t bb = band_of[c];
            if (std::find(tri_b[e].begin(), tri_b[e].end(), bb) == tri_b[e].end()) tri_b[e].push_back(bb);
        }
    std::vector<std::vector<int32_t>> btri(nb), boff(nb, std::vector<int32_t>(1, 0)), bsp(nb);
    for (int tc = 0; tc < ntc; ++tc) {
        for (int32_t q = m->tcol_off[tc]; q < m->tcol_off[tc + 1]; ++q) {
            const int32_t e = m->tcol_list[q];
            for (int32_t bb : tri_b[e]) btri[bb].push_back(e);
        }
        for (int bb = 0; bb < nb; ++bb) boff[bb].push_back((int32_t)btri[bb].size());
    }
    for (size_t q = 0; q + 3 < m->spairs.size(); q += 4)
        for (int32_t bb : tri_b[m->spairs[q]])
            for (int k = 0; k < 4; ++k) bsp[bb].push_back(m->spairs[q + k]);
    std::vector<std::vector<int32_t>> halo(nb);
    size_t rows_max = 0, tri_max = 0, sp_max = 0, scr_max = 0, task_max = 0, pack_max = 0;
    for (int bb = 0; bb < nb; ++bb) {
        const int64_t n0 = start[bstart[bb]], n1 = start[bstart[bb + 1]];
        std::vector<int32_t> &h = halo[bb];
        for (int32_t e : btri[bb])
            for (int i = 0; i < 6; ++i) {
                const int32_t v = m->tri[6 * (size_t)e + i];
                if (v < n0 || v >= n1) h.push_back(v);
            }
        std::sort(h.begin(), h.end());
        h.erase(std::unique(h.begin(), h.end()), h.end());
        rows_max = std::max(rows_max, (size_t)(2 * (n1 - n0) + 2 * h.size()));
        tri_max = std::max(tri_max, btri[bb].size());
        sp_max = std::max(sp_max, bsp[bb].size());
        size_t scr = 0, ntask = 0;
        for (int c = bstart[bb]; c < bstart[bb + 1]; ++c)
            for (int sc = 0; sc < nc; ++sc)
                if (adm[(size_t)c * nc + sc]) {
                    scr += 3 * (size_t)o->rmax * (size_t)(2 * size_of(c) + 2 * size_of(sc));
                    ntask += 3;
                }
        scr_max = std::max(scr_max, scr);
        task_max = std::max(task_max, ntask);
        pack_max = std::max(pack_max, 3 * (size_t)nc * (size_t)(bstart[bb + 1] - bstart[bb]));
    }
    // device buffers of the assembly
    Scratch S;
    double2 *zb = nullptr, *scr = nullptr;
    int32_t *d_map = nullptr, *d_tri = nullptr, *d_sp = nullptr, *d_rank = nullptr;
    AcaTask *d_tasks = nullptr;
    PackTask *d_pack = nullptr;
    const size_t band_elems = rows_max * (size_t)n2;
    MBEM_TRY(S.alloc(&zb, 3 * band_elems));
    MBEM_TRY(S.alloc(&scr, scr_max));
    MBEM_TRY(S.alloc(&d_map, (size_t)nn));
    MBEM_TRY(S.alloc(&d_tri, tri_max));
    MBEM_TRY(S.alloc(&d_sp, sp_max));
    MBEM_TRY(S.alloc(&d_rank, task_max));
    MBEM_TRY(S.alloc(&d_tasks, task_max));
    MBEM_TRY(S.alloc(&d_pack, pack_max));
    BlrOp *b = new (std::nothrow) BlrOp;
    if (!b) { set_error("host allocation"); return MBEM_ENOMEM; }
    op->blr = b;
    b->L = L;
    b->nc = nc;
    b->start = start;
    if (hipMalloc((void **)&b->d_cl_of, sizeof(int32_t) * nn) != hipSuccess) {
        set_error("block low-rank tables: device allocation");
        return MBEM_ENOMEM;
    }
    MBEM_HIP(hipMemcpyAsync(b->d_cl_of, cl_of.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice, s));
    b->tiles.resize(3 * (size_t)nc * nc);
    // geometry, kernel constants and the mass matrix once
    MBEM_TRY(fill_prepare(op, s, false));
    MBEM_TRY(geom_build(m, s, false));
    MBEM_TRY(mass_run(op, s));
    Events ev;
    double t_fill = 0, t_aca = 0;
    int n_lowrank = 0, max_rank = 0;
    double sum_rank = 0;
    int64_t stored = 0;
    std::vector<int32_t> rmap(nn, 0);
    std::vector<AcaTask> tasks;
    std::vector<int32_t> ranks;
    std::vector<PackTask> packs;
    for (int bb = 0; bb < nb; ++bb) {
        const int cb = bstart[bb], ce = bstart[bb + 1];
        const int64_t n0 = start[cb], n1 = start[ce];
        // rows: the band's nodes first (node - n0), then its halo
        for (int64_t v = n0; v < n1; ++v) rmap[v] = (int32_t)(v - n0);
        for (size_t q = 0; q < halo[bb].size(); ++q) rmap[halo[bb][q]] = (int32_t)(n1 - n0 + q);
        const size_t rows = (size_t)(2 * (n1 - n0)) + 2 * halo[bb].size();
        MBEM_HIP(hipMemcpyAsync(d_map, rmap.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice, s));
        MBEM_HIP(hipMemcpyAsync(d_tri, btri[bb].data(), sizeof(int32_t) * btri[bb].size(), hipMemcpyHostToDevice, s));
        MBEM_HIP(hipMemcpyAsync(d_sp, bsp[bb].data(), sizeof(int32_t) * bsp[bb].size(), hipMemcpyHostToDevice, s));
        for (int q = 0; q < 3; ++q)
            MBEM_HIP(hipMemsetAsync(zb + q * band_elems, 0, sizeof(double2) * rows * n2, s));
        FillBand fb;
        fb.tcol = d_tri;
        fb.tcol_off = boff[bb];
        fb.spairs = d_sp;
        fb.n_spairs = (int64_t)bsp[bb].size() / 4;
        fb.row_map = d_map;
        for (int q = 0; q < 3; ++q) fb.Z[q] = zb + q * band_elems;
        MBEM_HIP(hipEventRecord(ev.a, s));
        MBEM_TRY(fill_band_run(op, fb, s));
        MBEM_HIP(hipEventRecord(ev.b, s));
        // cross approximation of the admissible tiles of the band's clusters
        tasks.clear();
        int64_t off = 0;
        for (int c = cb; c < ce; ++c) {
            const int32_t mt = (int32_t)(2 * size_of(c));
            const int64_t rorg = 2 * (int64_t)(start[c] - n0) * n2;   // first row of c in the band
            for (int sc = 0; sc < nc; ++sc) {
                if (!adm[(size_t)c * nc + sc]) continue;
                const int32_t ns = (int32_t)(2 * size_of(sc));
                for (int q = 0; q < 3; ++q) {
                    AcaTask a{q, mt, ns, 0, rorg + 2 * (int64_t)start[sc], off, off + (int64_t)o->rmax * mt};
                    off += (int64_t)o->rmax * (mt + ns);
                    tasks.push_back(a);
                }
            }
        }
        if (!tasks.empty()) {
            MBEM_HIP(hipMemcpyAsync(d_tasks, tasks.data(), sizeof(AcaTask) * tasks.size(), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_aca, dim3((unsigned)tasks.size()), dim3(kAcaThreads), 0, s, d_tasks, zb,
                               zb + band_elems, zb + 2 * band_elems, (int64_t)n2, o->eps, o->rmax, scr, d_rank);
            MBEM_HIP(hipGetLastError());
        }
        MBEM_HIP(hipEventRecord(ev.c, s));
        ranks.assign(tasks.size(), -1);
        if (!tasks.empty())
            MBEM_HIP(hipMemcpyAsync(ranks.data(), d_rank, sizeof(int32_t) * tasks.size(), hipMemcpyDeviceToHost, s));
        MBEM_HIP(hipStreamSynchronize(s));
        t_fill += Events::ms(ev.a, ev.b);
        t_aca += Events::ms(ev.b, ev.c);
        // storage of the band's tiles: what each one keeps
        const size_t ncb = (size_t)(ce - cb);
        std::vector<int32_t> keep_rank(3 * ncb * nc, -1);   // [c - cb][q][sc]
        size_t ti = 0;
        int64_t elems = 0;
        for (int c = cb; c < ce; ++c) {
            const int64_t mt = 2 * size_of(c);
            for (int sc = 0; sc < nc; ++sc) {
                const int64_t ns = 2 * size_of(sc);
                const bool a = adm[(size_t)c * nc + sc];
                for (int q = 0; q < 3; ++q) {
                    int32_t r = -1;
                    if (a) {
                        const int32_t got = ranks[ti++];
                        if (got >= 0 && (o->keep_lowrank || (int64_t)got * (mt + ns) < mt * ns)) r = got;
                    }
                    keep_rank[((size_t)(c - cb) * 3 + q) * nc + sc] = r;
                    elems += r < 0 ? mt * ns : (int64_t)r * (mt + ns);
                }
            }
        }
        double2 *store = nullptr;
        if (elems > 0) {
            hipError_t e = hipMalloc((void **)&store, sizeof(double2) * elems);
            if (e != hipSuccess) {
                set_error(std::string("block low-rank storage: ") + hipGetErrorString(e));
                return MBEM_ENOMEM;
            }
            b->store.push_back(store);
        }
        stored += elems * (int64_t)sizeof(double2);
        packs.clear();
        int64_t pos = 0;
        ti = 0;
        for (int c = cb; c < ce; ++c) {
            const int32_t mt = (int32_t)(2 * size_of(c));
            const int64_t rorg = 2 * (int64_t)(start[c] - n0) * n2;
            for (int sc = 0; sc < nc; ++sc) {
                const int32_t ns = (int32_t)(2 * size_of(sc));
                const bool a = adm[(size_t)c * nc + sc];
                for (int q = 0; q < 3; ++q) {
                    const int32_t r = keep_rank[((size_t)(c - cb) * 3 + q) * nc + sc];
                    BlrTile &T = b->tiles[((size_t)q * nc + c) * nc + sc];
                    T = BlrTile{q, c, sc, r, mt, ns, 2 * (int64_t)start[c], 2 * (int64_t)start[sc], store + pos,
                                nullptr, 0, 0};
                    PackTask P{q, r, mt, ns, rorg + 2 * (int64_t)start[sc], 0, 0, store + pos, nullptr};
                    if (a) {
                        P.u = tasks[ti].u;
                        P.v = tasks[ti].v;
                        ++ti;
                    }
                    if (r < 0) pos += (int64_t)mt * ns;
                    else {
                        T.vt = store + pos + (int64_t)mt * r;
                        P.vt = T.vt;
                        pos += (int64_t)r * (mt + ns);
                        ++n_lowrank;
                        max_rank = std::max(max_rank, (int)r);
                        sum_rank += r;
                    }
                    if (r != 0) packs.push_back(P);
                }
            }
        }
        if (!packs.empty()) {
            MBEM_HIP(hipMemcpyAsync(d_pack, packs.data(), sizeof(PackTask) * packs.size(), hipMemcpyHostToDevice, s));
            // tasks along y, at most 65535 per launch
            for (size_t p0 = 0; p0 < packs.size(); p0 += 65535) {
                const size_t ny = std::min<size_t>(65535, packs.size() - p0);
                hipLaunchKernelGGL(k_blr_pack, dim3(64, (unsigned)ny), dim3(256), 0, s, d_pack + p0, zb,
                                   zb + band_elems, zb + 2 * band_elems, (int64_t)n2, scr);
                MBEM_HIP(hipGetLastError());
            }
            MBEM_HIP(hipGetLastError());
        }
        // the host lists of the next band overwrite what these copies read
        MBEM_HIP(hipStreamSynchronize(s));
        for (int64_t v = n0; v < n1; ++v) rmap[v] = 0;
        for (int32_t v : halo[bb]) rmap[v] = 0;
    }
    // product workspace and device tables
    std::vector<int32_t> lr, dn;
    int64_t w = 0, zz = 0;
    for (size_t q = 0; q < b->tiles.size(); ++q) {
        BlrTile &T = b->tiles[q];
        const int nv = T.op == 0 ? 2 : 1;
        T.z = zz;
        if (T.rank != 0) zz += nv * (int64_t)T.m;
        if (T.rank > 0) {
            T.w = w;
            w += nv * (int64_t)T.rank;
            lr.push_back((int32_t)q);
        } else if (T.rank < 0) {
            dn.push_back((int32_t)q);
        }
    }
    b->n_lr = (int32_t)lr.size();
    b->n_dense = (int32_t)dn.size();
    hipError_t e1 = hipMalloc((void **)&b->d_tiles, sizeof(BlrTile) * b->tiles.size());
    hipError_t e2 = hipMalloc((void **)&b->d_lr, sizeof(int32_t) * std::max<size_t>(1, lr.size()));
    hipError_t e3 = hipMalloc((void **)&b->d_w, sizeof(double2) * std::max<int64_t>(1, w));
    hipError_t e4 = hipMalloc((void **)&b->d_z, sizeof(double2) * std::max<int64_t>(1, zz));
    hipError_t e5 = hipMalloc((void **)&b->d_dense, sizeof(int32_t) * std::max<size_t>(1, dn.size()));
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess || e5 != hipSuccess) {
        set_error("block low-rank tables: device allocation");
        return MBEM_ENOMEM;
    }
    MBEM_HIP(hipMemcpyAsync(b->d_tiles, b->tiles.data(), sizeof(BlrTile) * b->tiles.size(), hipMemcpyHostToDevice, s));
    if (!lr.empty()) MBEM_HIP(hipMemcpyAsync(b->d_lr, lr.data(), sizeof(int32_t) * lr.size(), hipMemcpyHostToDevice, s));
    if (!dn.empty()) MBEM_HIP(hipMemcpyAsync(b->d_dense, dn.data(), sizeof(int32_t) * dn.size(), hipMemcpyHostToDevice, s));
    MBEM_HIP(hipStreamSynchronize(s));
    if (bs) {
        bs->stored_bytes = stored;
        bs->dense_bytes = 3 * (int64_t)n2 * n2 * (int64_t)sizeof(double2);
        bs->n_clusters = nc;
        bs->n_tiles = (int32_t)b->tiles.size();
        bs->n_admissible = 3 * n_adm;
        bs->n_lowrank = n_lowrank;
        bs->max_rank = max_rank;
        bs->mean_rank = n_lowrank ? sum_rank / n_lowrank : 0.0;
        bs->t_fill_ms = t_fill;
        bs->t_aca_ms = t_aca;
    }
    return MBEM_OK;
}

}  // namespace mbem
