// Galerkin fill of K1, K2^eps, K2^mu (Sec. 4.1-4.2, fused as in Sec. 6.1)
// and of the mass matrix (eq. mass_matrix).
//
//  * regular pairs: 7 x 7 quadrature-point pairs per element pair; the
//    twelve weighted kernel values of every point pair go to LDS and are
//    contracted with the shape functions in two steps (trial side, then test
//    side after the triangles are merged by node) before being added to Z.
//    FP64 (k_regular): one workgroup per (test triangle, chunk of 4
//    Morton-consecutive trial triangles), one launch per (test colour, chunk
//    colour) so that the workgroups of a launch own disjoint rows x columns
//    of Z.  complex64 (k_regular_range): one workgroup per (test triangle,
//    range of 64 consecutive trial nodes), one launch per test colour, the
//    node sums held in registers over all trial triangles of the range so
//    that each entry is updated once per test triangle;
//  * singular pairs (coincident, common edge, common vertex): Sauter-Schwab
//    quadrature, 6 / 5 / 2 regions x n^4 Gauss points, two wavefronts per
//    pair, FP64;
//  * MIXED precision: far regular pairs in FP32, near regular pairs and all
//    singular pairs in FP64, everything accumulated into complex64 Z.
#include <complex>
#include <type_traits>

#include <new>

#include "mbem_internal.h"
#include "kappa.h"
#include "near_store.h"
#include "p2_device.h"
#include "ssq_map.h"

namespace mbem {

constexpr int kWave = 64;

// -------------------------------------------------------------- helpers --
__device__ inline void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add(float *p, double v) { unsafeAtomicAdd(p, (float)v); }
__device__ inline void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// Map a linear workgroup id so that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous range of tiles.
__device__ inline int64_t xcd_remap(int64_t bid, int64_t total) {
    const int64_t q = total / 8, r = total % 8;
    const int64_t xcd = bid % 8, local = bid / 8;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// ---------------------------------------------------- regular pairs ---
// One workgroup per (test triangle e, trial chunk of kChunk Morton-
// consecutive triangles); one launch per (test colour, chunk colour), so
// that the workgroups of a launch write disjoint rows x columns of Z and
// accumulate with plain read-modify-write (device-scope float atomics are
// performed beyond the L2 on this multi-die part and are far slower).
//  A: one point pair per lane (4 x 49 lanes): twelve weighted kernel values;
//  B: trial-side contraction per triangle, Tf[fs][p][j][c] = sum_q kap N_j(q);
//  C: per (row group, chunk node, beta): Ts[p] = the sum of Tf over the
//     chunk's triangles that contain the node (node merge), then the
//     test-side contraction out[i] = sum_p N_i(p) Ts[p], added to Z once per
//     (row, node) of the chunk; consecutive lanes walk along a row so that
//     the accesses of a wavefront are contiguous.
template <typename T, typename TS>
struct RegArgs {
    int64_t nt, n2, n_te, n_ch, total;
    const int32_t *te_list, *ch_list;   // this launch's colour classes
    const T *qp;            // [kQPF][nt*7]
    const double *qp64;     // FP64 table (near pairs of the mixed path)
    const int32_t *tri;
    const double *frames;   // [nn][9] nodal triads (node-attached tangents)
    const T *rtab;          // node-attached: [nt][points][6][2][2] tangent components
    const int32_t *chunks;  // kChunkRec ints per trial chunk
    const double *einfo;    // [nt][4]
    double near_r;
    int mode;               // 0: every regular pair in T; 1: pairs closer
                            // than near_r in FP64, the others in T;
                            // 3: the pairs the near mask leaves (far pairs);
                            // 4: the pairs it marks (near pairs), added to
                            // the near store
    unsigned long long *near_count;
    const uint8_t *nmask;   // modes 3, 4: [nt][n_chunks] near bits per chunk
    int64_t n_chunks;
    NearView near;          // mode 4: the FP64 near store
    const int2 *tiles;      // mode 4: this launch's (test triangle, chunk) tiles
    const KernelConst *K;   // device copy, staged in LDS by every workgroup
    const int32_t *row_map; // null, or node -> row node of a band buffer
    // FP64 dense fill: the first writer (in launch order) of an entry loads
    // nothing and stores its sum, so Z needs no clearing; first_on = 0
    // elsewhere
    const int32_t *row_first, *col_first;
    int first_on;
    TS *Z[3];
};

// Copy the kernel constants (a few hundred doubles) into LDS; every use
// after the next barrier is a uniform LDS read issued where it is needed.
__device__ __forceinline__ void stage_kconst(const KernelConst *src, KernelConst *dst, int tid, int nthr) {
    constexpr int nw = (int)(sizeof(KernelConst) / sizeof(double));
    static_assert(sizeof(KernelConst) % sizeof(double) == 0, "KernelConst is a block of doubles");
    const double *s = (const double *)src;
    double *d = (double *)dst;
    for (int i = tid; i < nw; i += nthr) d[i] = s[i];
}

// operator block op of the argument block, selected without a runtime index
// into the argument struct (which would force a private copy of it)
template <typename TS>
__device__ __forceinline__ TS *zblock(TS *const (&Z)[3], int op) {
    return op == 0 ? Z[0] : (op == 1 ? Z[1] : Z[2]);
}

template <typename T>
__device__ inline vec3<T> qload(const T *qp, int64_t nq, int f, int64_t i) {
    return {qp[(int64_t)f * nq + i], qp[(int64_t)(f + 1) * nq + i], qp[(int64_t)(f + 2) * nq + i]};
}

constexpr int kPairLanes = 49 * kChunk;   // 196

// Phase-C destinations of one workgroup: 6 row groups (op, alpha) x 2 ns
// columns (slot, beta) items, each touching the 6 rows of the test
// triangle's nodes; at most 6 x 2 x 24 items.  Their current values are
// prefetched into LDS by direct global-to-LDS loads as soon as the
// workgroup knows its tile, so the read of the read-modify-write overlaps
// the kernel evaluations.
constexpr int kItemsMax = 6 * 2 * 24;

// P2 shape functions at the points of the 7-point rule (rule7: centroid,
// then the two three-point orbits with (6 -+ sqrt 15)/21), evaluated at
// compile time: n7(q, j) = N_j(xi_q, eta_q).  The literal is sqrt(15)
// rounded to double, so the values equal those of rule7 + p2_shape.
__host__ __device__ constexpr double n7(int q, int j) {
    const double r15 = 3.8729833462074168851792653997824;
    const double s = q == 0 ? 1.0 / 3.0 : (q <= 3 ? (6.0 - r15) / 21.0 : (6.0 + r15) / 21.0);
    const int r = q == 0 ? 0 : (q - 1) % 3;
    const double xi = q == 0 ? s : (r == 1 ? 1.0 - 2.0 * s : s);
    const double eta = q == 0 ? s : (r == 2 ? 1.0 - 2.0 * s : s);
    const double L0 = 1.0 - xi - eta, L1 = xi, L2 = eta;
    return j == 0 ? L0 * (2.0 * L0 - 1.0) : j == 1 ? L1 * (2.0 * L1 - 1.0)
         : j == 2 ? L2 * (2.0 * L2 - 1.0) : j == 3 ? 4.0 * L0 * L1
         : j == 4 ? 4.0 * L1 * L2 : 4.0 * L2 * L0;
}

// out[j] = sum_q n7(q, j) v[q] through the symmetry of the rule: the three
// points of an orbit carry the same weight pattern, so with the orbit sums
// S_a = v1 + v2 + v3, S_b = v4 + v5 + v6 every vertex function is
// N(centroid) v0 + B_a S_a + B_b S_b plus (A - B) times the value at the
// orbit point nearest that vertex, and every mid-edge function
// N(centroid) v0 + E_a S_a + E_b S_b plus (F - E) times the value at the
// orbit point nearest the opposite vertex (A, B, E, F: the shape-function
// values at the orbit points).  44 real operations instead of 84.
template <typename T>
__host__ __device__ inline void contract7(const cx<T> v[7], cx<T> out[6]) {
    constexpr double c0v = n7(0, 0), c0e = n7(0, 3);
    constexpr double Ba = n7(2, 0), Bb = n7(5, 0), Da = n7(1, 0) - Ba, Db = n7(4, 0) - Bb;
    constexpr double Ea = n7(1, 3), Eb = n7(4, 3), Ga = n7(3, 3) - Ea, Gb = n7(6, 3) - Eb;
    const cx<T> Sa = v[1] + v[2] + v[3], Sb = v[4] + v[5] + v[6];
    const cx<T> V = (T)c0v * v[0] + (T)Ba * Sa + (T)Bb * Sb;
    const cx<T> E = (T)c0e * v[0] + (T)Ea * Sa + (T)Eb * Sb;
    out[0] = V + (T)Da * v[1] + (T)Db * v[4];
    out[1] = V + (T)Da * v[2] + (T)Db * v[5];
    out[2] = V + (T)Da * v[3] + (T)Db * v[6];
    out[3] = E + (T)Ga * v[3] + (T)Gb * v[6];    // edge 0-1, opposite vertex 2
    out[4] = E + (T)Ga * v[1] + (T)Gb * v[4];    // edge 1-2, opposite vertex 0
    out[5] = E + (T)Ga * v[2] + (T)Gb * v[5];    // edge 2-0, opposite vertex 1
}

// component-major kernel-value buffer: entry (c, lane) at c * kR1Stride + lane;
// the stride (= 1 mod 16) spreads consecutive components over the banks
constexpr int kR1Stride = 209;

// NODAL: node-attached tangents.  The kernel values stay in the point
// frames; the trial contraction takes the 2 x 2 components of each trial
// node's tangents in the frame of each trial point, the test contraction
// those of each test node in the frames of the test points (the kernels are
// linear in the test and in the trial vector).
// STORE (mode 4): the near pairs of a MIXED operator in FP64, their blocks
// added to the FP64 near store instead of Z (the store's slots of one
// launch are disjoint like its rows x columns).
template <typename T, typename TS, bool DK = false, bool NODAL = false, bool STORE = false>
__global__ __launch_bounds__(256) void k_regular(RegArgs<T, TS> a) {
    // point-pair kernel values; the trial-side contraction is later written
    // over them in place
    __shared__ cx<T> s_r1[12 * kR1Stride];
    // NODAL: s_ra[p][i][alpha][gamma] = N_i(x_p) t_alpha,i . t_gamma(x_p) of
    // the test triangle, s_rb[fs][q][j][beta][delta] likewise for the trial
    // triangles of the chunk
    __shared__ T s_ra[NODAL ? 168 : 1];
    __shared__ T s_rb[NODAL ? kChunk * 168 : 1];
    // prefetched destination values.  FP32: in LDS by direct global-to-LDS
    // loads, plane (i, re / im) (i: row of the test triangle), item it.
    // FP64: in registers (pre), which keeps the LDS of a workgroup low enough
    // for three workgroups per compute unit.
    constexpr bool kF64 = std::is_same<TS, double>::value;
    __shared__ __align__(16) TS s_dst[kF64 ? 1 : 2 * 6 * kItemsMax];
    constexpr int kRounds = (kItemsMax + 255) / 256;
    double2 pre[kF64 ? kRounds : 1][6];
    __shared__ int64_t s_row[6][6];    // [2 op + alpha][i]: offset of row 2 te_i + alpha
    __shared__ int32_t s_rec[kChunkRec];
    __shared__ int s_act[kChunk];      // 0 skip, 1 compute in T, 2 in FP64
    __shared__ KernelConst s_K;
    const int tid = threadIdx.x;
    stage_kconst(a.K, &s_K, tid, blockDim.x);
    const int64_t tile = xcd_remap(blockIdx.x, a.total);
    const int64_t e = STORE ? a.tiles[tile].x : a.te_list[tile / a.n_ch];
    const int64_t ch = STORE ? a.tiles[tile].y : a.ch_list[tile % a.n_ch];
    for (int i = tid; i < kChunkRec; i += blockDim.x) s_rec[i] = a.chunks[ch * kChunkRec + i];
    if (tid < 36) {
        const int g = tid / 6, i = tid % 6;
        int64_t node = a.tri[6 * e + i];
        if (a.row_map) node = a.row_map[node];
        s_row[g][i] = 2 * (2 * node + (g & 1)) * a.n2;
    }
    if (tid < kChunk) {
        const int64_t f = ch * kChunk + tid;
        bool act = f < a.nt;
        if (act) {
            const int32_t *te = a.tri + 6 * e, *tf = a.tri + 6 * f;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) act = act && (te[i] != tf[j]);
        }
        int kind = act ? 1 : 0;
        if (act && a.mode == 1) {
            const double *ce = a.einfo + 4 * e, *cf = a.einfo + 4 * f;
            const double dx = ce[0] - cf[0], dy = ce[1] - cf[1], dz = ce[2] - cf[2];
            if (sqrt(dx * dx + dy * dy + dz * dz) - ce[3] - cf[3] < a.near_r) {
                kind = 2;
                atomicAdd(a.near_count, 1ull);
            }
        }
        if (act && a.mode >= 3) {
            // one classification for both launches: the near mask
            const bool near = (a.nmask[e * a.n_chunks + ch] >> tid) & 1;
            kind = (a.mode == 3) != near ? 1 : 0;
        }
        s_act[tid] = kind;
    }
    const int64_t nq = a.nt * kQP;
    if constexpr (NODAL) {
        // the test triangle's and the chunk's rows of the precomputed table
        for (int it = tid; it < (kChunk + 1) * 168; it += blockDim.x) {
            const int side = it / 168, r = it % 168;          // side 0: test, 1 + fs: trial
            const int64_t el = side == 0 ? e : ch * kChunk + side - 1;
            const T v = el < a.nt ? a.rtab[el * 168 + r] : (T)0;
            if (side == 0) s_ra[r] = v;
            else s_rb[(side - 1) * 168 + r] = v;
        }
    }
    // point data of this lane's pair, loaded before the barrier so that the
    // loads overlap those of the chunk record
    const int fsl = tid / 49, pl = (tid % 49) / 7, ql = tid % 7;
    const int64_t ix = e * kQP + pl, iy = (ch * kChunk + fsl) * kQP + ql;
    vec3<T> x = {0, 0, 0}, n = {0, 0, 0}, y = {0, 0, 0};
    vec3<T> ta[2] = {x, x}, sa[2] = {x, x}, tb[2] = {x, x};
    T ww = 0;
    if (tid < kPairLanes && ch * kChunk + fsl < a.nt) {
        x = qload(a.qp, nq, QX, ix);
        n = qload(a.qp, nq, QN, ix);
        ta[0] = qload(a.qp, nq, QT1, ix);
        ta[1] = qload(a.qp, nq, QT2, ix);
        sa[0] = qload(a.qp, nq, QS1, ix);
        sa[1] = qload(a.qp, nq, QS2, ix);
        y = qload(a.qp, nq, QX, iy);
        tb[0] = qload(a.qp, nq, QT1, iy);
        tb[1] = qload(a.qp, nq, QT2, iy);
        ww = a.qp[(int64_t)QW * nq + ix] * a.qp[(int64_t)QW * nq + iy];
    }
    __syncthreads();
    int any = 0;
#pragma unroll
    for (int k = 0; k < kChunk; ++k) any |= s_act[k];
    // uniform over the workgroup; a first writer still stores its zeros
    if (!any && !a.first_on) return;
    const int rfirst = a.first_on ? a.row_first[e] : 0, cfirst = a.first_on ? a.col_first[ch] : 0;
    const int ns = s_rec[0];
    const int rowlen = 2 * ns;
    const int nitems = 6 * rowlen;
    // item it -> row group g = it / rowlen through a float reciprocal: the
    // exact quotient (it + 1/2) / rowlen is at least 1/(2 rowlen) > 0.01 away
    // from an integer for it < 6 rowlen <= 288, far beyond float rounding
    const float inv_rowlen = 1.0f / (float)rowlen;
    // item it: row group g = 2 op + alpha, slot sl, beta; destination of
    // row i of the test triangle: Z[op][2 te_i + alpha][2 node(sl) + beta].
    // No other workgroup of this launch touches these entries (colour
    // classes), and earlier launches completed in stream order.
    if constexpr (!STORE) {
        const int wave = tid / 64;
#pragma unroll
        for (int k = 0; k < kRounds; ++k) {
            const int base = 256 * k, it = base + tid;
            const bool on = it < nitems;
            const int itc = on ? it : 0;
            const int g = (int)(((float)itc + 0.5f) * inv_rowlen);
            const int rem = itc - g * rowlen;
            const int sl = rem >> 1, be = rem & 1, op = g >> 1;
            const int64_t col = 2 * (2 * (int64_t)s_rec[1 + sl] + be);
            const TS *Z = zblock(a.Z, op) + col;
            const int first = base + wave * 64;        // wave-uniform item of lane 0
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const TS *src = Z + s_row[g][i];
                if constexpr (kF64) {
                    const bool first = ((rfirst >> i) & (cfirst >> sl) & 1) != 0;
                    pre[k][i] = double2{0.0, 0.0};
                    if (on && !first) pre[k][i] = *(const double2 *)src;
                } else {
                    TS *dre = s_dst + (2 * i) * kItemsMax + first, *dim = s_dst + (2 * i + 1) * kItemsMax + first;
                    if (on) {
                        __builtin_amdgcn_global_load_lds((const void *)src,
                                                         (__attribute__((address_space(3))) void *)dre, 4, 0, 0);
                        __builtin_amdgcn_global_load_lds((const void *)(src + 1),
                                                         (__attribute__((address_space(3))) void *)dim, 4, 0, 0);
                    }
                }
            }
        }
    }
    // A: kernel values
    if (tid < kPairLanes) {
        cx<T> k[12];
        const int kind = s_act[fsl];
        if (kind == 1) {
            kappa12<T, DK>(s_K, x, n, ta, sa, y, tb, ww, k);
        } else if (!std::is_same<T, double>::value && kind == 2) {
            // near pair: FP64 kernel differences (cancellation), then rounded
            const double *q64 = a.qp64;
            const dvec3 x = qload(q64, nq, QX, ix), n = qload(q64, nq, QN, ix);
            const dvec3 ta[2] = {qload(q64, nq, QT1, ix), qload(q64, nq, QT2, ix)};
            const dvec3 sa[2] = {qload(q64, nq, QS1, ix), qload(q64, nq, QS2, ix)};
            const dvec3 y = qload(q64, nq, QX, iy);
            const dvec3 tb[2] = {qload(q64, nq, QT1, iy), qload(q64, nq, QT2, iy)};
            const double ww = q64[(int64_t)QW * nq + ix] * q64[(int64_t)QW * nq + iy];
            cx<double> kd[12];
            kappa12<double, DK>(s_K, x, n, ta, sa, y, tb, ww, kd);
#pragma unroll
            for (int c = 0; c < 12; ++c) k[c] = cx<T>{(T)kd[c].re, (T)kd[c].im};
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) k[c] = cx<T>{0, 0};
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) s_r1[c * kR1Stride + tid] = k[c];
    }
    __syncthreads();
    // B: trial side per triangle, in place: Tf[c][fs][p][j] = sum_q N_j(q) k
    // over the 7 entries (c, fs, p, q = 0..6) it replaces (j = 0..5)
    if constexpr (!NODAL) {
        for (int it = tid; it < 12 * kChunk * 7; it += blockDim.x) {
            const int c = it / (kChunk * 7), fp = it % (kChunk * 7);   // fp = 7 fs + p
            cx<T> *row = s_r1 + c * kR1Stride + 7 * fp;
            cx<T> kv[7], tf[6];
#pragma unroll
            for (int q = 0; q < 7; ++q) kv[q] = row[q];
            contract7(kv, tf);
#pragma unroll
            for (int j = 0; j < 6; ++j) row[j] = tf[j];
        }
    } else {
        // the two delta components of (op, gamma) become the two beta ones:
        // Tf[op,gamma,beta][fs][p][j] = sum_q sum_delta s_rb[fs][q][j][beta][delta] k[op,gamma,delta]
        for (int it = tid; it < 6 * kChunk * 7; it += blockDim.x) {
            const int og = it / (kChunk * 7), fp = it % (kChunk * 7);   // og = 2 op + gamma
            cx<T> *r0 = s_r1 + (2 * og) * kR1Stride + 7 * fp, *r1 = r0 + kR1Stride;
            const T *rb = s_rb + (fp / 7) * 168;
            cx<T> k0[7], k1[7];
#pragma unroll
            for (int q = 0; q < 7; ++q) { k0[q] = r0[q]; k1[q] = r1[q]; }
            // every input is in registers: each output may overwrite its slot
            // (three j at a time: unrolled fully, the weight loads of all j
            // would be hoisted and the FP64 kernel would run at one wave per
            // SIMD)
#pragma unroll 3
            for (int j = 0; j < 6; ++j) {
                cx<T> o0 = {0, 0}, o1 = {0, 0};
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    const T *w = rb + (q * 6 + j) * 4;
                    o0 = o0 + w[0] * k0[q] + w[1] * k1[q];
                    o1 = o1 + w[2] * k0[q] + w[3] * k1[q];
                }
                r0[j] = o0;
                r1[j] = o1;
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);             // prefetched destinations have landed (FP32)
    __syncthreads();
    // C: test side, lanes along (slot, beta) of one (op, alpha) row group;
    // the chunk's triangles that share the slot's node are summed here
    // (node merge): Ts[p] = sum over incidences (fs, loc) of Tf[fs][p][loc]
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        const int it = 256 * k + tid;
        if (it >= nitems) break;
        const int g = (int)(((float)it + 0.5f) * inv_rowlen);    // g = 2 op + alpha
        const int rem = it - g * rowlen;
        const int sl = rem >> 1, be = rem & 1, op = g >> 1;
        const int u1 = s_rec[26 + sl];
        cx<T> out[6];
        if constexpr (!NODAL) {
            const int c = 2 * g + be;                            // 4 op + 2 alpha + beta
            cx<T> tv[7];
#pragma unroll
            for (int p = 0; p < 7; ++p) tv[p] = cx<T>{0, 0};
            for (int u = s_rec[25 + sl]; u < u1; ++u) {
                const int fl = s_rec[50 + u];
                const cx<T> *src = s_r1 + c * kR1Stride + (fl >> 3) * 49 + (fl & 7);
#pragma unroll
                for (int p = 0; p < 7; ++p) tv[p] = tv[p] + src[7 * p];
            }
            contract7(tv, out);
        } else {
            // components (op, gamma, beta) for gamma = 0, 1 at 4 op + beta and
            // 4 op + 2 + beta; out[i] = sum_p sum_gamma s_ra[p][i][alpha][gamma] Ts[gamma][p]
            // (point-major, so that only the six outputs stay live)
            const int al = g & 1;
            const int c0 = 4 * op + be;
            const int u0 = s_rec[25 + sl];
#pragma unroll
            for (int i = 0; i < 6; ++i) out[i] = cx<T>{0, 0};
#pragma unroll 1
            for (int p = 0; p < 7; ++p) {
                cx<T> t0 = {0, 0}, t1 = {0, 0};
                for (int u = u0; u < u1; ++u) {
                    const int fl = s_rec[50 + u];
                    const cx<T> *src0 = s_r1 + c0 * kR1Stride + (fl >> 3) * 49 + (fl & 7) + 7 * p;
                    t0 = t0 + src0[0];
                    t1 = t1 + src0[2 * kR1Stride];
                }
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    const T *w = s_ra + (p * 6 + i) * 4 + 2 * al;
                    out[i] = out[i] + w[0] * t0 + w[1] * t1;
                }
            }
        }
        if constexpr (STORE) {
            // only node pairs of a computed (near) element pair are in the
            // store's pattern: skip slots whose triangles were all skipped
            bool touched = false;
            for (int u = s_rec[25 + sl]; u < u1; ++u) touched = touched || s_act[s_rec[50 + u] >> 3] != 0;
            if (!touched) continue;
            const int64_t nj = s_rec[1 + sl];
            const int c = 4 * op + 2 * (g & 1) + be;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                double2 *v = a.near.val + 12 * near_slot(a.near, a.tri[6 * e + i], nj) + c;
                v->x += (double)out[i].re;
                v->y += (double)out[i].im;
            }
            continue;
        }
        TS *Z = zblock(a.Z, op) + 2 * (2 * (int64_t)s_rec[1 + sl] + be);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const cx<T> acc = out[i];
            TS *dst = Z + s_row[g][i];
            TS ore, oim;
            if constexpr (kF64) {
                ore = pre[k][i].x;
                oim = pre[k][i].y;
            } else {
                ore = s_dst[(2 * i) * kItemsMax + it];
                oim = s_dst[(2 * i + 1) * kItemsMax + it];
            }
            dst[0] = ore + (TS)acc.re;         // race-free: see the colouring above
            dst[1] = oim + (TS)acc.im;
        }
    }
}

// ------------------------------------ regular pairs by column range ---
// One workgroup per (test triangle e, range J of consecutive trial nodes);
// one launch per test colour, so that the workgroups of a launch write
// disjoint rows (test colour) x columns (ranges) of Z.  The workgroup walks
// the trial triangles that touch J in batches:
//  A: one point pair per lane: twelve weighted kernel values (as k_regular);
//  B: trial-side contraction per triangle, in place (as k_regular);
//  C: every lane owns one (node j of J, beta) and OWN row groups
//     g = 2 op + alpha, and adds the batch's incidences of j to its OWN x 7
//     point sums Y[g][p] += Tf[2 g + beta][f][p][loc] (node merge);
// after the last batch the lanes contract their sums with the test shape
// functions and add them to Z: each entry of the workgroup's 6 x 6 rows
// and 2 |J| columns is read and written once, in runs of 2 |J| consecutive
// entries per row.  A triangle touching several ranges is evaluated once
// per range (about 1.7 times on average for ranges of 64 nodes of a
// Morton-ordered mesh); in exchange the trial chunks' colours and their
// separate read-modify-write passes over Z are gone.
//   mode 0: every regular pair;
//   mode 1: complex64 operator without a near store: far pairs in FP32,
//           near pairs with their distance and kernel scalars (where the
//           two media's terms cancel) in FP64, rounded, and the rest of
//           their kernel values in FP32;
//   mode 3: the pairs the near mask leaves (the far pairs, with a store).
template <typename T, typename TS>
struct RngArgs {
    int64_t nt, n2, nn, n_te, nrng, total;
    const int32_t *te_list;     // this launch's test colour class
    const T *qp;                // [kQPF][nt*7]
    const double *qp64;         // FP64 table (near pairs of mode 1)
    const int32_t *tri;
    const int32_t *rng_off, *rng_rec;
    const int32_t *row_first;   // per triangle: bit a set = first writer of node a's rows
    const double *einfo;        // [nt][4]
    double near_r;
    int mode;
    unsigned long long *near_count;
    const uint8_t *nmask;       // mode 3: [nt][n_chunks] near bits
    int64_t n_chunks;
    const KernelConst *K;
    TS *Z[3];
};

template <int NB>
struct RngStride {
    static constexpr int v = ((49 * NB + 14) / 16) * 16 + 1;   // >= 49 NB, = 1 mod 16
};

template <typename T, typename TS, int THREADS, int WAVES, bool NEAR>
__global__ __launch_bounds__(THREADS, WAVES) void k_regular_range(RngArgs<T, TS> a) {
    constexpr RngLayout L = kRng;
    constexpr int NB = L.nb, RNG = L.rng;
    constexpr int OWN = 12 * RNG / THREADS;        // row groups per lane
    constexpr int STR = RngStride<NB>::v;
    static_assert(OWN * THREADS == 12 * RNG && 6 % OWN == 0, "lanes own whole row groups");
    static_assert(!NEAR || !std::is_same<T, double>::value, "near pairs are the complex64 fill's");
    static_assert(49 * NB <= THREADS, "one point pair per lane");
    __shared__ cx<T> s_r1[12 * STR];
    __shared__ T s_tp[kQPF * kQP];       // the test triangle's point table, field-major
    __shared__ int32_t s_rec[L.rec()];
    __shared__ int32_t s_te[6];
    __shared__ KernelConst s_K;
    const int tid = threadIdx.x;
    const int64_t tile = xcd_remap(blockIdx.x, a.total);
    const int64_t e = a.te_list[tile / a.nrng];
    const int64_t r = tile % a.nrng;
    stage_kconst(a.K, &s_K, tid, THREADS);
    const int64_t nq = a.nt * kQP;
    if (tid < kQPF * kQP) s_tp[tid] = a.qp[(int64_t)(tid / kQP) * nq + e * kQP + tid % kQP];
    if (tid < 6) s_te[tid] = a.tri[6 * e + tid];
    // C and the updates of Z: lane (jl, be) of the range, row groups g0 ..
    const int jl = (tid % (2 * RNG)) >> 1, be = tid & 1, g0 = OWN * (tid / (2 * RNG));
    const int64_t jglob = r * RNG + jl;
    // A: this lane's point pair (batch-local triangle fsl, test point pl,
    // trial point ql)
    const int fsl = tid / 49, pl = (tid % 49) / 7, ql = tid % 7;
    const int32_t b0 = a.rng_off[r], b1 = a.rng_off[r + 1];

    // batch b into s_rec; returns its number of triangles
    auto batch = [&](int32_t b) -> int {
        __syncthreads();                  // the previous batch is done with s_r1 and s_rec
        if (tid < L.rec()) s_rec[tid] = a.rng_rec[(int64_t)b * L.rec() + tid];
        __syncthreads();
        return s_rec[0];
    };
    // kind of the pair (e, f), evaluated by each of its 49 lanes: 0 skip
    // (shares a vertex with e, or mode 3 and near), 1 regular pair in T,
    // 2 near pair (mode 1; counted once, by the lane `count`, in the range
    // of f's first vertex)
    auto pair_kind = [&](int64_t f, bool count) -> int {
        const int32_t *tf = a.tri + 6 * f;
        bool act = true;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) act = act && (s_te[i] != tf[j]);
        if (!act) return 0;
        if (a.mode == 1) {
            const double *ce = a.einfo + 4 * e, *cf = a.einfo + 4 * f;
            const double dx = ce[0] - cf[0], dy = ce[1] - cf[1], dz = ce[2] - cf[2];
            if (sqrt(dx * dx + dy * dy + dz * dz) - ce[3] - cf[3] < a.near_r) {
                if (count && tf[0] / RNG == r) atomicAdd(a.near_count, 1ull);
                return 2;
            }
        }
        if (a.mode == 3 && ((a.nmask[e * a.n_chunks + f / kChunk] >> (f % kChunk)) & 1)) return 0;
        return 1;
    };
    // B: Tf[c][fs][p][j] = sum_q N_j(q) k, in place over (c, fs, p)
    auto trial_side = [&](int nbt) {
        __syncthreads();
        for (int it = tid; it < 12 * 7 * nbt; it += THREADS) {
            const int c = it / (7 * nbt), fp = it % (7 * nbt);
            cx<T> *row = s_r1 + c * STR + 7 * fp;
            cx<T> kv[7], tfv[6];
#pragma unroll
            for (int q = 0; q < 7; ++q) kv[q] = row[q];
            contract7(kv, tfv);
#pragma unroll
            for (int j = 0; j < 6; ++j) row[j] = tfv[j];
        }
        __syncthreads();
    };
    // C: the batch's incidences of this lane's node into sums v
    auto merge = [&](cx<T> (&v)[OWN][7]) {
        const int u1 = s_rec[L.off() + jl + 1];
        for (int u = s_rec[L.off() + jl]; u < u1; ++u) {
            const int fl = s_rec[L.inc() + u];
            const cx<T> *src = s_r1 + (fl >> 3) * 49 + (fl & 7) + (2 * g0 + be) * STR;
#pragma unroll
            for (int k = 0; k < OWN; ++k)
#pragma unroll
                for (int p = 0; p < 7; ++p) v[k][p] = v[k][p] + src[2 * k * STR + 7 * p];
        }
    };
    // test side: out[i] = sum_p N_i(p) v[g][p], added to row 2 te_i + alpha,
    // column 2 j + beta of block op, or stored there by the first test
    // triangle (in colour order) of node te_i: every workgroup writes all
    // its rows x columns, so Z needs no clearing before the fill.  No other
    // workgroup of this launch touches these entries; earlier launches
    // completed in stream order.
    const int first = a.row_first[e];
    auto add_to_z = [&](const cx<T> (&v)[OWN][7]) {
#pragma unroll
        for (int k = 0; k < OWN; ++k) {
            const int g = g0 + k, op = g >> 1, al = g & 1;
            cx<T> out[6];
            contract7(v[k], out);
            TS *Z = zblock(a.Z, op) + 2 * (2 * jglob + be);
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                TS *dst = Z + 2 * (2 * (int64_t)s_te[i] + al) * a.n2;
                if ((first >> i) & 1) {
                    dst[0] = (TS)out[i].re;
                    dst[1] = (TS)out[i].im;
                } else {
                    dst[0] += (TS)out[i].re;
                    dst[1] += (TS)out[i].im;
                }
            }
        }
    };

    cx<T> Y[OWN][7];
#pragma unroll
    for (int k = 0; k < OWN; ++k)
#pragma unroll
        for (int p = 0; p < 7; ++p) Y[k][p] = cx<T>{0, 0};
    for (int32_t b = b0; b < b1; ++b) {
        const int nbt = batch(b);
        if (tid < 49 * nbt) {
            cx<T> k[12];
            const int64_t f = s_rec[1 + fsl];
            const int kind = pair_kind(f, pl == 0 && ql == 0);
            if (kind != 0) {
                const int64_t iy = f * kQP + ql;
                const T *tp = s_tp + pl;
                const vec3<T> n = {tp[QN * kQP], tp[(QN + 1) * kQP], tp[(QN + 2) * kQP]};
                const vec3<T> ta[2] = {{tp[QT1 * kQP], tp[(QT1 + 1) * kQP], tp[(QT1 + 2) * kQP]},
                                       {tp[QT2 * kQP], tp[(QT2 + 1) * kQP], tp[(QT2 + 2) * kQP]}};
                const vec3<T> sa[2] = {{tp[QS1 * kQP], tp[(QS1 + 1) * kQP], tp[(QS1 + 2) * kQP]},
                                       {tp[QS2 * kQP], tp[(QS2 + 1) * kQP], tp[(QS2 + 2) * kQP]}};
                const vec3<T> tb[2] = {qload(a.qp, nq, QT1, iy), qload(a.qp, nq, QT2, iy)};
                const T ww = tp[QW * kQP] * a.qp[(int64_t)QW * nq + iy];
                KScal<T> sc;
                vec3<T> Rh;
                if (NEAR && kind == 2) {
                    // near pair: the distance and the kernel scalars (whose
                    // two media's terms cancel) in FP64, then rounded
                    const dvec3 Rv = qload(a.qp64, nq, QX, e * kQP + pl) - qload(a.qp64, nq, QX, iy);
                    const double R = sqrt(dot(Rv, Rv));
                    const dvec3 u = (1.0 / R) * Rv;
                    Rh = {(T)u.x, (T)u.y, (T)u.z};
                    const KScal<double> sd = kernel_scalars<double>(s_K, R);
                    sc = {cx<T>{(T)sd.D0.re, (T)sd.D0.im}, cx<T>{(T)sd.df.re, (T)sd.df.im},
                          cx<T>{(T)sd.dg.re, (T)sd.dg.im}, cx<T>{(T)sd.Ge.re, (T)sd.Ge.im},
                          cx<T>{(T)sd.Gm.re, (T)sd.Gm.im}};
                } else {
                    const vec3<T> x = {tp[QX * kQP], tp[(QX + 1) * kQP], tp[(QX + 2) * kQP]};
                    const vec3<T> Rv = x - qload(a.qp, nq, QX, iy);
                    const T R = sqrt(dot(Rv, Rv));
                    Rh = ((T)1 / R) * Rv;
                    sc = kernel_scalars<T>(s_K, R);
                }
                kappa_combine<T>(sc, Rh, n, ta, sa, tb, ww, k);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) k[c] = cx<T>{0, 0};
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) s_r1[c * STR + tid] = k[c];
        }
        trial_side(nbt);
        merge(Y);
    }
    if (jglob < a.nn) add_to_z(Y);
}

// --------------------------------------------- Sauter-Schwab pairs ---
// (maps of the four-dimensional rule: ssq_map.h)

template <typename TS>
struct SsqArgs {
    int64_t n2, npairs;
    const int32_t *pairs;   // e, f, class, perm codes
    const int32_t *tri;
    const double *xyz, *frames;
    int order;
    double glx[kMaxSSQ], glw[kMaxSSQ];   // Gauss-Legendre on [0,1]
    const KernelConst *K;   // device copy
    const int32_t *row_map; // null, or node -> row node of a band buffer
    TS *Z[3];
    NearView near;          // MIXED with the near store: added there in FP64
};

// Two wavefronts per pair.  Every lane evaluates one quadrature point per
// batch (kernel values and the six test / trial shape functions) into LDS;
// then 120 consumer lanes, one real component (2 c + re/im) of the twelve
// kernel values each, split the batch's points into kStreams interleaved
// streams and accumulate the 6 x 6 outer products N_i(x) N_j(y) kappa in
// registers.  The streams are summed through the same LDS buffer at the end.
constexpr int kSsqThreads = 128;
constexpr int kStreams = 5;
constexpr int kPtStride = 37;   // 24 kernel reals, N_i(x), N_j(y); padded
// node-attached tangents: 24 kernel reals, then per test node i the 2 x 2
// N_i(x) t_alpha,i . t_gamma(x) and per trial node j N_j(y) t_beta,j . t_delta(y)
constexpr int kPtStrideNodal = 73;

// Launch shape of the singular-pair kernels.  NODAL: rows of 73 doubles put
// 75 KB of LDS on a workgroup (two per compute unit), and the 2 x 2
// contractions make the consumers the larger part: four wavefronts per
// workgroup, the first two producing, all of them consuming (ten streams).
template <bool NODAL>
struct SsqShape {
    static constexpr int threads = NODAL ? 2 * kSsqThreads : kSsqThreads;
    static constexpr int streams = NODAL ? 2 * kStreams : kStreams;
    static constexpr int stride = NODAL ? kPtStrideNodal : kPtStride;
    static_assert(streams * 36 * 24 <= kSsqThreads * stride, "reduction buffer");
};

// NODAL: the tangents of the two triangles' nodes, s_tn[side][k][b][3]
__device__ __forceinline__ void ssq_stage_tangents(const double *frames, const int32_t *tri, int32_t e,
                                                   int32_t f, double *s_tn, int tid) {
    if (tid < 72) {
        const int side = tid / 36, r = tid % 36, k = r / 6, b = (r / 3) % 2, d = r % 3;
        s_tn[tid] = frames[9 * (int64_t)tri[6 * (side ? f : e) + k] + 3 + 3 * b + d];
    }
}

// One LDS row: the twelve kernel values, then the shape data of the point
// pair (shape functions, or with node-attached tangents their products
// with the nodal tangents' components in the two point frames).
template <bool NODAL>
__device__ __forceinline__ void ssq_row(double *pt, const cx<double> k[12], const P2Point &X, const P2Point &Y,
                                        const double *s_tn) {
#pragma unroll
    for (int q = 0; q < 12; ++q) { pt[2 * q] = k[q].re; pt[2 * q + 1] = k[q].im; }
    if constexpr (!NODAL) {
#pragma unroll
        for (int q = 0; q < 6; ++q) { pt[24 + q] = X.N[q]; pt[30 + q] = Y.N[q]; }
    } else {
        const dvec3 tx[2] = {X.t1, X.t2}, ty[2] = {Y.t1, Y.t2};
#pragma unroll
        for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const double *ue = s_tn + 6 * q + 3 * b, *uf = s_tn + 36 + 6 * q + 3 * b;
                const dvec3 te = {ue[0], ue[1], ue[2]}, tf = {uf[0], uf[1], uf[2]};
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    pt[24 + 4 * q + 2 * b + g] = X.N[q] * dot(te, tx[g]);
                    pt[48 + 4 * q + 2 * b + g] = Y.N[q] * dot(tf, ty[g]);
                }
            }
    }
}

// Consumer lane (component comp = 2 c + re/im, stream): accumulate its
// stream's rows of the batch into acc[i][j].
template <bool NODAL>
__device__ __forceinline__ void ssq_consume(const double *s_pt, int stream, int comp, double acc[36]) {
    using Sh = SsqShape<NODAL>;
    if constexpr (!NODAL) {
        for (int r = stream; r < kSsqThreads; r += Sh::streams) {
            const double *row = s_pt + r * Sh::stride;
            const double kv = row[comp];
            double u[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) u[j] = row[30 + j] * kv;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const double nx = row[24 + i];
#pragma unroll
                for (int j = 0; j < 6; ++j) acc[6 * i + j] += nx * u[j];
            }
        }
    } else {
        // lane (c = 4 op + 2 alpha + beta, re / im): acc[i][j] +=
        // sum_{gamma,delta} A_i[alpha][gamma] B_j[beta][delta] k[op,gamma,delta]
        const int c = comp >> 1, ri = comp & 1;
        const int op = c >> 2, al = (c >> 1) & 1, be = c & 1;
        for (int r = stream; r < kSsqThreads; r += Sh::streams) {
            const double *row = s_pt + r * Sh::stride;
            const double k00 = row[2 * (4 * op) + ri], k01 = row[2 * (4 * op + 1) + ri];
            const double k10 = row[2 * (4 * op + 2) + ri], k11 = row[2 * (4 * op + 3) + ri];
            double u0[6], u1[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                const double b0 = row[48 + 4 * j + 2 * be], b1 = row[48 + 4 * j + 2 * be + 1];
                u0[j] = b0 * k00 + b1 * k01;
                u1[j] = b0 * k10 + b1 * k11;
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const double a0 = row[24 + 4 * i + 2 * al], a1 = row[24 + 4 * i + 2 * al + 1];
#pragma unroll
                for (int j = 0; j < 6; ++j) acc[6 * i + j] += a0 * u0[j] + a1 * u1[j];
            }
        }
    }
}

// Sum the consumer streams through LDS in a fixed order and add the pair's
// 6 x 6 x 12 block to Z (atomics: a node pair collects several element pairs).
template <typename TS, bool NODAL>
__device__ __forceinline__ void ssq_flush(const SsqArgs<TS> &a, int32_t e, int32_t f, double *s_pt,
                                          const double acc[36], int tid) {
    using Sh = SsqShape<NODAL>;
    const int comp = tid % 24, stream = tid / 24;
    if (tid < 24 * Sh::streams) {
#pragma unroll
        for (int k = 0; k < 36; ++k) s_pt[(stream * 36 + k) * 24 + comp] = acc[k];
    }
    __syncthreads();
    const int32_t *te = a.tri + 6 * e, *tf = a.tri + 6 * f;
    for (int it = tid; it < 36 * 12; it += Sh::threads) {
        const int k = it / 12, cc = it % 12;
        double re = 0, im = 0;
#pragma unroll
        for (int s = 0; s < Sh::streams; ++s) {
            re += s_pt[(s * 36 + k) * 24 + 2 * cc];
            im += s_pt[(s * 36 + k) * 24 + 2 * cc + 1];
        }
        const int i = k / 6, j = k % 6;
        const int op = cc / 4, al = (cc / 2) % 2, be = cc % 2;
        if (a.near.bits) {
            // every node pair of a singular element pair is in the pattern
            double *dst = (double *)(a.near.val + 12 * near_slot(a.near, te[i], tf[j]) + cc);
            atomic_add(dst, re);
            atomic_add(dst + 1, im);
            continue;
        }
        const int64_t tn = a.row_map ? a.row_map[te[i]] : te[i];
        const int64_t row = 2 * tn + al, col = 2 * (int64_t)tf[j] + be;
        TS *dst = zblock(a.Z, op) + 2 * (row * a.n2 + col);
        atomic_add(dst, re);
        atomic_add(dst + 1, im);
    }
}

template <typename TS, bool DK = false, bool NODAL = false>
__global__ __launch_bounds__(SsqShape<NODAL>::threads) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_ssq(SsqArgs<TS> a) {
    using Sh = SsqShape<NODAL>;
    __shared__ double s_pt[kSsqThreads * Sh::stride];
    __shared__ double s_tn[NODAL ? 72 : 1];
    const int tid = threadIdx.x;
    const int64_t pid = blockIdx.x;
    const int32_t e = a.pairs[4 * pid], f = a.pairs[4 * pid + 1];
    if constexpr (NODAL) {
        ssq_stage_tangents(a.frames, a.tri, e, f, s_tn, tid);
        __syncthreads();
    }
    const int cls = a.pairs[4 * pid + 2], code = a.pairs[4 * pid + 3];
    const int n = a.order, n4 = n * n * n * n;
    const int nreg = cls == 3 ? 6 : (cls == 2 ? 5 : 2);
    const int npts = nreg * n4;
    const int comp = tid % 24, stream = tid / 24;    // consumer role
    const bool consumer = tid < 24 * Sh::streams;
    double acc[36];
#pragma unroll
    for (int k = 0; k < 36; ++k) acc[k] = 0.0;
    for (int base = 0; base < npts; base += kSsqThreads) {
        const int idx = base + tid;
        if (tid < kSsqThreads) {
            double *pt = s_pt + tid * Sh::stride;
            if (idx < npts) {
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
                P2Point X, Y;
                p2_point(a.xyz, a.frames, a.tri + 6 * e, xe, ye, X);
                p2_point(a.xyz, a.frames, a.tri + 6 * f, xf, yf, Y);
                const dvec3 ta[2] = {X.t1, X.t2}, sa[2] = {X.s1, X.s2}, tb[2] = {Y.t1, Y.t2};
                cx<double> k[12];
                kappa12<double, DK>(*a.K, X.x, X.n, ta, sa, Y.x, tb, wg * X.J * Y.J, k);
                ssq_row<NODAL>(pt, k, X, Y, s_tn);
            } else {
#pragma unroll
                for (int q = 0; q < (NODAL ? 72 : 36); ++q) pt[q] = 0.0;
            }
        }
        __syncthreads();
        if (consumer) ssq_consume<NODAL>(s_pt, stream, comp, acc);
        __syncthreads();
    }
    ssq_flush<TS, NODAL>(a, e, f, s_pt, acc, tid);
}

// ------------------------------------- the paper's own scheme ---
// Regular pairs on the 12-point rule (144 point pairs per element pair) and
// singular pairs as Sauter-Schwab on kappa^s plus the 12-point rule on the
// remainder kappa - kappa^s.  Same tiles, colour classes and chunk records
// as k_regular; the chunk's four trial triangles are taken one at a time:
//  A: 144 lanes, one point pair each: kernel values into s_k[c][pair];
//  B: 144 lanes (c, p): the trial-side contraction of the 12 values of
//     (c, p) into s_tf[c][fs][p][j];
//  C: as in k_regular, with the test-side contraction over 12 points.
constexpr int kPP12 = kQP12 * kQP12;
constexpr int kK12Stride = 145;     // = 1 mod 16: consecutive components spread over the banks

__host__ __device__ constexpr double n12(int q, int j) {
    const double L0 = r12_bary(q, 0), L1 = r12_bary(q, 1), L2 = r12_bary(q, 2);
    return j == 0 ? L0 * (2.0 * L0 - 1.0) : j == 1 ? L1 * (2.0 * L1 - 1.0)
         : j == 2 ? L2 * (2.0 * L2 - 1.0) : j == 3 ? 4.0 * L0 * L1
         : j == 4 ? 4.0 * L1 * L2 : 4.0 * L2 * L0;
}

template <typename T>
__device__ __forceinline__ void contract12(const cx<T> v[kQP12], cx<T> out[6]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        cx<T> acc = {0, 0};
#pragma unroll
        for (int q = 0; q < kQP12; ++q) acc = acc + (T)n12(q, j) * v[q];
        out[j] = acc;
    }
}

template <typename T, typename TS, bool NODAL = false>
__global__ __launch_bounds__(256) void k_regular12(RegArgs<T, TS> a) {
    __shared__ cx<T> s_k[12 * kK12Stride];
    __shared__ cx<T> s_tf[12 * kChunk * kQP12 * 6];   // [c][fs][p][j]
    // NODAL (node-attached tangents, as k_regular): s_ra[p][i][alpha][gamma]
    // = N_i(x_p) t_alpha,i . t_gamma(x_p), s_rb[fs][q][j][beta][delta] likewise
    constexpr int kR12 = kQP12 * 24;
    __shared__ T s_ra[NODAL ? kR12 : 1];
    __shared__ T s_rb[NODAL ? kChunk * kR12 : 1];
    constexpr bool kF64 = std::is_same<TS, double>::value;
    __shared__ __align__(16) TS s_dst[kF64 ? 1 : 2 * 6 * kItemsMax];
    constexpr int kRounds = (kItemsMax + 255) / 256;
    double2 pre[kF64 ? kRounds : 1][6];
    __shared__ int64_t s_row[6][6];
    __shared__ int32_t s_rec[kChunkRec];
    __shared__ int s_act[kChunk];
    __shared__ KernelConst s_K;
    const int tid = threadIdx.x;
    stage_kconst(a.K, &s_K, tid, blockDim.x);
    const int64_t tile = xcd_remap(blockIdx.x, a.total);
    const int64_t e = a.te_list[tile / a.n_ch];
    const int64_t ch = a.ch_list[tile % a.n_ch];
    for (int i = tid; i < kChunkRec; i += blockDim.x) s_rec[i] = a.chunks[ch * kChunkRec + i];
    if (tid < 36) {
        const int g = tid / 6, i = tid % 6;
        int64_t node = a.tri[6 * e + i];
        if (a.row_map) node = a.row_map[node];
        s_row[g][i] = 2 * (2 * node + (g & 1)) * a.n2;
    }
    if (tid < kChunk) {
        const int64_t f = ch * kChunk + tid;
        bool act = f < a.nt;
        if (act) {
            const int32_t *te = a.tri + 6 * e, *tf = a.tri + 6 * f;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) act = act && (te[i] != tf[j]);
        }
        int kind = act ? 1 : 0;
        if (act && a.mode == 1) {
            const double *ce = a.einfo + 4 * e, *cf = a.einfo + 4 * f;
            const double dx = ce[0] - cf[0], dy = ce[1] - cf[1], dz = ce[2] - cf[2];
            if (sqrt(dx * dx + dy * dy + dz * dz) - ce[3] - cf[3] < a.near_r) {
                kind = 2;
                atomicAdd(a.near_count, 1ull);
            }
        }
        s_act[tid] = kind;
    }
    if constexpr (NODAL) {
        for (int it = tid; it < (kChunk + 1) * kR12; it += blockDim.x) {
            const int side = it / kR12, r = it % kR12;          // side 0: test, 1 + fs: trial
            const int64_t el = side == 0 ? e : ch * kChunk + side - 1;
            const T v = el < a.nt ? a.rtab[el * kR12 + r] : (T)0;
            if (side == 0) s_ra[r] = v;
            else s_rb[(side - 1) * kR12 + r] = v;
        }
    }
    __syncthreads();
    int any = 0;
#pragma unroll
    for (int k = 0; k < kChunk; ++k) any |= s_act[k];
    if (!any) return;
    const int ns = s_rec[0];
    const int rowlen = 2 * ns;
    const int nitems = 6 * rowlen;
    const float inv_rowlen = 1.0f / (float)rowlen;
    {
        const int wave = tid / 64;
#pragma unroll
        for (int k = 0; k < kRounds; ++k) {
            const int base = 256 * k, it = base + tid;
            const bool on = it < nitems;
            const int itc = on ? it : 0;
            const int g = (int)(((float)itc + 0.5f) * inv_rowlen);
            const int rem = itc - g * rowlen;
            const int sl = rem >> 1, be = rem & 1, op = g >> 1;
            const int64_t col = 2 * (2 * (int64_t)s_rec[1 + sl] + be);
            const TS *Z = zblock(a.Z, op) + col;
            const int first = base + wave * 64;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const TS *src = Z + s_row[g][i];
                if constexpr (kF64) {
                    if (on) pre[k][i] = *(const double2 *)src;
                } else {
                    TS *dre = s_dst + (2 * i) * kItemsMax + first, *dim = s_dst + (2 * i + 1) * kItemsMax + first;
                    if (on) {
                        __builtin_amdgcn_global_load_lds((const void *)src,
                                                         (__attribute__((address_space(3))) void *)dre, 4, 0, 0);
                        __builtin_amdgcn_global_load_lds((const void *)(src + 1),
                                                         (__attribute__((address_space(3))) void *)dim, 4, 0, 0);
                    }
                }
            }
        }
    }
    const int64_t nq = a.nt * kQP12;
    const int pl = tid / kQP12, ql = tid % kQP12;      // point pair of lane tid < 144
    for (int fs = 0; fs < kChunk; ++fs) {
        const int kind = s_act[fs];                     // uniform
        if (tid < kPP12) {
            cx<T> k[12];
            const int64_t ix = e * kQP12 + pl, iy = (ch * kChunk + fs) * kQP12 + ql;
            if (kind == 1) {
                const vec3<T> x = qload(a.qp, nq, QX, ix), n = qload(a.qp, nq, QN, ix);
                const vec3<T> ta[2] = {qload(a.qp, nq, QT1, ix), qload(a.qp, nq, QT2, ix)};
                const vec3<T> sa[2] = {qload(a.qp, nq, QS1, ix), qload(a.qp, nq, QS2, ix)};
                const vec3<T> y = qload(a.qp, nq, QX, iy);
                const vec3<T> tb[2] = {qload(a.qp, nq, QT1, iy), qload(a.qp, nq, QT2, iy)};
                const T ww = a.qp[(int64_t)QW * nq + ix] * a.qp[(int64_t)QW * nq + iy];
                kappa12<T>(s_K, x, n, ta, sa, y, tb, ww, k);
            } else if (!std::is_same<T, double>::value && kind == 2) {
                const double *q64 = a.qp64;
                const dvec3 x = qload(q64, nq, QX, ix), n = qload(q64, nq, QN, ix);
                const dvec3 ta[2] = {qload(q64, nq, QT1, ix), qload(q64, nq, QT2, ix)};
                const dvec3 sa[2] = {qload(q64, nq, QS1, ix), qload(q64, nq, QS2, ix)};
                const dvec3 y = qload(q64, nq, QX, iy);
                const dvec3 tb[2] = {qload(q64, nq, QT1, iy), qload(q64, nq, QT2, iy)};
                const double ww = q64[(int64_t)QW * nq + ix] * q64[(int64_t)QW * nq + iy];
                cx<double> kd[12];
                kappa12<double>(s_K, x, n, ta, sa, y, tb, ww, kd);
#pragma unroll
                for (int c = 0; c < 12; ++c) k[c] = cx<T>{(T)kd[c].re, (T)kd[c].im};
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) k[c] = cx<T>{0, 0};
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) s_k[c * kK12Stride + tid] = k[c];
        }
        __syncthreads();
        if constexpr (!NODAL) {
            if (tid < kPP12) {
                const int c = tid / kQP12, p = tid % kQP12;
                cx<T> kv[kQP12], tf[6];
#pragma unroll
                for (int q = 0; q < kQP12; ++q) kv[q] = s_k[c * kK12Stride + p * kQP12 + q];
                contract12(kv, tf);
#pragma unroll
                for (int j = 0; j < 6; ++j) s_tf[((c * kChunk + fs) * kQP12 + p) * 6 + j] = tf[j];
            }
        } else if (tid < 6 * kQP12) {
            // the two delta components of (op, gamma) become the two beta ones
            const int og = tid / kQP12, p = tid % kQP12;     // og = 2 op + gamma
            const cx<T> *k0 = s_k + (2 * og) * kK12Stride + p * kQP12, *k1 = k0 + kK12Stride;
            const T *rb = s_rb + fs * kR12;
            cx<T> *d0 = s_tf + (((2 * og) * kChunk + fs) * kQP12 + p) * 6;
            cx<T> *d1 = s_tf + (((2 * og + 1) * kChunk + fs) * kQP12 + p) * 6;
#pragma unroll 1
            for (int j = 0; j < 6; ++j) {
                cx<T> o0 = {0, 0}, o1 = {0, 0};
#pragma unroll
                for (int q = 0; q < kQP12; ++q) {
                    const T *w = rb + (q * 6 + j) * 4;
                    o0 = o0 + w[0] * k0[q] + w[1] * k1[q];
                    o1 = o1 + w[2] * k0[q] + w[3] * k1[q];
                }
                d0[j] = o0;
                d1[j] = o1;
            }
        }
        __syncthreads();
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        const int it = 256 * k + tid;
        if (it >= nitems) break;
        const int g = (int)(((float)it + 0.5f) * inv_rowlen);
        const int rem = it - g * rowlen;
        const int sl = rem >> 1, be = rem & 1, op = g >> 1;
        const int u1 = s_rec[26 + sl];
        cx<T> out[6];
        if constexpr (!NODAL) {
            const int c = 2 * g + be;
            cx<T> tv[kQP12];
#pragma unroll
            for (int p = 0; p < kQP12; ++p) tv[p] = cx<T>{0, 0};
            for (int u = s_rec[25 + sl]; u < u1; ++u) {
                const int fl = s_rec[50 + u];
                const cx<T> *src = s_tf + ((c * kChunk + (fl >> 3)) * kQP12) * 6 + (fl & 7);
#pragma unroll
                for (int p = 0; p < kQP12; ++p) tv[p] = tv[p] + src[6 * p];
            }
            contract12(tv, out);
        } else {
            // components (op, gamma, beta), gamma = 0, 1: 4 op + beta, 4 op + 2 + beta
            const int al = g & 1, c0 = 4 * op + be, u0 = s_rec[25 + sl];
#pragma unroll
            for (int i = 0; i < 6; ++i) out[i] = cx<T>{0, 0};
#pragma unroll 1
            for (int p = 0; p < kQP12; ++p) {
                cx<T> t0 = {0, 0}, t1 = {0, 0};
                for (int u = u0; u < u1; ++u) {
                    const int fl = s_rec[50 + u];
                    const cx<T> *src0 = s_tf + ((c0 * kChunk + (fl >> 3)) * kQP12 + p) * 6 + (fl & 7);
                    t0 = t0 + src0[0];
                    t1 = t1 + src0[2 * kChunk * kQP12 * 6];
                }
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    const T *w = s_ra + (p * 6 + i) * 4 + 2 * al;
                    out[i] = out[i] + w[0] * t0 + w[1] * t1;
                }
            }
        }
        TS *Z = zblock(a.Z, op) + 2 * (2 * (int64_t)s_rec[1 + sl] + be);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            TS *dst = Z + s_row[g][i];
            TS ore, oim;
            if constexpr (kF64) {
                ore = pre[k][i].x;
                oim = pre[k][i].y;
            } else {
                ore = s_dst[(2 * i) * kItemsMax + it];
                oim = s_dst[(2 * i + 1) * kItemsMax + it];
            }
            dst[0] = ore + (TS)out[i].re;
            dst[1] = oim + (TS)out[i].im;
        }
    }
}

// Singular pairs of the paper's scheme, one launch: per pair the Sauter-
// Schwab points with the singular kernels kappa^s, then the 144 point pairs
// of the 12-point rule with the remainders (constants a.K[0] = the kernels,
// a.K[1] = the shifted truncated series of the remainders); the
// accumulation into the pair's 6 x 6 x 12 block is that of k_ssq.
template <typename TS, bool NODAL = false>
__global__ __launch_bounds__(SsqShape<NODAL>::threads) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_ssq_paper(SsqArgs<TS> a) {
    using Sh = SsqShape<NODAL>;
    __shared__ double s_pt[kSsqThreads * Sh::stride];
    __shared__ double s_tn[NODAL ? 72 : 1];
    const int tid = threadIdx.x;
    const int64_t pid = blockIdx.x;
    const int32_t e = a.pairs[4 * pid], f = a.pairs[4 * pid + 1];
    if constexpr (NODAL) {
        ssq_stage_tangents(a.frames, a.tri, e, f, s_tn, tid);
        __syncthreads();
    }
    const int cls = a.pairs[4 * pid + 2], code = a.pairs[4 * pid + 3];
    const int n = a.order, n4 = n * n * n * n;
    const int nreg = cls == 3 ? 6 : (cls == 2 ? 5 : 2);
    const int nssq = nreg * n4, npts = nssq + kPP12;
    const int comp = tid % 24, stream = tid / 24;
    const bool consumer = tid < 24 * Sh::streams;
    double acc[36];
#pragma unroll
    for (int k = 0; k < 36; ++k) acc[k] = 0.0;
    for (int base = 0; base < npts; base += kSsqThreads) {
        const int idx = base + tid;
        if (tid < kSsqThreads) {
            double *pt = s_pt + tid * Sh::stride;
            if (idx < npts) {
                P2Point X, Y;
                cx<double> k[12];
                if (idx < nssq) {
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
                    p2_point(a.xyz, a.frames, a.tri + 6 * e, xe, ye, X);
                    p2_point(a.xyz, a.frames, a.tri + 6 * f, xf, yf, Y);
                    const dvec3 ta[2] = {X.t1, X.t2}, sa[2] = {X.s1, X.s2}, tb[2] = {Y.t1, Y.t2};
                    kappa12_sing(a.K[0], X.x, X.n, ta, sa, Y.x, tb, wg * X.J * Y.J, k);
                } else {
                    const int rr = idx - nssq, p = rr / kQP12, q = rr % kQP12;
                    double xe, ye, we, xf, yf, wf;
                    rule12(p, xe, ye, we);
                    rule12(q, xf, yf, wf);
                    p2_point(a.xyz, a.frames, a.tri + 6 * e, xe, ye, X);
                    p2_point(a.xyz, a.frames, a.tri + 6 * f, xf, yf, Y);
                    const dvec3 ta[2] = {X.t1, X.t2}, sa[2] = {X.s1, X.s2}, tb[2] = {Y.t1, Y.t2};
                    kappa12_rem(a.K[0], a.K[1], X.x, X.n, ta, sa, Y.x, tb, we * wf * X.J * Y.J, k);
                }
                ssq_row<NODAL>(pt, k, X, Y, s_tn);
            } else {
#pragma unroll
                for (int q = 0; q < (NODAL ? 72 : 36); ++q) pt[q] = 0.0;
            }
        }
        __syncthreads();
        if (consumer) ssq_consume<NODAL>(s_pt, stream, comp, acc);
        __syncthreads();
    }
    ssq_flush<TS, NODAL>(a, e, f, s_pt, acc, tid);
}

// ---------------------------------------------------------- mass ---
// Element mass blocks on the 7-point rule, added to the node CSR values
// through the precomputed slot map; a node pair holds a 2 x 2 block, value
// (a, b) at mval[4 slot + 2 a + b].  Interpolated frame: int N_k N_l delta_ab
// (the frame is orthonormal at every point); node-attached tangents:
// int N_k N_l (P t_a,k) . (P t_b,l).
__global__ void k_mass(int64_t nt, const double *__restrict__ qp, const int32_t *__restrict__ tri,
                       const double *__restrict__ frames, int frame, const int32_t *__restrict__ slot,
                       double *__restrict__ mval) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nt * 36) return;
    const int64_t e = id / 36;
    const int k = (int)(id % 36) / 6, l = (int)(id % 6);
    const int64_t nq = nt * kQP;
    const int64_t vk = tri[6 * e + k], vl = tri[6 * e + l];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < kQP; ++q) {
        double xi, eta, w, N[6], d1[6], d2[6];
        rule7(q, xi, eta, w);
        p2_shape(xi, eta, N, d1, d2);
        const int64_t i = e * kQP + q;
        const double wn = qp[QW * nq + i] * N[k] * N[l];
        if (frame == 0) {
            s[0] += wn;
        } else {
            const dvec3 n = {qp[QN * nq + i], qp[(QN + 1) * nq + i], qp[(QN + 2) * nq + i]};
            const dvec3 tk[2] = {project_tangent(nodal_tangent(frames, vk, 0), n),
                                 project_tangent(nodal_tangent(frames, vk, 1), n)};
            const dvec3 tl[2] = {project_tangent(nodal_tangent(frames, vl, 0), n),
                                 project_tangent(nodal_tangent(frames, vl, 1), n)};
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) s[2 * a + b] += wn * dot(tk[a], tl[b]);
        }
    }
    double *dst = mval + 4 * (int64_t)slot[id];
    if (frame == 0) {
        unsafeAtomicAdd(dst, s[0]);
        unsafeAtomicAdd(dst + 3, s[0]);
    } else {
        for (int c = 0; c < 4; ++c) unsafeAtomicAdd(dst + c, s[c]);
    }
}

// ------------------------------------------------------------ host ---
void derive_constants(const mbem_params *p, double2 *ka, double2 *ki, double2 *eps_i,
                      double2 *mu_i) {
    std::complex<double> er(p->eps_r_re, p->eps_r_im), mr(p->mu_r_re, p->mu_r_im);
    std::complex<double> k = p->k0 * std::sqrt(er * mr);
    if (k.imag() < 0) k = -k;
    *ka = {p->k0, 0.0};
    *ki = {k.real(), k.imag()};
    *eps_i = {er.real(), er.imag()};
    *mu_i = {mr.real(), mr.imag()};
}

static KernelConst make_kconst(const mbem_op *op, bool deriv) {
    using C = std::complex<double>;
    KernelConst K{};
    const C ka(op->ka.x, op->ka.y), ki(op->ki.x, op->ki.y);
    const C ea(1.0, 0.0), ei(op->eps_i.x, op->eps_i.y);
    const C ma(1.0, 0.0), mi(op->mu_i.x, op->mu_i.y);
    K.ka_re = ka.real(); K.ka_im = ka.imag(); K.ki_re = ki.real(); K.ki_im = ki.imag();
    K.eps_a_re = 1.0; K.eps_a_im = 0.0; K.eps_i_re = ei.real(); K.eps_i_im = ei.imag();
    K.mu_a_re = 1.0; K.mu_a_im = 0.0; K.mu_i_re = mi.real(); K.mu_i_im = mi.imag();
    K.kmax = std::max(std::abs(ka), std::abs(ki));
    const C I(0.0, 1.0);
    // c_n(k) = (i k)^n / n!, and d c_n / dk = i c_{n-1}(k)
    C cna(1.0, 0.0), cni(1.0, 0.0), cni_prev(0.0, 0.0);
    const C dk = ki / (2.0 * ei);          // dk_i / deps_i
    if (deriv) { K.ka_re = dk.real(); K.ka_im = dk.imag(); }
    for (int n = 0; n <= kSeriesTerms; ++n) {
        if (n > 0) { cni_prev = cni; cna *= I * ka / (double)n; cni *= I * ki / (double)n; }
        C vD, vF, vG, vE, vM;
        if (!deriv) {
            const C d = cna - cni;
            vD = ka * ka * cna - ki * ki * cni;
            vF = (n >= 2) ? (double)((n - 1) * (n - 3)) * d : C(0.0);
            vG = (n >= 2) ? -(double)(n - 1) * d : C(0.0);
            vE = (double)(n - 1) * (ea * cna - ei * cni);
            vM = (double)(n - 1) * (ma * cna - mi * cni);
        } else {
            const C dci = n > 0 ? I * cni_prev : C(0.0);   // d c_n(k_i) / dk_i
            vD = -(2.0 * ki * cni + ki * ki * dci) * dk;
            vF = (n >= 2) ? -(double)((n - 1) * (n - 3)) * dci * dk : C(0.0);
            vG = (n >= 2) ? (double)(n - 1) * dci * dk : C(0.0);
            vE = (double)(n - 1) * (-cni - ei * dci * dk);
            vM = (double)(n - 1) * (-mi * dci * dk);
        }
        K.cD[2 * n] = vD.real(); K.cD[2 * n + 1] = vD.imag();
        K.cF[2 * n] = vF.real(); K.cF[2 * n + 1] = vF.imag();
        K.cG[2 * n] = vG.real(); K.cG[2 * n + 1] = vG.imag();
        K.cE[2 * n] = vE.real(); K.cE[2 * n + 1] = vE.imag();
        K.cM[2 * n] = vM.real(); K.cM[2 * n + 1] = vM.imag();
    }
    return K;
}

// Constants of the remainders kappa - kappa^s of the paper's scheme: the
// Taylor series without their singular terms, truncated after n = 6, with
// the coefficients shifted to non-negative powers of R (D0: c_{m+1}, df and
// dg: c_{m+3}, G: c_{m+2} multiply R^m).
static KernelConst make_rem_kconst(const mbem_op *op) {
    using C = std::complex<double>;
    constexpr int kPaperTerms = 6;
    KernelConst K = make_kconst(op, false);
    KernelConst R = K;
    for (int i = 0; i < 2 * (kSeriesTerms + 1); ++i) R.cD[i] = R.cF[i] = R.cG[i] = R.cE[i] = R.cM[i] = 0.0;
    const C ka(op->ka.x, op->ka.y), ki(op->ki.x, op->ki.y);
    const C ea(1.0, 0.0), ei(op->eps_i.x, op->eps_i.y);
    const C ma(1.0, 0.0), mi(op->mu_i.x, op->mu_i.y);
    const C I(0.0, 1.0);
    C cna(1.0, 0.0), cni(1.0, 0.0);
    auto put = [](double *c, int m, C v) { c[2 * m] = v.real(); c[2 * m + 1] = v.imag(); };
    for (int n = 0; n <= kPaperTerms; ++n) {
        if (n > 0) { cna *= I * ka / (double)n; cni *= I * ki / (double)n; }
        const C d = cna - cni;
        if (n >= 1) put(R.cD, n - 1, ka * ka * cna - ki * ki * cni);
        if (n >= 3) {
            put(R.cF, n - 3, (double)((n - 1) * (n - 3)) * d);
            put(R.cG, n - 3, -(double)(n - 1) * d);
        }
        if (n >= 2) {
            put(R.cE, n - 2, (double)(n - 1) * (ea * cna - ei * cni));
            put(R.cM, n - 2, (double)(n - 1) * (ma * cna - mi * cni));
        }
    }
    return R;
}

// Node-attached tangents: per triangle and point of the regular rule (NQ
// points), rtab[e][p][k][b][g] = N_k(p) t_b,k . t_g(p), the components of the
// triangle's nodal tangents in the point frame times the shape function; one
// thread per entry, once per fill.
template <typename T, int NQ>
__global__ void k_nodal_table(int64_t nt, const T *__restrict__ qp, const int32_t *__restrict__ tri,
                              const double *__restrict__ frames, T *__restrict__ rtab) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nt * NQ * 24) return;
    const int64_t e = id / (NQ * 24);
    const int r = (int)(id % (NQ * 24));
    const int pq = r / 24, j = (r / 4) % 6, b = (r / 2) % 2, g = r % 2;
    const int64_t nq = nt * NQ;
    const double *t = frames + 9 * (int64_t)tri[6 * e + j] + 3 + 3 * b;
    const vec3<T> tg = qload(qp, nq, g ? QT2 : QT1, e * NQ + pq);
    const double nk = NQ == kQP ? n7(pq, j) : n12(pq, j);
    rtab[id] = (T)nk * ((T)t[0] * tg.x + (T)t[1] * tg.y + (T)t[2] * tg.z);
}

template <typename T, int NQ>
static int nodal_table_run(mbem_op *op, const T *qp, hipStream_t s) {
    const mbem_mesh *m = op->mesh;
    const size_t bytes = sizeof(T) * (size_t)m->nt * NQ * 24;
    if (op->rtab_bytes < bytes) {
        if (op->d_rtab) MBEM_HIP(hipFree(op->d_rtab));
        op->d_rtab = nullptr;
        op->rtab_bytes = 0;
        MBEM_HIP(hipMalloc(&op->d_rtab, bytes));
        op->rtab_bytes = bytes;
    }
    const int64_t n = m->nt * NQ * 24;
    hipLaunchKernelGGL((k_nodal_table<T, NQ>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, m->nt, qp,
                       m->d_tri, m->d_frames, (T *)op->d_rtab);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

// Near radius of the mixed path: params.near_radius, or 1.89 / sqrt|k_a^2 -
// k_i^2| (the gap below which FP32 cancellation of the R^-3 terms reaches
// about 1e-7).
static double near_radius_of(const mbem_op *op) {
    const std::complex<double> ka(op->ka.x, op->ka.y), ki(op->ki.x, op->ki.y);
    const double dk2 = std::abs(ka * ka - ki * ki);
    return op->p.near_radius > 0 ? op->p.near_radius : (dk2 > 0 ? 1.89 / std::sqrt(dk2) : 0.0);
}

template <typename T, typename TS, bool DK = false, bool P12 = false, bool NODAL = false, bool STORE = false>
static int launch_regular(mbem_op *op, int mode, const T *qp, unsigned long long *cnt,
                          hipStream_t s, const FillBand *band = nullptr) {
    const mbem_mesh *m = op->mesh;
    RegArgs<T, TS> a;
    a.nt = m->nt;
    a.n2 = op->n2;
    a.qp = qp;
    a.qp64 = P12 ? m->d_qp12 : m->d_qp;
    a.tri = m->d_tri;
    a.frames = m->d_frames;
    a.rtab = nullptr;
    if constexpr (NODAL) {
        MBEM_TRY((nodal_table_run<T, P12 ? kQP12 : kQP>(op, qp, s)));
        a.rtab = (const T *)op->d_rtab;
    }
    a.chunks = m->d_chunks;
    a.einfo = m->d_elem;
    a.mode = mode;
    a.near_count = cnt;
    a.nmask = op->d_nmask;
    a.n_chunks = (m->nt + kChunk - 1) / kChunk;
    a.near = op->near_view();
    a.tiles = nullptr;
    a.K = op->d_kconst;
    a.near_r = near_radius_of(op);
    a.row_map = band ? band->row_map : nullptr;
    a.row_first = m->d_row_first;
    a.col_first = m->d_col_first;
    a.first_on = std::is_same<TS, double>::value && !DK && !P12 && !NODAL && !STORE && !band && mode == 0;
    for (int o = 0; o < 3; ++o) a.Z[o] = (TS *)(band ? band->Z[o] : op->K[o]);
    const std::vector<int32_t> &toff = band ? band->tcol_off : m->tcol_off;
    const int32_t *tlist = band ? band->tcol : m->d_tcol;
    const int ntc = (int)toff.size() - 1, ncc = (int)m->ccol_off.size() - 1;
    if constexpr (STORE) {
        // only the tiles with near pairs, launch by launch
        for (int64_t L = 0; L + 1 < (int64_t)op->near_tile_off.size(); ++L) {
            a.tiles = op->d_ntiles + op->near_tile_off[L];
            a.total = op->near_tile_off[L + 1] - op->near_tile_off[L];
            if (a.total == 0) continue;
            hipLaunchKernelGGL((k_regular<T, TS, DK, NODAL, true>), dim3((unsigned)a.total), dim3(256), 0, s, a);
            MBEM_HIP(hipGetLastError());
        }
        return MBEM_OK;
    }
    for (int tc = 0; tc < ntc; ++tc)
        for (int cc = 0; cc < ncc; ++cc) {
            a.te_list = tlist + toff[tc];
            a.n_te = toff[tc + 1] - toff[tc];
            a.ch_list = m->d_ccol + m->ccol_off[cc];
            a.n_ch = m->ccol_off[cc + 1] - m->ccol_off[cc];
            a.total = a.n_te * a.n_ch;
            if (a.total == 0) continue;
            if (a.total > 0x7fffffffLL) { set_error("too many element pairs for one launch"); return MBEM_EINVAL; }
            if constexpr (P12)
                hipLaunchKernelGGL((k_regular12<T, TS, NODAL>), dim3((unsigned)a.total), dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_regular<T, TS, DK, NODAL, STORE>), dim3((unsigned)a.total), dim3(256), 0, s, a);
            MBEM_HIP(hipGetLastError());
        }
    return MBEM_OK;
}

// The regular pairs by column range (k_regular_range): one launch per
// test colour.
template <typename T, typename TS>
static int launch_regular_range(mbem_op *op, int mode, const T *qp, unsigned long long *cnt, hipStream_t s) {
    const mbem_mesh *m = op->mesh;
    constexpr int threads = 12 * kRng.rng / 3;
    // wavefronts per SIMD asked of the compiler: the FP32 kernel fits four
    constexpr int waves = std::is_same<T, double>::value ? 2 : 4;
    RngArgs<T, TS> a;
    a.nt = m->nt;
    a.n2 = op->n2;
    a.nn = m->nn;
    a.nrng = m->nrng;
    a.qp = qp;
    a.qp64 = m->d_qp;
    a.tri = m->d_tri;
    a.rng_off = m->d_rng_off;
    a.rng_rec = m->d_rng_rec;
    a.row_first = m->d_row_first;
    a.einfo = m->d_elem;
    a.near_r = near_radius_of(op);
    a.mode = mode;
    a.near_count = cnt;
    a.nmask = op->d_nmask;
    a.n_chunks = (m->nt + kChunk - 1) / kChunk;
    a.K = op->d_kconst;
    for (int o = 0; o < 3; ++o) a.Z[o] = (TS *)op->K[o];
    if (mode == 3 && !a.nmask) { set_error("far-pair fill without a near mask"); return MBEM_EINVAL; }
    if (mode == 1 && (std::is_same<T, double>::value || !cnt)) {
        set_error("range fill: near pairs need a complex64 operator and a counter");
        return MBEM_EINVAL;
    }
    const int ntc = (int)m->tcol_off.size() - 1;
    for (int tc = 0; tc < ntc; ++tc) {
        a.te_list = m->d_tcol + m->tcol_off[tc];
        a.n_te = m->tcol_off[tc + 1] - m->tcol_off[tc];
        a.total = a.n_te * a.nrng;
        if (a.total == 0) continue;
        if (a.total > 0x7fffffffLL) { set_error("too many workgroups for one launch"); return MBEM_EINVAL; }
        if (mode == 1)
            hipLaunchKernelGGL((k_regular_range<T, TS, threads, waves, !std::is_same<T, double>::value>),
                               dim3((unsigned)a.total), dim3(threads), 0, s, a);
        else
            hipLaunchKernelGGL((k_regular_range<T, TS, threads, waves, false>), dim3((unsigned)a.total),
                               dim3(threads), 0, s, a);
        MBEM_HIP(hipGetLastError());
    }
    return MBEM_OK;
}

template <typename TS, bool DK = false, bool PAPER = false, bool NODAL = false>
static int launch_ssq(mbem_op *op, hipStream_t s, const FillBand *band = nullptr) {
    const mbem_mesh *m = op->mesh;
    SsqArgs<TS> a;
    a.n2 = op->n2;
    a.npairs = band ? band->n_spairs : m->n_spairs;
    a.pairs = band ? band->spairs : m->d_spairs;
    a.row_map = band ? band->row_map : nullptr;
    a.tri = m->d_tri;
    a.xyz = m->d_xyz;
    a.frames = m->d_frames;
    a.order = op->p.ssq_order > 0 ? op->p.ssq_order : 4;
    if (a.order > kMaxSSQ) { set_error("ssq_order above 8 is not supported"); return MBEM_EINVAL; }
    double x[kMaxSSQ], w[kMaxSSQ];
    gauss_legendre(a.order, x, w);
    for (int i = 0; i < kMaxSSQ; ++i) {
        a.glx[i] = i < a.order ? 0.5 * (1.0 + x[a.order - 1 - i]) : 0.0;
        a.glw[i] = i < a.order ? 0.5 * w[a.order - 1 - i] : 0.0;
    }
    a.K = PAPER ? op->d_kconst + 1 : op->d_kconst;   // paper: the kernels, then the remainders
    for (int o = 0; o < 3; ++o) a.Z[o] = (TS *)(band ? band->Z[o] : op->K[o]);
    a.near = band ? NearView{} : op->near_view();
    if (a.npairs == 0) return MBEM_OK;
    if constexpr (PAPER)
        hipLaunchKernelGGL((k_ssq_paper<TS, NODAL>), dim3((unsigned)a.npairs), dim3(SsqShape<NODAL>::threads), 0, s,
                           a);
    else
        hipLaunchKernelGGL((k_ssq<TS, DK, NODAL>), dim3((unsigned)a.npairs), dim3(SsqShape<NODAL>::threads), 0, s, a);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

int mass_run(mbem_op *op, hipStream_t s) {
    const mbem_mesh *m = op->mesh;
    MBEM_HIP(hipMemsetAsync(op->d_mval, 0, sizeof(double) * 4 * m->m_col.size(), s));
    const int64_t n = m->nt * 36;
    hipLaunchKernelGGL(k_mass, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       m->nt, m->d_qp, m->d_tri, m->d_frames, op->p.frame, m->d_mslot, op->d_mval);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

// What a fill leaves on the op between its enqueueing and its collection:
// events at its phase boundaries, the pinned staging of the kernel constants
// and of the near-pair count, and the device counter.
struct FillState {
    hipEvent_t ev[7] = {};               // 0..5 phase marks, 6 start
    KernelConst *h_k = nullptr;          // pinned, three
    unsigned long long *h_cnt = nullptr; // pinned
    unsigned long long *d_cnt = nullptr;
    bool pending = false, counted = false;
};

void fill_state_free(FillState *f) {
    if (!f) return;
    for (auto &e : f->ev)
        if (e) (void)hipEventDestroy(e);
    if (f->h_k) (void)hipHostFree(f->h_k);
    if (f->h_cnt) (void)hipHostFree(f->h_cnt);
    if (f->d_cnt) (void)hipFree(f->d_cnt);
    delete f;
}

static int fill_state(mbem_op *op, FillState **out) {
    if (!op->fs) {
        FillState *f = new (std::nothrow) FillState;
        if (!f) { set_error("host allocation"); return MBEM_ENOMEM; }
        op->fs = f;
        for (auto &e : f->ev) MBEM_HIP(hipEventCreate(&e));
        MBEM_HIP(hipHostMalloc((void **)&f->h_k, 3 * sizeof(KernelConst), hipHostMallocDefault));
        MBEM_HIP(hipHostMalloc((void **)&f->h_cnt, sizeof(unsigned long long), hipHostMallocDefault));
        MBEM_HIP(hipMalloc((void **)&f->d_cnt, sizeof(unsigned long long)));
    }
    *out = op->fs;
    return MBEM_OK;
}

int fill_prepare(mbem_op *op, hipStream_t s, bool deriv) {
    const bool paper = op->p.quadrature == MBEM_QUAD_PAPER;
    FillState *f = nullptr;
    MBEM_TRY(fill_state(op, &f));
    // the staging buffer may still feed the previous fill's copy
    if (f->pending) MBEM_HIP(hipEventSynchronize(f->ev[5]));
    // [0]: the kernels of the regular pairs, [1]: the kernels of the singular
    // pairs, [2]: the remainders (paper's scheme)
    if (!op->d_kconst) MBEM_HIP(hipMalloc((void **)&op->d_kconst, 3 * sizeof(KernelConst)));
    f->h_k[0] = make_kconst(op, deriv);
    f->h_k[1] = f->h_k[0];
    f->h_k[2] = KernelConst{};
    if (paper) {
        f->h_k[0].kmax = 1e300;           // regular pairs: the closed forms at every distance
        f->h_k[2] = make_rem_kconst(op);
    }
    MBEM_HIP(hipMemcpyAsync(op->d_kconst, f->h_k, 3 * sizeof(KernelConst), hipMemcpyHostToDevice, s));
    return MBEM_OK;
}

int fill_band_run(mbem_op *op, const FillBand &band, hipStream_t s) {
    if (op->prec != MBEM_FP64 || op->p.quadrature != MBEM_QUAD_DEFAULT) {
        set_error("band fills are built for the FP64 default scheme only");
        return MBEM_EINVAL;
    }
    if (op->p.frame == MBEM_FRAME_NODAL) {
        MBEM_TRY((launch_regular<double, double, false, false, true>(op, 0, op->mesh->d_qp, nullptr, s, &band)));
        MBEM_TRY((launch_ssq<double, false, false, true>(op, s, &band)));
    } else {
        MBEM_TRY((launch_regular<double, double>(op, 0, op->mesh->d_qp, nullptr, s, &band)));
        MBEM_TRY(launch_ssq<double>(op, s, &band));
    }
    return MBEM_OK;
}

int fill_enqueue(mbem_op *op, hipStream_t s, bool deriv, bool geom) {
    const mbem_mesh *m = op->mesh;
    const bool paper = op->p.quadrature == MBEM_QUAD_PAPER;
    if (paper && deriv) { set_error("the eps derivative is built for the default quadrature only"); return MBEM_EINVAL; }
    if (deriv && op->prec != MBEM_FP64) { set_error("derivative operators are filled in FP64"); return MBEM_EINVAL; }
    const bool nodal = op->p.frame == MBEM_FRAME_NODAL;
    MBEM_TRY(fill_prepare(op, s, deriv));
    FillState *f = op->fs;
    hipEvent_t *ev = f->ev;
    MBEM_HIP(hipEventRecord(ev[6], s));
    const size_t esz = op->prec == MBEM_FP64 ? 16 : 8;
    // The complex64 regular pairs go by column ranges, unless the previous
    // fill of this operator found most of them near: a near pair's FP64
    // evaluation is repeated for every range its trial triangle touches
    // (about 1.75 times), which made the column-range fill twice as slow as
    // the chunk kernel on a body whose pairs are 78 % near.
    const int64_t n_reg = m->nt * m->nt - m->n_spairs;
    const bool mixed_chunks = op->prec == MBEM_MIXED && !deriv && !paper && !nodal && !op->p.near_store &&
                              n_reg > 0 && op->n_near > 0.3 * (double)n_reg;
    // the default-scheme fills (FP64 by chunks, complex64 by column ranges)
    // write every entry themselves; the others add to a cleared Z
    const bool range_fill = !deriv && !paper && !nodal && !mixed_chunks;
    if (!range_fill)
        for (int o = 0; o < 3; ++o) MBEM_HIP(hipMemsetAsync(op->K[o], 0, esz * op->n2 * op->n2, s));
    f->counted = op->prec != MBEM_FP64 && !deriv && !(op->p.near_store && !paper && !nodal);
    if (f->counted) MBEM_HIP(hipMemsetAsync(f->d_cnt, 0, sizeof(unsigned long long), s));
    MBEM_HIP(hipEventRecord(ev[0], s));
    if (geom) MBEM_TRY(geom_build(m, s, paper));
    // the near store's pattern for this fill's near radius (one host wait)
    const bool store = op->prec == MBEM_MIXED && !deriv && !paper && !nodal && op->p.near_store;
    if (store) MBEM_TRY(near_build_run(op, near_radius_of(op), s));
    else if (op->near_on) near_free(op);
    MBEM_HIP(hipEventRecord(ev[1], s));
    unsigned long long *cnt = f->counted ? f->d_cnt : nullptr;
    if (paper && op->prec == MBEM_FP64) {
        if (nodal) MBEM_TRY((launch_regular<double, double, false, true, true>(op, 0, m->d_qp12, nullptr, s)));
        else MBEM_TRY((launch_regular<double, double, false, true>(op, 0, m->d_qp12, nullptr, s)));
    } else if (paper) {
        if (nodal) MBEM_TRY((launch_regular<float, float, false, true, true>(op, 1, m->d_qp12_32, cnt, s)));
        else MBEM_TRY((launch_regular<float, float, false, true>(op, 1, m->d_qp12_32, cnt, s)));
    } else if (deriv) {
        if (nodal) MBEM_TRY((launch_regular<double, double, true, false, true>(op, 0, m->d_qp, nullptr, s)));
        else MBEM_TRY((launch_regular<double, double, true>(op, 0, m->d_qp, nullptr, s)));
    } else if (op->prec == MBEM_FP64) {
        if (nodal) MBEM_TRY((launch_regular<double, double, false, false, true>(op, 0, m->d_qp, nullptr, s)));
        else MBEM_TRY((launch_regular<double, double>(op, 0, m->d_qp, nullptr, s)));
    } else if (store) {
        MBEM_TRY((launch_regular_range<float, float>(op, 3, m->d_qp32, nullptr, s)));
    } else if (nodal) {
        MBEM_TRY((launch_regular<float, float, false, false, true>(op, 1, m->d_qp32, cnt, s)));
    } else if (mixed_chunks) {
        MBEM_TRY((launch_regular<float, float>(op, 1, m->d_qp32, cnt, s)));
    } else {
        MBEM_TRY((launch_regular_range<float, float>(op, 1, m->d_qp32, cnt, s)));
    }
    MBEM_HIP(hipEventRecord(ev[2], s));
    // near pairs: inside the regular launches, or with the near store in a
    // launch of their own in FP64
    if (store) MBEM_TRY((launch_regular<double, double, false, false, false, true>(op, 4, m->d_qp, nullptr, s)));
    MBEM_HIP(hipEventRecord(ev[3], s));
    if (paper && op->prec == MBEM_FP64 && nodal) MBEM_TRY((launch_ssq<double, false, true, true>(op, s)));
    else if (paper && op->prec == MBEM_FP64) MBEM_TRY((launch_ssq<double, false, true>(op, s)));
    else if (paper && nodal) MBEM_TRY((launch_ssq<float, false, true, true>(op, s)));
    else if (paper) MBEM_TRY((launch_ssq<float, false, true>(op, s)));
    else if (deriv && nodal) MBEM_TRY((launch_ssq<double, true, false, true>(op, s)));
    else if (deriv) MBEM_TRY((launch_ssq<double, true>(op, s)));
    else if (op->prec == MBEM_FP64 && nodal) MBEM_TRY((launch_ssq<double, false, false, true>(op, s)));
    else if (op->prec == MBEM_FP64) MBEM_TRY(launch_ssq<double>(op, s));
    else if (nodal) MBEM_TRY((launch_ssq<float, false, false, true>(op, s)));
    else MBEM_TRY(launch_ssq<float>(op, s));
    MBEM_HIP(hipEventRecord(ev[4], s));
    MBEM_TRY(mass_run(op, s));
    if (f->counted)
        MBEM_HIP(hipMemcpyAsync(f->h_cnt, f->d_cnt, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    MBEM_HIP(hipEventRecord(ev[5], s));
    f->pending = true;
    return MBEM_OK;
}

int fill_collect(mbem_op *op, double *t_total_ms) {
    FillState *f = op->fs;
    if (!f || !f->pending) { set_error("no fill to collect"); return MBEM_EINVAL; }
    MBEM_HIP(hipEventSynchronize(f->ev[5]));
    f->pending = false;
    auto ms = [&](int a, int b) {
        float t = 0.f;
        return hipEventElapsedTime(&t, f->ev[a], f->ev[b]) == hipSuccess ? (double)t : 0.0;
    };
    if (f->counted) op->n_near = (int64_t)*f->h_cnt;
    else if (!op->near_on) op->n_near = 0;     // with the near store: counted by its build
    op->t_phase[0] = ms(0, 1);
    op->t_phase[1] = ms(1, 2);
    op->t_phase[2] = ms(2, 3);
    op->t_phase[3] = ms(3, 4);
    op->t_phase[4] = ms(4, 5);
    if (t_total_ms) *t_total_ms = ms(6, 5);
    return MBEM_OK;
}

int fill_run(mbem_op *op, hipStream_t s, bool deriv, bool geom) {
    MBEM_TRY(fill_enqueue(op, s, deriv, geom));
    return fill_collect(op, nullptr);
}

}  // namespace mbem
