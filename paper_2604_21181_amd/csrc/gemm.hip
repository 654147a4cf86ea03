// Complex GEMMs on the matrix cores for the multi-right-hand-side solve.
//
// Every product here has the shape
//     C[b][m] = sum_k op(A[m][k]) * B[b][k]        (complex, op = id or conj)
// with both operands contiguous along k: A is a stored operator block
// (row-major) or a Krylov basis block, B holds one vector per row (the
// right-hand sides of a block).  The complex product is carried out as a
// real GEMM of twice the size in k and in the output columns:
//     A_r = [a_re a_im a_re a_im ...]  (the complex row read as floats)
//     B'  row 2b   = [ b_re  -b_im ...]   -> Re C      (conj: [b_re  b_im])
//     B'  row 2b+1 = [ b_im   b_re ...]   -> Im C      (conj: [b_im -b_re])
// B' is formed while staging B through LDS; A is used as stored.
//
// FP32 (complex64 operator, FP32 accumulation): v_mfma_f32_32x32x2f32 on
// three real products per complex one (3M, below) instead of the doubled
// real GEMM; one template per tile shape; the shape is chosen at run time by
// measuring every candidate on the problem at hand (autotune below).
// FP64 (basis projections, Gram matrices, refinement residuals):
// v_mfma_f64_16x16x4f64 on 64 x 64 tiles with an optional split of k.
#include <algorithm>
#include <cstdio>
#include <type_traits>

#include "gemm.h"

namespace mbem {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Each of the 8 XCDs receives workgroups round-robin; give each one a
// contiguous range of tiles so that tiles sharing rows of A meet in one L2.
__device__ inline int64_t xcd_tile(int64_t bid, int64_t total) {
    const int64_t q = total / 8, r = total % 8;
    const int64_t xcd = bid % 8, local = bid / 8;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

struct TileRef {
    int q;            // problem
    int64_t bidx;     // batch entry
    int64_t tm, tn;   // tile coordinates
};

__device__ inline TileRef locate(const CgemmList &L, int64_t tile) {
    TileRef t;
    t.q = 0;
    if (L.np > 1 && tile >= L.p[1].tile0) t.q = 1;
    if (L.np > 2 && tile >= L.p[2].tile0) t.q = 2;
    return t;
}

// Uniform selection of one of the (at most three) problems without
// dynamic indexing of the kernel argument.
#define MBEM_PICK(L, q, field) ((q) == 0 ? (L).p[0].field : (q) == 1 ? (L).p[1].field : (L).p[2].field)

// ------------------------------------------------------------- FP32 ----
// Three real products per complex product (the 3M method):
//   T1 = (A_re + A_im) B_re^T,  T2 = A_re (B_im - B_re)^T,  T3 = A_im (B_re + B_im)^T,
//   Re C = T1 - T3,  Im C = T1 + T2,
// so 3 instead of 4 real multiply-adds per complex one.  Per stage of 8
// complex k the three A planes and the three B planes are formed while
// staging through LDS, each row stored k-interleaved (position 4 h + s for
// k = 2 s + h) so that a lane reads its four MFMA inputs with one 16-byte
// load.  BN counts real output columns (two per complex column), as the
// tile shapes of the autotuner are named.
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN)) void k_cgemm_f32(CgemmList L) {
    static_assert(WN >= 64 && WM >= 32, "a wavefront covers at least 32 x 32 complex outputs");
    constexpr int NWN = BN / WN;
    constexpr int NT = 64 * (BM / WM) * NWN;
    constexpr int BC = BN / 2, WC = WN / 2;       // complex output columns per tile / wave
    constexpr int TM = WM / 32, TC = WC / 32;
    constexpr int LD = 12;                        // 8 k + pad, in floats
    constexpr int NA = (BM * 4 + NT - 1) / NT;    // float4 (two complex k) loads of A per stage
    constexpr int NB = (BC * 4 + NT - 1) / NT;
    __shared__ __align__(16) float sA[2][3][BM * LD];
    __shared__ __align__(16) float sB[2][3][BC * LD];

    const int64_t tile = xcd_tile(blockIdx.x, L.total);
    const int q = locate(L, tile).q;
    const int64_t t = tile - MBEM_PICK(L, q, tile0);
    const int64_t per = MBEM_PICK(L, q, tiles);
    const int64_t tn_count = MBEM_PICK(L, q, tn);
    const int64_t bidx = t / per, r = t % per;
    const int64_t m0 = (r / tn_count) * BM, b0 = (r % tn_count) * BC;
    const int64_t M = MBEM_PICK(L, q, M), Nb = MBEM_PICK(L, q, Nb), K = MBEM_PICK(L, q, K);
    const int64_t lda = MBEM_PICK(L, q, lda), ldb = MBEM_PICK(L, q, ldb), ldc = MBEM_PICK(L, q, ldc);
    const float2 *A = (const float2 *)MBEM_PICK(L, q, A) + bidx * MBEM_PICK(L, q, sa);
    const float2 *B = (const float2 *)MBEM_PICK(L, q, B) + bidx * MBEM_PICK(L, q, sb);
    float2 *C = (float2 *)MBEM_PICK(L, q, C) + bidx * MBEM_PICK(L, q, sc);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / NWN, wn = wave % NWN;
    const int h = lane >> 5, l32 = lane & 31;

    f32x4 ra[NA], rb[NB];
    auto ld2 = [](const float2 *src, int64_t kc, int64_t Kend) {
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (kc + 1 < Kend) v = *(const f32x4 *)src;
        else if (kc < Kend) { const float2 w = src[0]; v = {w.x, w.y, 0.f, 0.f}; }
        return v;
    };
    auto gload = [&](int64_t kc0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int idx = tid + i * NT;
            const int64_t m = m0 + (idx >> 2), kc = kc0 + 2 * (idx & 3);
            ra[i] = (idx < BM * 4 && m < M) ? ld2(A + m * lda + kc, kc, K) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int idx = tid + i * NT;
            const int64_t b = b0 + (idx >> 2), kc = kc0 + 2 * (idx & 3);
            rb[i] = (idx < BC * 4 && b < Nb) ? ld2(B + b * ldb + kc, kc, K) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
    };
    // complex k = 2 kk + j of the pair (kk = idx & 3) -> position 4 (k & 1) + (k >> 1)
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int idx = tid + i * NT;
            if (idx < BM * 4) {
                const f32x4 v = ra[i];
                const int row = idx >> 2, kk = idx & 3;
                float *s0 = &sA[buf][0][row * LD], *s1 = &sA[buf][1][row * LD], *s2 = &sA[buf][2][row * LD];
                s0[kk] = v.x + v.y;  s1[kk] = v.x;  s2[kk] = v.y;          // k = 2 kk (even: h = 0)
                s0[4 + kk] = v.z + v.w;  s1[4 + kk] = v.z;  s2[4 + kk] = v.w;   // k = 2 kk + 1
            }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int idx = tid + i * NT;
            if (idx < BC * 4) {
                const f32x4 v = rb[i];
                const int row = idx >> 2, kk = idx & 3;
                float *s0 = &sB[buf][0][row * LD], *s1 = &sB[buf][1][row * LD], *s2 = &sB[buf][2][row * LD];
                s0[kk] = v.x;  s1[kk] = v.y - v.x;  s2[kk] = v.x + v.y;
                s0[4 + kk] = v.z;  s1[4 + kk] = v.w - v.z;  s2[4 + kk] = v.z + v.w;
            }
        }
    };

    f32x16 acc[3][TM][TC];
#pragma unroll
    for (int p3 = 0; p3 < 3; ++p3)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TC; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[p3][i][j][e] = 0.f;

    const int64_t nst = (K + 7) / 8;   // stages of 8 complex k
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
        const int cur = (int)(st & 1);
        if (st + 1 < nst) gload((st + 1) * 8);
        // lane (l32, h) feeds MFMA step s with complex k = 2 s + h
        f32x4 a[3][TM], b[3][TC];
#pragma unroll
        for (int p3 = 0; p3 < 3; ++p3) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
                a[p3][i] = *(const f32x4 *)&sA[cur][p3][(wm * WM + i * 32 + l32) * LD + 4 * h];
#pragma unroll
            for (int j = 0; j < TC; ++j)
                b[p3][j] = *(const f32x4 *)&sB[cur][p3][(wn * WC + j * 32 + l32) * LD + 4 * h];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int p3 = 0; p3 < 3; ++p3)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TC; ++j)
                        acc[p3][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p3][i][s], b[p3][j][s],
                                                                             acc[p3][i][j], 0, 0, 0);
        if (st + 1 < nst) sstore(cur ^ 1);
        __syncthreads();
    }
    // accumulator (lane, e): complex column l32, row 8 (e / 4) + 4 h + e % 4
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t m = m0 + wm * WM + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                const int64_t b = b0 + wn * WC + j * 32 + l32;
                const float t1 = acc[0][i][j][e], t2 = acc[1][i][j][e], t3 = acc[2][i][j][e];
                if (m < M && b < Nb) C[b * ldc + m] = float2{t1 - t3, t1 + t2};
            }
}

// ------------------------------------------------------------- FP64 ----
// 64 rows x 32 complex columns per workgroup, 4 waves of 32 x 16, the 3M
// method as in the FP32 kernel (op(A) = conj(A) negates the A_im plane);
// k split over gridDim.y: split y covers complex k in [y kchunk,
// (y + 1) kchunk) and writes its partial product at C + y * split_stride.
// The product is scaled by alpha; with rmw it is added to what C holds
// (one split only).
template <typename TA, typename TB, bool CONJ>
__global__ __launch_bounds__(256) void k_cgemm_f64(CgemmList L, int64_t kchunk, int64_t split_stride, double alpha,
                                                   int rmw) {
    constexpr int BM = 64, BC = 32, WM = 32, WC = 16;
    constexpr int LD = 10;   // 8 complex k + pad, in doubles
    __shared__ __align__(16) double sA[2][3][BM * LD];
    __shared__ __align__(16) double sB[2][3][BC * LD];

    const int64_t tile = xcd_tile(blockIdx.x, L.total);
    const int q = locate(L, tile).q;
    const int64_t t = tile - MBEM_PICK(L, q, tile0);
    const int64_t per = MBEM_PICK(L, q, tiles);
    const int64_t tn_count = MBEM_PICK(L, q, tn);
    const int64_t bidx = t / per, r = t % per;
    const int64_t m0 = (r / tn_count) * BM, b0 = (r % tn_count) * BC;
    const int64_t M = MBEM_PICK(L, q, M), Nb = MBEM_PICK(L, q, Nb), Kall = MBEM_PICK(L, q, K);
    const int64_t lda = MBEM_PICK(L, q, lda), ldb = MBEM_PICK(L, q, ldb), ldc = MBEM_PICK(L, q, ldc);
    const TA *A = (const TA *)MBEM_PICK(L, q, A) + bidx * MBEM_PICK(L, q, sa);
    const TB *B = (const TB *)MBEM_PICK(L, q, B) + bidx * MBEM_PICK(L, q, sb);
    double2 *C = (double2 *)MBEM_PICK(L, q, C) + bidx * MBEM_PICK(L, q, sc) + blockIdx.y * split_stride;
    const int64_t kbeg = blockIdx.y * kchunk;
    const int64_t K = std::min(Kall, kbeg + kchunk);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int g = lane >> 4, l16 = lane & 15;

    // per stage: A 64 rows x 8 complex (two adjacent k per thread), B 32
    // rows x 8 complex (one per thread)
    double ra[4], rb[2];
    auto ld1 = [](const auto *p, int64_t kc, int64_t Kend, double *o) {
        if (kc < Kend) { o[0] = (double)p[kc].x; o[1] = (double)p[kc].y; }
        else { o[0] = 0.0; o[1] = 0.0; }
    };
    auto gload = [&](int64_t kc0) {
        {
            const int row = tid >> 2, kq = 2 * (tid & 3);
            const int64_t m = m0 + row;
            if (m < M) {
                const TA *p = A + m * lda;
                ld1(p, kc0 + kq, K, ra);
                ld1(p, kc0 + kq + 1, K, ra + 2);
            } else { ra[0] = ra[1] = ra[2] = ra[3] = 0.0; }
        }
        {
            const int row = tid >> 3, kq = tid & 7;
            const int64_t b = b0 + row;
            if (b < Nb) ld1(B + b * ldb, kc0 + kq, K, rb);
            else { rb[0] = rb[1] = 0.0; }
        }
    };
    // complex k of the stage -> position 2 (k & 3) + (k >> 2): lane g reads
    // the two k = g, 4 + g of its MFMA steps with one 16-byte load
    auto pos = [](int k) { return 2 * (k & 3) + (k >> 2); };
    auto sstore = [&](int buf) {
        {
            const int row = tid >> 2, kq = 2 * (tid & 3);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double ar = ra[2 * u], ai = CONJ ? -ra[2 * u + 1] : ra[2 * u + 1];
                const int o = row * LD + pos(kq + u);
                sA[buf][0][o] = ar + ai;
                sA[buf][1][o] = ar;
                sA[buf][2][o] = ai;
            }
        }
        {
            const int row = tid >> 3, kq = tid & 7;
            const int o = row * LD + pos(kq);
            const double br = rb[0], bi = rb[1];
            sB[buf][0][o] = br;
            sB[buf][1][o] = bi - br;
            sB[buf][2][o] = br + bi;
        }
    };

    f64x4 acc[3][2];
#pragma unroll
    for (int p3 = 0; p3 < 3; ++p3)
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[p3][i] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int64_t nst = K > kbeg ? (K - kbeg + 7) / 8 : 0;
    if (nst > 0) {
        gload(kbeg);
        sstore(0);
    }
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
        const int cur = (int)(st & 1);
        if (st + 1 < nst) gload(kbeg + (st + 1) * 8);
        // lane (l16, g) feeds MFMA step s with complex k = 4 s + g of the stage
        f64x2 a[3][2], bb[3];
#pragma unroll
        for (int p3 = 0; p3 < 3; ++p3) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[p3][i] = *(const f64x2 *)&sA[cur][p3][(wm * WM + i * 16 + l16) * LD + 2 * g];
            bb[p3] = *(const f64x2 *)&sB[cur][p3][(wn * WC + l16) * LD + 2 * g];
        }
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int p3 = 0; p3 < 3; ++p3)
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[p3][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p3][i][s2], bb[p3][s2], acc[p3][i], 0, 0, 0);
        if (st + 1 < nst) sstore(cur ^ 1);
        __syncthreads();
    }
    // accumulator (lane, e): complex column l16, row g + 4 e
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t m = m0 + wm * WM + i * 16 + g + 4 * e;
            const int64_t b = b0 + wn * WC + l16;
            if (m < M && b < Nb) {
                const double t1 = acc[0][i][e], t2 = acc[1][i][e], t3 = acc[2][i][e];
                const double v = t1 - t3, w = t1 + t2;
                double2 *c = C + b * ldc + m;
                if (rmw) {
                    const double2 o = *c;
                    *c = double2{o.x + alpha * v, o.y + alpha * w};
                } else {
                    *c = double2{alpha * v, alpha * w};
                }
            }
        }
}

// Sum of the k-split partial products (compact [split][batch][Nb][M]) into
// the output layout; ACC adds to what the output holds.
template <bool ACC>
__global__ void k_split_reduce(const double2 *part, int splits, int64_t M, int64_t Nb, int64_t batch,
                               double2 *out, int64_t ldc, int64_t sc, double alpha) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t per = M * Nb, stride = per * batch;
    if (id >= stride) return;
    const int64_t bi = id / per, r = id % per, b = r / M, m = r % M;
    double2 s = {0.0, 0.0};
    for (int y = 0; y < splits; ++y) { const double2 v = part[y * stride + id]; s.x += v.x; s.y += v.y; }
    double2 *o = out + bi * sc + b * ldc + m;
    if (ACC) { o->x += alpha * s.x; o->y += alpha * s.y; }
    else *o = {alpha * s.x, alpha * s.y};
}

// ------------------------------------------------------------- host ----
namespace {
struct F32Cfg { int BM, BN, WM, WN; };
constexpr F32Cfg kF32Cfg[kGemmConfigs] = {
    {128, 128, 64, 64}, {128, 64, 64, 64}, {64, 128, 32, 64}, {64, 64, 32, 64},
    {256, 128, 64, 64}, {128, 256, 64, 64},
};

int64_t plan(CgemmList &L, int BM, int BN) {
    int64_t tile0 = 0;
    for (int q = 0; q < L.np; ++q) {
        CgemmProb &P = L.p[q];
        const int64_t tm = (P.M + BM - 1) / BM, tn = (2 * P.Nb + BN - 1) / BN;
        P.tn = tn;
        P.tiles = tm * tn;
        P.tile0 = tile0;
        tile0 += P.tiles * P.batch;
    }
    L.total = tile0;
    return tile0;
}

template <int BM, int BN, int WM, int WN>
int launch_f32(CgemmList L, hipStream_t s) {
    const int64_t total = plan(L, BM, BN);
    if (total == 0) return MBEM_OK;
    constexpr int NT = 64 * (BM / WM) * (BN / WN);
    hipLaunchKernelGGL((k_cgemm_f32<BM, BN, WM, WN>), dim3((unsigned)total), dim3(NT), 0, s, L);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}
}  // namespace

bool cgemm_list_valid(const CgemmList &L, size_t esz_a, size_t esz_b) {
    if (L.np < 1 || L.np > 3) return false;
    for (int q = 0; q < L.np; ++q) {
        const CgemmProb &P = L.p[q];
        if (P.M < 0 || P.Nb < 0 || P.K < 0 || P.batch < 1) return false;
        if (P.lda < P.K || P.ldb < P.K || P.ldc < P.M) return false;
        // 16-byte vector loads of two complex64 need even strides and offsets
        if (esz_a == 8 && ((P.lda | P.sa) & 1 || ((uintptr_t)P.A & 15))) return false;
        if (esz_b == 8 && ((P.ldb | P.sb) & 1 || ((uintptr_t)P.B & 15))) return false;
        if (!P.A || !P.B || !P.C) return false;
    }
    return true;
}

int cgemm_f32_run(CgemmList L, int cfg, hipStream_t s) {
    switch (cfg) {
        case 0: return launch_f32<128, 128, 64, 64>(L, s);
        case 1: return launch_f32<128, 64, 64, 64>(L, s);
        case 2: return launch_f32<64, 128, 32, 64>(L, s);
        case 3: return launch_f32<64, 64, 32, 64>(L, s);
        case 4: return launch_f32<256, 128, 64, 64>(L, s);
        case 5: return launch_f32<128, 256, 64, 64>(L, s);
        default: set_error("unknown GEMM configuration"); return MBEM_EINVAL;
    }
}

void cgemm_f32_config(int cfg, int *bm, int *bn, int *wm, int *wn) {
    const F32Cfg c = kF32Cfg[std::clamp(cfg, 0, kGemmConfigs - 1)];
    *bm = c.BM; *bn = c.BN; *wm = c.WM; *wn = c.WN;
}

int cgemm_f64_run(CgemmList L, bool a_c64, bool conj_a, int splits, double2 *work, hipStream_t s,
                  bool accumulate, double alpha) {
    const int64_t total = plan(L, 64, 64);
    if (total == 0) return MBEM_OK;
    if (splits < 1) splits = 1;
    int64_t kmax = 0;
    for (int q = 0; q < L.np; ++q) kmax = std::max(kmax, L.p[q].K);
    const int64_t kchunk = std::max<int64_t>(8, ((kmax + splits - 1) / splits + 7) / 8 * 8);
    splits = (int)std::max<int64_t>(1, (kmax + kchunk - 1) / kchunk);
    const bool staged = splits > 1;
    if (staged && (L.np != 1 || !work)) { set_error("split GEMM needs one problem and a workspace"); return MBEM_EINVAL; }
    CgemmList Lw = L;
    int64_t stride = 0;
    if (staged) {
        // partial products in a compact [split][batch][Nb][M] layout
        CgemmProb &P = Lw.p[0];
        P.C = work;
        P.ldc = P.M;
        P.sc = P.M * P.Nb;
        stride = P.sc * P.batch;
    }
    const dim3 grid((unsigned)total, (unsigned)splits);
    // one split: the kernel scales (and accumulates) itself; several: the
    // reduction does
    const double kalpha = staged ? 1.0 : alpha;
    const int krmw = !staged && accumulate ? 1 : 0;
    if (a_c64 && conj_a)
        hipLaunchKernelGGL((k_cgemm_f64<float2, double2, true>), grid, dim3(256), 0, s, Lw, kchunk, stride, kalpha, krmw);
    else if (a_c64)
        hipLaunchKernelGGL((k_cgemm_f64<float2, double2, false>), grid, dim3(256), 0, s, Lw, kchunk, stride, kalpha, krmw);
    else if (conj_a)
        hipLaunchKernelGGL((k_cgemm_f64<double2, double2, true>), grid, dim3(256), 0, s, Lw, kchunk, stride, kalpha, krmw);
    else
        hipLaunchKernelGGL((k_cgemm_f64<double2, double2, false>), grid, dim3(256), 0, s, Lw, kchunk, stride, kalpha, krmw);
    MBEM_HIP(hipGetLastError());
    if (staged) {
        const CgemmProb &P = L.p[0];
        const int64_t n = P.M * P.Nb * P.batch;
        const unsigned g = (unsigned)((n + 255) / 256);
        if (accumulate)
            hipLaunchKernelGGL(k_split_reduce<true>, dim3(g), dim3(256), 0, s, work, splits, P.M, P.Nb,
                               (int64_t)P.batch, (double2 *)P.C, P.ldc, P.sc, alpha);
        else
            hipLaunchKernelGGL(k_split_reduce<false>, dim3(g), dim3(256), 0, s, work, splits, P.M, P.Nb,
                               (int64_t)P.batch, (double2 *)P.C, P.ldc, P.sc, alpha);
        MBEM_HIP(hipGetLastError());
    }
    return MBEM_OK;
}

int64_t cgemm_f64_work(const CgemmList &L, int splits) {
    if (L.np != 1) return 0;
    const CgemmProb &P = L.p[0];
    return (int64_t)std::max(splits, 1) * P.M * P.Nb * P.batch;
}

// Measure every FP32 tile shape on this exact problem list (one warm-up,
// then the best of `reps` timed launches) and return the fastest.
int cgemm_f32_autotune(const CgemmList &L, hipStream_t s, int reps, float *ms_out, int *best) {
    hipEvent_t e0, e1;
    MBEM_HIP(hipEventCreate(&e0));
    MBEM_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    int arg = 0;
    int st = MBEM_OK;
    for (int c = 0; c < kGemmConfigs && st == MBEM_OK; ++c) {
        st = cgemm_f32_run(L, c, s);
        float tmin = 1e30f;
        for (int r = 0; r < reps && st == MBEM_OK; ++r) {
            (void)hipEventRecord(e0, s);
            st = cgemm_f32_run(L, c, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tmin = std::min(tmin, ms);
        }
        if (ms_out) ms_out[c] = tmin;
        if (tmin < best_ms) { best_ms = tmin; arg = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best) *best = arg;
    return st;
}

}  // namespace mbem
