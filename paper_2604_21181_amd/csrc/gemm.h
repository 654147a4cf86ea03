// Complex GEMMs with both operands contiguous along k (gemm.hip).
#pragma once

#include "mbem_internal.h"

namespace mbem {

constexpr int kGemmConfigs = 6;   // FP32 tile shapes known to the autotuner

// C[b][m] = sum_k op(A[m][k]) B[b][k] for m < M, b < Nb, k < K, over
// `batch` independent entries spaced sa, sb, sc elements apart.
// Leading dimensions and strides count complex elements.
struct CgemmProb {
    const void *A = nullptr;
    const void *B = nullptr;
    void *C = nullptr;
    int64_t lda = 0, ldb = 0, ldc = 0;
    int64_t sa = 0, sb = 0, sc = 0;
    int64_t M = 0, Nb = 0, K = 0;
    int32_t batch = 1;
    // filled by the launcher
    int64_t tn = 0, tiles = 0, tile0 = 0;
};

// Up to three problems served by one launch (their tiles are concatenated).
struct CgemmList {
    CgemmProb p[3];
    int np = 0;
    int64_t total = 0;
};

bool cgemm_list_valid(const CgemmList &L, size_t esz_a, size_t esz_b);
// complex64 A, B, C; FP32 accumulation on MFMA; cfg in [0, kGemmConfigs)
int cgemm_f32_run(CgemmList L, int cfg, hipStream_t s);
void cgemm_f32_config(int cfg, int *bm, int *bn, int *wm, int *wn);
int cgemm_f32_autotune(const CgemmList &L, hipStream_t s, int reps, float *ms_out, int *best);
// A complex64 (a_c64) or complex128, B and C complex128; FP64 accumulation.
// C = alpha op(A) B, or C += alpha op(A) B with `accumulate`.  splits > 1
// divides k among workgroups (one problem only) and sums the partial
// products from `work` (cgemm_f64_work elements).
int cgemm_f64_run(CgemmList L, bool a_c64, bool conj_a, int splits, double2 *work, hipStream_t s,
                  bool accumulate = false, double alpha = 1.0);
int64_t cgemm_f64_work(const CgemmList &L, int splits);

}  // namespace mbem
