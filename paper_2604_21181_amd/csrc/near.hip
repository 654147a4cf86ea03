// The FP64 near store of a MIXED operator.
//
// The hypersingular part of the kernel differences cancels only as R -> 0
// (Sec. 2.3, eq. Hdiff_infinite), which is why the near element pairs and
// the singular pairs are evaluated in FP64 on the mixed path.  With the
// store their contributions are also summed and kept in FP64: a sparse
// node-pair store beside the complex64 blocks, holding for every node pair
// (i, j) touched by a near or singular element pair the 2 x 2 (alpha, beta)
// blocks of K1, K2^eps and K2^mu.  The far element pairs go to the complex64
// blocks; Z is their sum.
//
// The pattern is built on the device at every fill (the near radius moves
// with the wavenumbers): a bit row per node, set by the element pairs that
// touch it, then per row the count of set bits before each 32-bit word (so
// that a pair's slot is found in constant time) and a CSR of the columns.
// The same pass records, per (test triangle, trial chunk of the regular-pair
// fill), which of the chunk's triangles are near partners: the FP32 far
// launch skips them and the FP64 near launch computes only them, so both
// take the one classification.
#include "mbem_internal.h"
#include "near_store.h"

namespace mbem {

namespace {

// One thread per (test triangle e, trial chunk): classify the chunk's
// triangles (singular: a shared vertex node; near: regular with centroid
// distance minus both radii below near_r) and set the pattern bits of the
// 6 x 6 node pairs of every near or singular pair.  The classification is
// symmetric in the two triangles, so the pattern is symmetric (the
// transposed product walks it by rows).
__global__ void k_near_mark(int64_t nt, int64_t nch, int64_t nw, const int32_t *__restrict__ tri,
                            const double *__restrict__ einfo, double near_r, const int32_t *__restrict__ tcolour,
                            const int32_t *__restrict__ ccolour, int ncc, uint32_t *bits, uint8_t *mask,
                            unsigned long long *count) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nt * nch) return;
    const int64_t e = id / nch, ch = id % nch;
    const int32_t *te = tri + 6 * e;
    const double *ce = einfo + 4 * e;
    unsigned m = 0;
    for (int fs = 0; fs < kChunk; ++fs) {
        const int64_t f = ch * kChunk + fs;
        if (f >= nt) break;
        const int32_t *tf = tri + 6 * f;
        bool sing = false;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) sing = sing || te[a] == tf[b];
        bool near = false;
        if (!sing) {
            const double *cf = einfo + 4 * f;
            const double dx = ce[0] - cf[0], dy = ce[1] - cf[1], dz = ce[2] - cf[2];
            // symmetric in (e, f) to the last bit, so that the pattern is
            near = sqrt(dx * dx + dy * dy + dz * dz) - (ce[3] + cf[3]) < near_r;
        }
        if (!sing && !near) continue;
        if (near) m |= 1u << fs;
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
                const int64_t j = tf[b];
                atomicOr(bits + (int64_t)te[a] * nw + (j >> 5), 1u << (j & 31));
            }
    }
    mask[id] = (uint8_t)m;
    if (m) {
        atomicAdd(count, (unsigned long long)__popc(m));
        atomicAdd(count + 2 + (int64_t)tcolour[e] * ncc + ccolour[ch], 1ull);
    }
}

// Every tile with near pairs at the next free place of its launch's run.
// (The order inside a launch does not matter: its tiles write disjoint
// slots.)
__global__ void k_near_tiles(int64_t nt, int64_t nch, const uint8_t *__restrict__ mask,
                             const int32_t *__restrict__ tcolour, const int32_t *__restrict__ ccolour, int ncc,
                             unsigned long long *cursor, int2 *tiles) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nt * nch || !mask[id]) return;
    const int64_t e = id / nch, ch = id % nch;
    const unsigned long long pos = atomicAdd(cursor + (int64_t)tcolour[e] * ncc + ccolour[ch], 1ull);
    tiles[pos] = make_int2((int)e, (int)ch);
}

// One wavefront per node row: the count of set bits before every word of
// the row (a wavefront prefix sum over 64 words at a time), and the row's
// total.
__global__ __launch_bounds__(256) void k_near_count(int64_t nn, int64_t nw, const uint32_t *__restrict__ bits,
                                                    int32_t *wpre, int32_t *rcount) {
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x % 64;
    if (i >= nn) return;
    int32_t base = 0;
    for (int64_t w0 = 0; w0 < nw; w0 += 64) {
        const int64_t w = w0 + lane;
        const int32_t c = w < nw ? __popc(bits[i * nw + w]) : 0;
        int32_t inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t v = __shfl_up(inc, o, 64);
            if (lane >= o) inc += v;
        }
        if (w < nw) wpre[i * nw + w] = base + inc - c;
        base += __shfl(inc, 63, 64);
    }
    if (lane == 0) rcount[i] = base;
}

// Exclusive prefix sum of the row counts (rptr[0..nn], in place over
// rptr[1..nn] = counts) by one workgroup: per-thread runs, then the runs'
// offsets.  rptr[nn] and, through it, the pattern size come last.
__global__ __launch_bounds__(1024) void k_near_scan(int64_t nn, int32_t *rptr, unsigned long long *nnz) {
    __shared__ int64_t s_sum[1024];
    const int t = threadIdx.x;
    const int64_t per = (nn + 1023) / 1024;
    const int64_t a = t * per, b = a + per < nn ? a + per : nn;
    int64_t run = 0;
    for (int64_t k = a; k < b; ++k) run += rptr[k + 1];
    s_sum[t] = run;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < 1024; ++k) { const int64_t v = s_sum[k]; s_sum[k] = acc; acc += v; }
        rptr[0] = 0;
        *nnz = (unsigned long long)acc;
    }
    __syncthreads();
    int64_t acc = s_sum[t];
    for (int64_t k = a; k < b; ++k) { acc += rptr[k + 1]; rptr[k + 1] = (int32_t)acc; }
}

// One wavefront per node row: every lane writes the columns of its words'
// set bits at their slots (increasing order along the row).
__global__ __launch_bounds__(256) void k_near_cols(int64_t nn, int64_t nw, const uint32_t *__restrict__ bits,
                                                   const int32_t *__restrict__ wpre, const int32_t *__restrict__ rptr,
                                                   int32_t *col) {
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x % 64;
    if (i >= nn) return;
    for (int64_t w = lane; w < nw; w += 64) {
        uint32_t word = bits[i * nw + w];
        int64_t k = (int64_t)rptr[i] + wpre[i * nw + w];
        while (word) {
            const int b = __ffs(word) - 1;
            col[k++] = (int32_t)(32 * w + b);
            word &= word - 1u;
        }
    }
}

// Z32[op][2 i + al][2 j + be] += store value, one thread per stored value.
__global__ void k_near_fold(int64_t nn, int64_t n2, NearView v, int64_t nnz, float2 *K0, float2 *K1,
                            float2 *K2) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= 12 * nnz) return;
    const int64_t s = id / 12;
    const int c = (int)(id % 12), op = c >> 2, al = (c >> 1) & 1, be = c & 1;
    // row of slot s: the last row whose offset is <= s
    int64_t lo = 0, hi = nn;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (v.rptr[mid] <= s) lo = mid; else hi = mid;
    }
    const int64_t i = lo, j = v.col[s];
    float2 *K = op == 0 ? K0 : (op == 1 ? K1 : K2);
    float2 &z = K[(2 * i + al) * n2 + 2 * j + be];
    const double2 a = v.val[12 * s + c];
    z.x = (float)((double)z.x + a.x);
    z.y = (float)((double)z.y + a.y);
}

// Kc[op][(2 i + al) n2 + 2 j + be] += store value (complex128 blocks; any
// block pointer may be null), one thread per stored value.
__global__ void k_near_add_dense(int64_t nn, int64_t n2, NearView v, int64_t nnz, double2 *K0, double2 *K1,
                                 double2 *K2) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= 12 * nnz) return;
    const int64_t s = id / 12;
    const int c = (int)(id % 12), op = c >> 2, al = (c >> 1) & 1, be = c & 1;
    double2 *K = op == 0 ? K0 : (op == 1 ? K1 : K2);
    if (!K) return;
    int64_t lo = 0, hi = nn;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (v.rptr[mid] <= s) lo = mid; else hi = mid;
    }
    double2 &z = K[(2 * lo + al) * n2 + 2 * (int64_t)v.col[s] + be];
    const double2 a = v.val[12 * s + c];
    z.x += a.x;
    z.y += a.y;
}

}  // namespace

int near_add_dense_run(const mbem_op *op, double2 *K1, double2 *K2e, double2 *K2m, hipStream_t s) {
    if (!op->near_on || op->near_nnz == 0) return MBEM_OK;
    hipLaunchKernelGGL(k_near_add_dense, dim3((unsigned)((12 * op->near_nnz + 255) / 256)), dim3(256), 0, s,
                       op->mesh->nn, op->n2, op->near_view(), op->near_nnz, K1, K2e, K2m);
    MBEM_HIP(hipGetLastError());
    return MBEM_OK;
}

void near_free(mbem_op *op) {
    void *ps[] = {op->d_nbits, op->d_nwpre, op->d_nrptr, op->d_ncol, op->d_nval, op->d_nmask, op->d_ncount,
                  op->d_ntiles, op->d_ncursor};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    op->d_nbits = nullptr; op->d_nwpre = op->d_nrptr = op->d_ncol = nullptr;
    op->d_nval = nullptr; op->d_nmask = nullptr; op->d_ncount = nullptr;
    op->d_ntiles = nullptr; op->d_ncursor = nullptr;
    op->near_on = false;
    op->near_nw = op->near_nnz = op->near_cap = op->near_tile_cap = 0;
    op->near_tile_off.clear();
}

int near_build_run(mbem_op *op, double near_r, hipStream_t s) {
    const mbem_mesh *m = op->mesh;
    const int64_t nn = m->nn, nt = m->nt, nch = (nt + kChunk - 1) / kChunk;
    const int64_t nw = (nn + 31) / 32;
    const int ntc = (int)m->tcol_off.size() - 1, ncc = (int)m->ccol_off.size() - 1;
    const int64_t nlaunch = (int64_t)ntc * ncc;
    if (!op->d_nbits) {
        MBEM_HIP(hipMalloc((void **)&op->d_nbits, sizeof(uint32_t) * nn * nw));
        MBEM_HIP(hipMalloc((void **)&op->d_nwpre, sizeof(int32_t) * nn * nw));
        MBEM_HIP(hipMalloc((void **)&op->d_nrptr, sizeof(int32_t) * (nn + 1)));
        MBEM_HIP(hipMalloc((void **)&op->d_nmask, sizeof(uint8_t) * nt * nch));
        MBEM_HIP(hipMalloc((void **)&op->d_ncount, sizeof(unsigned long long) * (2 + nlaunch)));
        MBEM_HIP(hipMalloc((void **)&op->d_ncursor, sizeof(unsigned long long) * nlaunch));
        op->near_nw = nw;
    }
    MBEM_HIP(hipMemsetAsync(op->d_nbits, 0, sizeof(uint32_t) * nn * nw, s));
    MBEM_HIP(hipMemsetAsync(op->d_ncount, 0, sizeof(unsigned long long) * (2 + nlaunch), s));
    hipLaunchKernelGGL(k_near_mark, dim3((unsigned)((nt * nch + 255) / 256)), dim3(256), 0, s, nt, nch, nw,
                       m->d_tri, m->d_elem, near_r, m->d_tcolour, m->d_ccolour, ncc, op->d_nbits, op->d_nmask,
                       op->d_ncount);
    MBEM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_near_count, dim3((unsigned)((nn * 64 + 255) / 256)), dim3(256), 0, s, nn, nw, op->d_nbits,
                       op->d_nwpre, op->d_nrptr + 1);
    MBEM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_near_scan, dim3(1), dim3(1024), 0, s, nn, op->d_nrptr, op->d_ncount + 1);
    MBEM_HIP(hipGetLastError());
    std::vector<unsigned long long> h(2 + nlaunch);
    MBEM_HIP(hipMemcpyAsync(h.data(), op->d_ncount, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, s));
    MBEM_HIP(hipStreamSynchronize(s));
    const int64_t nnz = (int64_t)h[1];
    if (nnz > 0x7fffffffLL) { set_error("near store pattern too large"); return MBEM_ENOMEM; }
    // tiles with near pairs, grouped by launch
    op->near_tile_off.assign(nlaunch + 1, 0);
    for (int64_t L = 0; L < nlaunch; ++L) op->near_tile_off[L + 1] = op->near_tile_off[L] + (int64_t)h[2 + L];
    const int64_t ntile = op->near_tile_off[nlaunch];
    if (ntile > op->near_tile_cap) {
        if (op->d_ntiles) { MBEM_HIP(hipFree(op->d_ntiles)); op->d_ntiles = nullptr; }
        op->near_tile_cap = 0;
        if (hipMalloc((void **)&op->d_ntiles, sizeof(int2) * ntile) != hipSuccess) {
            set_error("near store: out of device memory");
            return MBEM_ENOMEM;
        }
        op->near_tile_cap = ntile;
    }
    if (nnz > op->near_cap) {
        if (op->d_ncol) { MBEM_HIP(hipFree(op->d_ncol)); op->d_ncol = nullptr; }
        if (op->d_nval) { MBEM_HIP(hipFree(op->d_nval)); op->d_nval = nullptr; }
        op->near_cap = 0;
        if (hipMalloc((void **)&op->d_ncol, sizeof(int32_t) * (nnz > 0 ? nnz : 1)) != hipSuccess ||
            hipMalloc((void **)&op->d_nval, sizeof(double2) * 12 * (nnz > 0 ? nnz : 1)) != hipSuccess) {
            set_error("near store: out of device memory");
            return MBEM_ENOMEM;
        }
        op->near_cap = nnz;
    }
    op->near_nnz = nnz;
    op->n_near = (int64_t)h[0];
    if (ntile > 0) {
        std::vector<unsigned long long> cur(op->near_tile_off.begin(), op->near_tile_off.end() - 1);
        MBEM_HIP(hipMemcpyAsync(op->d_ncursor, cur.data(), sizeof(unsigned long long) * nlaunch,
                                hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_near_tiles, dim3((unsigned)((nt * nch + 255) / 256)), dim3(256), 0, s, nt, nch,
                           op->d_nmask, m->d_tcolour, m->d_ccolour, ncc, op->d_ncursor, op->d_ntiles);
        MBEM_HIP(hipGetLastError());
        // the cursors are read from host memory until the copy has run
        MBEM_HIP(hipStreamSynchronize(s));
    }
    MBEM_HIP(hipMemsetAsync(op->d_nval, 0, sizeof(double2) * 12 * (nnz > 0 ? nnz : 1), s));
    hipLaunchKernelGGL(k_near_cols, dim3((unsigned)((nn * 64 + 255) / 256)), dim3(256), 0, s, nn, nw, op->d_nbits,
                       op->d_nwpre, op->d_nrptr, op->d_ncol);
    MBEM_HIP(hipGetLastError());
    op->near_on = true;
    return MBEM_OK;
}

int near_fold_run(mbem_op *op, hipStream_t s) {
    if (!op->near_on) return MBEM_OK;
    const NearView v = op->near_view();
    if (op->near_nnz > 0)
        hipLaunchKernelGGL(k_near_fold, dim3((unsigned)((12 * op->near_nnz + 255) / 256)), dim3(256), 0, s,
                           op->mesh->nn, op->n2, v, op->near_nnz, (float2 *)op->K[0], (float2 *)op->K[1],
                           (float2 *)op->K[2]);
    MBEM_HIP(hipGetLastError());
    MBEM_HIP(hipStreamSynchronize(s));
    near_free(op);
    return MBEM_OK;
}

}  // namespace mbem
