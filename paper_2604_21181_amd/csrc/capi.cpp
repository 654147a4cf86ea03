// The C ABI of include/mbem.h: handle management, orchestration of the
// device kernels, and the GMRES driver.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>

#include "gemm.h"
#include "mbem_internal.h"

namespace mbem {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

// The host spins on the tag.  Asking the stream for its state puts a marker
// into it, which idles the device for microseconds between two kernels, so
// that is done only after 20 ms without the tag (the steps that publish
// tags take far less): a failed or drained stream ends the wait with an
// error, and so does a minute without the tag.
int wait_host_tag(const unsigned long long *tag, unsigned long long seq, hipStream_t s, const char *what) {
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    auto next_query = t0 + std::chrono::milliseconds(20);
    for (unsigned spins = 1;; ++spins) {
        if (__atomic_load_n(tag, __ATOMIC_ACQUIRE) == seq) return MBEM_OK;
        if (spins % 1024) continue;
        const auto now = clock::now();
        if (now < next_query) continue;
        next_query = now + std::chrono::milliseconds(20);
        const hipError_t e = hipStreamQuery(s);
        if (e != hipSuccess && e != hipErrorNotReady) MBEM_HIP(e);
        if (e == hipSuccess && __atomic_load_n(tag, __ATOMIC_ACQUIRE) != seq) {
            set_error(std::string("the stream drained without the ") + what);
            return MBEM_EDEVICE;
        }
        if (now - t0 > std::chrono::seconds(60)) {
            set_error(std::string("no ") + what + " within a minute");
            return MBEM_EDEVICE;
        }
    }
}

template <typename T>
static int dalloc(T **p, size_t n) {
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * n);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return MBEM_ENOMEM;
    }
    return MBEM_OK;
}

template <typename T>
static int upload(T **p, const std::vector<T> &v, hipStream_t s) {
    MBEM_TRY(dalloc(p, v.size()));
    if (!v.empty()) MBEM_HIP(hipMemcpyAsync(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    return MBEM_OK;
}

static void dfree(void *p) {
    if (p) (void)hipFree(p);
}

// Frees a device allocation when the scope ends (error returns included).
struct Owned {
    void *p = nullptr;
    Owned() = default;
    Owned(const Owned &) = delete;
    Owned &operator=(const Owned &) = delete;
    ~Owned() { dfree(p); }
};

// Elapsed milliseconds between two events recorded on the stream.
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() { (void)hipEventCreate(&a); (void)hipEventCreate(&b); }
    ~Timer() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    void start(hipStream_t s) { (void)hipEventRecord(a, s); }
    double stop(hipStream_t s) {
        float ms = 0.f;
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
};

static int set_device(const mbem_ctx *ctx) {
    if (!ctx) { set_error("null context"); return MBEM_EINVAL; }
    MBEM_HIP(hipSetDevice(ctx->device));
    return MBEM_OK;
}

static void mesh_free_device(mbem_mesh *m) {
    void *ps[] = {m->d_xyz, m->d_tri, m->d_inc_ptr, m->d_inc, m->d_spairs, m->d_frames,
                  m->d_qp, m->d_qp32, m->d_elem, m->d_mptr, m->d_mcol, m->d_mslot,
                  m->d_chunks, m->d_tcol, m->d_ccol, m->d_tcolour, m->d_ccolour, m->d_qp12, m->d_qp12_32,
                  m->d_rng_off, m->d_rng_rec, m->d_row_first, m->d_col_first};
    for (void *p : ps) dfree(p);
}

static void op_free_device(mbem_op *op) {
    near_free(op);
    for (int o = 0; o < 3; ++o) dfree(op->K[o]);
    for (int o = 0; o < 3; ++o) dfree(op->K32[o]);
    dfree(op->d_mval);
    dfree(op->d_minv);
    dfree(op->d_minv_t);
    dfree(op->d_minv32);
    dfree(op->d_minv_t32);
    dfree(op->d_lu);
    dfree(op->d_work);
    dfree(op->d_kconst);
    dfree(op->d_rtab);
    if (op->h_pin) (void)hipHostFree(op->h_pin);
    op->h_pin = nullptr;
    blr_free(op->blr);
    op->blr = nullptr;
    fill_state_free(op->fs);
    op->fs = nullptr;
}

// ---------------------------------------------------------------- GMRES --
// trans: the same iteration on Z^T with P^-T (adjoint systems).
struct Gmres {
    const mbem_op *op;
    hipStream_t s;
    int64_t N;
    int m;              // Krylov dimension limit
    bool trans = false;
    bool lowp = false;          // MIXED: the complex64 copy of the block-Jacobi inverses
    double2 *V, *w, *z, *tmp, *hdev;
    double2 *W;                 // the products Z z_j of the steps, (m + 1) x N
    double2 *tpart = nullptr;   // partial sums of the transposed product
    double *ndev;
    double2 *hcol;              // the current step's projection coefficients (device)
    double2 *ppart;             // projection partials of both passes, 2 (m + 1) x chunks
    double *npart;              // per-chunk parts of |w|^2
    // two Hessenberg column slots in pinned host memory, each 2 (m + 1) + 1
    // values and a completion tag, and the same slots as the kernels
    // address them
    double2 *hpin[2] = {nullptr, nullptr};
    double2 *hmap[2] = {nullptr, nullptr};
    double2 *ypin = nullptr;    // the final coefficients y (pinned host memory)
    // matvec timing: events around the products of Arnoldi steps kTimed0 ..
    // kTimed0 + kTimedSteps - 1 only.  An event between two kernels costs
    // the stream several microseconds of idle time, and the first steps'
    // products start on an idle stream, so their events would also time
    // the host's launches.
    static constexpr int kTimed0 = 2, kTimedSteps = 2;
    hipEvent_t ev0[kTimedSteps] = {}, ev1[kTimedSteps] = {};
    double t_matvec = 0.0;
    int n_matvec = 0;
    ~Gmres() {
        for (int i = 0; i < kTimedSteps; ++i) {
            if (ev0[i]) (void)hipEventDestroy(ev0[i]);
            if (ev1[i]) (void)hipEventDestroy(ev1[i]);
        }
        if (tpart) (void)hipFree(tpart);
    }
    int apply(const double2 *x, double2 *y) {   // y = Z x or Z^T x
        return trans ? matvec_t_run(op, x, y, tpart, s) : matvec_run(op, x, y, tmp, s);
    }
    static bool timed(int q) { return q >= kTimed0 && q < kTimed0 + kTimedSteps; }
    int step_matvec(const double2 *x, double2 *y, int q) {
        if (!timed(q)) return apply(x, y);
        const int e = q - kTimed0;
        MBEM_HIP(hipEventRecord(ev0[e], s));
        if (trans) {
            MBEM_TRY(matvec_t_run(op, x, y, tpart, s));
            MBEM_HIP(hipEventRecord(ev1[e], s));
            return MBEM_OK;
        }
        return matvec_run(op, x, y, tmp, s, ev1[e]);   // ev1 right after the GEMV
    }
    void collect(int q) {   // once step q's column has arrived
        if (!timed(q)) return;
        const int e = q - kTimed0;
        float t = 0.f;
        if (hipEventSynchronize(ev1[e]) == hipSuccess &&
            hipEventElapsedTime(&t, ev0[e], ev1[e]) == hipSuccess) { t_matvec += t; ++n_matvec; }
    }
    // Wait until the tag `seq` of step `slot` is in pinned memory.
    int wait_column(int slot, unsigned long long seq) const {
        return wait_host_tag((const unsigned long long *)(hpin[slot] + 2 * (m + 1) + 1), seq, s,
                             "GMRES Arnoldi column");
    }
};

static int gmres_alloc(Gmres &g, const mbem_op *op, int maxit, hipStream_t s) {
    g.op = op;
    g.s = s;
    g.lowp = op->prec == MBEM_MIXED;
    g.N = 2 * op->n2;
    g.m = maxit;
    // V, w, z, matvec partials (4 n2), the coefficients y (m) and a norm,
    // the step's column, projection partials of both passes, norm partials
    const size_t nch = (size_t)arnoldi_chunks(g.N);
    const size_t col = 2 * (size_t)(maxit + 1) + 1;
    const size_t need = (size_t)(maxit + 1) * g.N + 2 * g.N + 4 * op->n2 + (size_t)maxit + 1 + col +
                        2 * (size_t)(maxit + 1) * nch + nch + 1 + (size_t)(maxit + 1) * g.N;
    mbem_op *mop = const_cast<mbem_op *>(op);
    if (op->work_elems < need) {
        dfree(mop->d_work);
        mop->d_work = nullptr;
        mop->work_elems = 0;
        MBEM_TRY(dalloc(&mop->d_work, need));
        mop->work_elems = need;
    }
    // two column slots of col values and a tag, written by the Arnoldi
    // kernels straight into fine-grained host memory, then y
    const size_t pin = 2 * (col + 1) + (size_t)maxit;
    if (op->pin_elems < pin) {
        if (mop->h_pin) (void)hipHostFree(mop->h_pin);
        mop->h_pin = nullptr;
        mop->pin_elems = 0;
        MBEM_HIP(hipHostMalloc((void **)&mop->h_pin, sizeof(double2) * pin,
                               hipHostMallocMapped | hipHostMallocCoherent));
        mop->pin_elems = pin;
    }
    g.hpin[0] = op->h_pin;
    g.hpin[1] = op->h_pin + col + 1;
    g.ypin = op->h_pin + 2 * (col + 1);
    for (int i = 0; i < 2; ++i) MBEM_HIP(hipHostGetDevicePointer((void **)&g.hmap[i], g.hpin[i], 0));
    g.V = op->d_work;
    g.w = g.V + (size_t)(maxit + 1) * g.N;
    g.z = g.w + g.N;
    g.tmp = g.z + g.N;                 // 4 n2 for the matvec partials
    g.hdev = g.tmp + 4 * op->n2;       // the coefficients y of the final combination
    g.ndev = (double *)(g.hdev + maxit);
    g.hcol = g.hdev + maxit + 1;
    g.ppart = g.hcol + col;
    g.npart = (double *)(g.ppart + 2 * (size_t)(maxit + 1) * nch);
    g.W = g.ppart + 2 * (size_t)(maxit + 1) * nch + (nch + 1) / 2 + 1;   // after the nch doubles of npart
    for (int i = 0; i < Gmres::kTimedSteps; ++i) {
        if (!g.ev0[i]) MBEM_HIP(hipEventCreate(&g.ev0[i]));
        if (!g.ev1[i]) MBEM_HIP(hipEventCreate(&g.ev1[i]));
    }
    if (g.trans && !g.tpart) MBEM_TRY(dalloc(&g.tpart, (size_t)matvec_t_work(op)));
    return MBEM_OK;
}

static inline std::complex<double> C(double2 v) { return {v.x, v.y}; }

// Right-preconditioned GMRES on Z P^-1, x0 = 0, CGS2 Arnoldi in FP64.
// Solves Z x = b to |r_k| <= tol |b| (Arnoldi estimate); beta = |b| is the
// caller's (it has just computed it).  x, b device.
// The host lags the device by one column: Arnoldi step k (preconditioner,
// matvec, two projection passes, norm, and V_{k+1} = w / h_{k+1,k} with the
// norm read on the device) is queued before the host waits for column k-1
// and applies its Givens rotation, so the stream never drains between
// steps.  When column k-1 meets the tolerance the queued step k is unused.
// Returns with x's last kernels queued, not finished.
static int gmres_solve(Gmres &g, const double2 *b, double beta, double tol, double2 *x, int *iters,
                       double *est) {
    const hipStream_t s = g.s;
    const int64_t N = g.N;
    if (!(beta > 0)) {
        MBEM_HIP(hipMemsetAsync(x, 0, sizeof(double2) * N, s));
        *iters = 0;
        *est = 0;
        return MBEM_OK;
    }
    const int m = g.m;
    // The Hessenberg matrix, column-major (column k holds rows 0..k+1),
    // kept across solves: allocating and zeroing (m + 1) m entries for every
    // solve, and releasing them, left the stream idle for about 0.1 ms at
    // each end of a solve; every entry read has been written first.
    static thread_local std::vector<std::complex<double>> Hbuf;
    if (Hbuf.size() < (size_t)(m + 1) * m) Hbuf.resize((size_t)(m + 1) * m);
    std::complex<double> *const H = Hbuf.data();
    std::vector<std::complex<double>> cs(m), sn(m), gv(m + 1);
    gv[0] = beta;
    // no tag of an earlier solve may match; no Arnoldi kernel of one is
    // pending (the caller synchronises between solves)
    for (int i = 0; i < 2; ++i) *(unsigned long long *)(g.hpin[i] + 2 * (m + 1) + 1) = 0ull;
    MBEM_TRY(vec_scale_copy(g.V, b, double2{1.0 / beta, 0.0}, N, s));
    // queue Arnoldi step k; its column lands in hpin[k % 2] with tag k + 1.
    // With a preconditioner the step's normalisation and column run as the
    // first launch of step k + 1 (fused with its block-Jacobi product), or
    // as arnoldi_finish after the last step.
    const bool fuse = mbj_present(g.op);
    auto tag_of = [&](int slot) { return (unsigned long long *)(g.hmap[slot] + 2 * (m + 1) + 1); };
    auto enqueue = [&](int k) -> int {
        const int slot = k & 1;
        double2 *vk = g.V + (size_t)k * N;
        if (fuse && k > 0) {
            const int ps = (k - 1) & 1;
            MBEM_TRY(mbj_scale_apply_run(g.op, g.w, g.npart, N, vk, g.z, g.hcol, k, g.hmap[ps], tag_of(ps),
                                         (unsigned long long)k, s, g.trans, g.lowp));
        } else {
            MBEM_TRY(mbj_apply_run(g.op, vk, g.z, s, g.trans, g.lowp));
        }
        double2 *wk = g.W + (size_t)k * N;   // Z z_k, kept for the residual of the solution
        MBEM_TRY(g.step_matvec(g.z, wk, k));
        MBEM_TRY(arnoldi_cgs2(wk, g.w, g.V, N, k + 1, N, g.ppart, g.npart, g.hcol, !fuse, g.hmap[slot],
                              tag_of(slot), (unsigned long long)k + 1, s));
        return MBEM_OK;
    };
    double res = 1.0;
    bool conv = false, breakdown = false;
    // wait for column k and fold it into the QR factorisation of H
    auto process = [&](int k) -> int {
        const int slot = k & 1;
        MBEM_TRY(g.wait_column(slot, (unsigned long long)k + 1));
        g.collect(k);
        const double2 *hb = g.hpin[slot];
        const double hn = hb[2 * (k + 1)].x;
        auto Hc = [&](int i) -> std::complex<double> & { return H[(size_t)k * (m + 1) + i]; };
        for (int i = 0; i <= k; ++i) Hc(i) = C(hb[i]) + C(hb[k + 1 + i]);
        Hc(k + 1) = hn;
        for (int i = 0; i < k; ++i) {
            const std::complex<double> t = cs[i] * Hc(i) + sn[i] * Hc(i + 1);
            Hc(i + 1) = -std::conj(sn[i]) * Hc(i) + cs[i] * Hc(i + 1);
            Hc(i) = t;
        }
        const std::complex<double> a = Hc(k), bb = Hc(k + 1);
        const double r = std::hypot(std::abs(a), std::abs(bb));
        if (r == 0) { cs[k] = 1; sn[k] = 0; }
        else if (std::abs(a) == 0) { cs[k] = 0; sn[k] = std::conj(bb) / std::abs(bb); }
        else { cs[k] = std::abs(a) / r; sn[k] = (a / std::abs(a)) * std::conj(bb) / r; }
        Hc(k) = cs[k] * a + sn[k] * bb;
        Hc(k + 1) = 0;
        gv[k + 1] = -std::conj(sn[k]) * gv[k];
        gv[k] = cs[k] * gv[k];
        res = std::abs(gv[k + 1]) / beta;
        breakdown = hn == 0;
        conv = res <= tol || breakdown;
        return MBEM_OK;
    };
    // The column that meets the tolerance normally finds the next step
    // already queued, and that step is wasted.  When the last two residual
    // estimates extrapolate (at their ratio) to the tolerance at column
    // q - 1, the host instead waits for that column before queueing step q:
    // a short drain of the stream if the guess is wrong, one step saved if
    // it is right.  With the fused start the column is published by step
    // q's first launch, so it is published here by arnoldi_finish (step q
    // then recomputes the same V_q and publishes the column once more).
    double r_prev = 0.0, r_last = 0.0;   // estimates after the last two columns
    int k = 0;       // columns folded into H
    for (int q = 0; q < m; ++q) {
        if (q >= 3 && r_prev > 0 && r_last * (r_last / r_prev) <= tol) {
            if (fuse)
                MBEM_TRY(arnoldi_finish(g.w, g.V, N, q, N, g.npart, g.hcol, g.hmap[(q - 1) & 1],
                                        tag_of((q - 1) & 1), (unsigned long long)q, s));
            MBEM_TRY(process(q - 1));
            k = q;
            r_prev = r_last;
            r_last = res;
            if (conv) break;
            MBEM_TRY(enqueue(q));
            continue;
        }
        MBEM_TRY(enqueue(q));
        if (q >= 1) {
            MBEM_TRY(process(q - 1));
            k = q;
            r_prev = r_last;
            r_last = res;
            if (conv) break;
        }
    }
    if (!conv) {
        if (fuse)
            MBEM_TRY(arnoldi_finish(g.w, g.V, N, m, N, g.npart, g.hcol, g.hmap[(m - 1) & 1], tag_of((m - 1) & 1),
                                    (unsigned long long)m, s));
        MBEM_TRY(process(m - 1));
        k = m;
    }
    conv = res <= tol || breakdown;
    // back substitution H y = g
    std::vector<std::complex<double>> y(k);
    for (int i = k - 1; i >= 0; --i) {
        std::complex<double> t = gv[i];
        for (int j = i + 1; j < k; ++j) t -= H[(size_t)j * (m + 1) + i] * y[j];
        y[i] = t / H[(size_t)i * (m + 1) + i];
    }
    // y through pinned memory: no earlier copy from it is pending (the
    // caller synchronises between solves), so the host needs no wait here
    for (int i = 0; i < k; ++i) g.ypin[i] = {y[i].real(), y[i].imag()};
    MBEM_HIP(hipMemcpyAsync(g.hdev, g.ypin, sizeof(double2) * k, hipMemcpyHostToDevice, s));
    MBEM_TRY(vec_combine(g.w, g.V, N, k, g.hdev, N, s));
    MBEM_TRY(mbj_apply_run(g.op, g.w, x, s, g.trans, g.lowp));
    *iters = k;
    *est = res;
    return conv ? MBEM_OK : MBEM_ENOCONV;
}

// Device buffers of the cross-section evaluation, grown on demand and kept
// across the points of a sweep.
struct CsWork {
    int64_t cap = 0;
    double *dirs = nullptr, *w = nullptr, *acc = nullptr;
    double2 *F = nullptr;
    CsWork() = default;
    CsWork(const CsWork &) = delete;
    CsWork &operator=(const CsWork &) = delete;
    ~CsWork() { release(); }
    void release() {
        dfree(dirs); dfree(w); dfree(acc); dfree(F);
        dirs = w = acc = nullptr; F = nullptr; cap = 0;
    }
    int reserve(int64_t ndir) {
        if (ndir <= cap) return MBEM_OK;
        release();
        MBEM_TRY(dalloc(&dirs, 3 * ndir));
        MBEM_TRY(dalloc(&w, ndir));
        MBEM_TRY(dalloc(&acc, 2));
        MBEM_TRY(dalloc(&F, 3 * ndir));
        cap = ndir;
        return MBEM_OK;
    }
};

// C_ext by the optical theorem, C_sca by the product rule on the unit sphere
// (Gauss-Legendre in cos theta x trapezoid in phi), C_abs by the surface
// integral of the currents; ntheta <= 0 picks 2 k0 a_max + 20.
// Post-processing reads the basis through p->frame: only the two frames
static int check_frame(const mbem_params *p) {
    if (p->frame != MBEM_FRAME_INTERPOLATED && p->frame != MBEM_FRAME_NODAL) {
        set_error("unknown tangential frame");
        return MBEM_EINVAL;
    }
    return MBEM_OK;
}

static int cross_sections_impl(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, const double2 *x,
                               const double *khat, const mbem_c128 *pol, int32_t ntheta, double *out,
                               CsWork &cw) {
    const hipStream_t s = ctx->stream;
    if (ntheta <= 0) ntheta = (int32_t)std::ceil(2.0 * p->k0 * mesh->amax) + 20;
    const int nphi = 2 * ntheta;
    const int64_t ndir = (int64_t)ntheta * nphi + 1;   // last one: khat
    std::vector<double> dirs(3 * ndir), w(ndir, 0.0), u(ntheta), wu(ntheta);
    gauss_legendre(ntheta, u.data(), wu.data());
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < ntheta; ++i)
        for (int j = 0; j < nphi; ++j) {
            const double ph = 2.0 * pi * j / nphi, st = std::sqrt(std::max(0.0, 1.0 - u[i] * u[i]));
            const int64_t d = (int64_t)i * nphi + j;
            dirs[3 * d] = st * std::cos(ph);
            dirs[3 * d + 1] = st * std::sin(ph);
            dirs[3 * d + 2] = u[i];
            w[d] = wu[i] * 2.0 * pi / nphi;
        }
    for (int k = 0; k < 3; ++k) dirs[3 * (ndir - 1) + k] = khat[k];
    MBEM_TRY(cw.reserve(ndir));
    MBEM_HIP(hipMemcpyAsync(cw.dirs, dirs.data(), sizeof(double) * 3 * ndir, hipMemcpyHostToDevice, s));
    MBEM_HIP(hipMemcpyAsync(cw.w, w.data(), sizeof(double) * ndir, hipMemcpyHostToDevice, s));
    MBEM_TRY(farfield_run(mesh, p, x, 1, cw.dirs, ndir, cw.F, s));
    MBEM_TRY(weighted_norm_run(ndir, cw.F, cw.w, cw.acc, s));
    MBEM_TRY(absorbed_run(mesh, p, x, cw.acc + 1, s));
    double acc[2];
    double2 Ff[3];
    MBEM_HIP(hipMemcpyAsync(acc, cw.acc, sizeof(acc), hipMemcpyDeviceToHost, s));
    MBEM_HIP(hipMemcpyAsync(Ff, cw.F + 3 * (ndir - 1), sizeof(Ff), hipMemcpyDeviceToHost, s));
    MBEM_HIP(hipStreamSynchronize(s));   // dirs and w are host vectors of this frame
    std::complex<double> pe(0.0, 0.0);
    for (int k = 0; k < 3; ++k) pe += std::conj(std::complex<double>(pol[k].re, pol[k].im)) * C(Ff[k]);
    out[0] = 4.0 * pi / p->k0 * pe.imag();
    out[1] = acc[0];
    out[2] = acc[1];
    return MBEM_OK;
}

}  // namespace mbem

using namespace mbem;

extern "C" {

const char *mbem_last_error(void) { return g_err.c_str(); }

int mbem_ctx_create(int device, void *hip_stream, mbem_ctx **out) {
    if (!out) { set_error("null output"); return MBEM_EINVAL; }
    int n = 0;
    MBEM_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) { set_error("device ordinal out of range"); return MBEM_EINVAL; }
    mbem_ctx *c = new (std::nothrow) mbem_ctx;
    if (!c) { set_error("host allocation"); return MBEM_ENOMEM; }
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return MBEM_OK;
}

void mbem_ctx_destroy(mbem_ctx *ctx) { delete ctx; }

int mbem_morton_order(const double *xyz, int64_t n_nodes, const int64_t *tri6, int64_t n_tris,
                      int64_t *node_order, int64_t *tri_order) {
    if (!xyz || !tri6 || n_nodes <= 0 || n_tris <= 0) { set_error("bad arguments"); return MBEM_EINVAL; }
    for (int64_t i = 0; i < 6 * n_tris; ++i)
        if (tri6[i] < 0 || tri6[i] >= n_nodes) { set_error("node index out of range"); return MBEM_EINVAL; }
    std::vector<int64_t> no, to;
    MBEM_TRY(morton_order_host(xyz, n_nodes, tri6, n_tris, no, to));
    if (node_order) std::copy(no.begin(), no.end(), node_order);
    if (tri_order) std::copy(to.begin(), to.end(), tri_order);
    return MBEM_OK;
}

int mbem_mesh_create(mbem_ctx *ctx, const double *xyz, int64_t n_nodes, const int64_t *tri6,
                     int64_t n_tris, mbem_mesh **out) {
    if (!out || !xyz || !tri6) { set_error("null argument"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    mbem_mesh *m = new (std::nothrow) mbem_mesh;
    if (!m) { set_error("host allocation"); return MBEM_ENOMEM; }
    m->ctx = ctx;
    int st = build_mesh_host(xyz, n_nodes, tri6, n_tris, m);
    MeshTables T;
    if (st == MBEM_OK) st = build_tables(m, T);
    const hipStream_t s = ctx->stream;
    auto fail = [&](int code) { mesh_free_device(m); delete m; return code; };
    if (st != MBEM_OK) return fail(st);
    m->n_spairs = (int64_t)T.spairs.size() / 4;
    for (int c = 0; c < 4; ++c) m->n_single[c] = T.n_single[c];
    m->m_ptr = T.m_ptr;
    m->m_col = T.m_col;
    m->tcol_off = T.tcol_off;
    m->nrng = (int64_t)T.rng_off.size() - 1;
    m->ccol_off = T.ccol_off;
    m->tcol_list = T.tcol_list;
    m->spairs = T.spairs;
    const int64_t nq = m->nt * kQP;
    std::vector<int32_t> tcolour(m->nt), ccolour(T.ccol_list.size());
    for (size_t c = 0; c + 1 < T.tcol_off.size(); ++c)
        for (int32_t q = T.tcol_off[c]; q < T.tcol_off[c + 1]; ++q) tcolour[T.tcol_list[q]] = (int32_t)c;
    for (size_t c = 0; c + 1 < T.ccol_off.size(); ++c)
        for (int32_t q = T.ccol_off[c]; q < T.ccol_off[c + 1]; ++q) ccolour[T.ccol_list[q]] = (int32_t)c;
    if ((st = upload(&m->d_tcolour, tcolour, s)) || (st = upload(&m->d_ccolour, ccolour, s)) ||
        (st = upload(&m->d_xyz, m->xyz, s)) || (st = upload(&m->d_tri, m->tri, s)) ||
        (st = upload(&m->d_inc_ptr, T.inc_ptr, s)) || (st = upload(&m->d_inc, T.inc, s)) ||
        (st = upload(&m->d_spairs, T.spairs, s)) || (st = upload(&m->d_mptr, T.m_ptr, s)) ||
        (st = upload(&m->d_mcol, T.m_col, s)) || (st = upload(&m->d_mslot, T.m_slot, s)) ||
        (st = upload(&m->d_chunks, T.chunks, s)) || (st = upload(&m->d_tcol, T.tcol_list, s)) ||
        (st = upload(&m->d_ccol, T.ccol_list, s)) || (st = upload(&m->d_rng_off, T.rng_off, s)) ||
        (st = upload(&m->d_rng_rec, T.rng_rec, s)) || (st = upload(&m->d_row_first, T.row_first, s)) ||
        (st = upload(&m->d_col_first, T.col_first, s)) ||
        (st = dalloc(&m->d_frames, 9 * m->nn)) || (st = dalloc(&m->d_qp, kQPF * nq)) ||
        (st = dalloc(&m->d_qp32, kQPF * nq)) || (st = dalloc(&m->d_elem, 4 * m->nt)) ||
        (st = dalloc(&m->d_qp12, kQPF * m->nt * kQP12)) || (st = dalloc(&m->d_qp12_32, kQPF * m->nt * kQP12)))
        return fail(st);
    if ((st = geom_build(m, s))) return fail(st);
    if (hipStreamSynchronize(s) != hipSuccess) { set_error("mesh upload failed"); return fail(MBEM_EDEVICE); }
    *out = m;
    return MBEM_OK;
}

void mbem_mesh_destroy(mbem_mesh *m) {
    if (!m) return;
    if (m->ctx) (void)hipSetDevice(m->ctx->device);
    if (m->ctx) (void)hipStreamSynchronize(m->ctx->stream);
    mesh_free_device(m);
    delete m;
}

int mbem_mesh_permutation(const mbem_mesh *m, int64_t *node_order, int64_t *tri_order) {
    if (!m) { set_error("null mesh"); return MBEM_EINVAL; }
    if (node_order) std::copy(m->node_order.begin(), m->node_order.end(), node_order);
    if (tri_order) std::copy(m->tri_order.begin(), m->tri_order.end(), tri_order);
    return MBEM_OK;
}

int mbem_mesh_frames(mbem_ctx *ctx, const mbem_mesh *m, double *frames) {
    if (!m || !frames) { set_error("null argument"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    std::vector<double> f(9 * m->nn);
    MBEM_HIP(hipMemcpyAsync(f.data(), m->d_frames, sizeof(double) * f.size(), hipMemcpyDeviceToHost, ctx->stream));
    MBEM_HIP(hipStreamSynchronize(ctx->stream));
    for (int64_t k = 0; k < m->nn; ++k)
        std::copy(f.begin() + 9 * k, f.begin() + 9 * k + 9, frames + 9 * m->node_order[k]);
    return MBEM_OK;
}

int mbem_mesh_info(const mbem_mesh *m, int64_t *info) {
    if (!m || !info) { set_error("null argument"); return MBEM_EINVAL; }
    info[0] = m->nn; info[1] = m->nt; info[2] = 4 * m->nn;
    info[3] = m->n_single[3]; info[4] = m->n_single[2]; info[5] = m->n_single[1];
    info[6] = 0; info[7] = 0;
    return MBEM_OK;
}

// Operator handle with its dense blocks and mass values allocated.
// Wavenumbers, interior material and the coefficients of the combined
// blocks (i/omega, (eps_i + 1)/2, (mu_i + 1)/2) of one frequency point.
static void op_set_material(mbem_op *op, const mbem_params *p) {
    op->p = *p;
    derive_constants(p, &op->ka, &op->ki, &op->eps_i, &op->mu_i);
    op->iw = {0.0, 1.0 / p->k0};
    op->ce = {(op->eps_i.x + 1.0) / 2.0, op->eps_i.y / 2.0};
    op->cm = {(op->mu_i.x + 1.0) / 2.0, op->mu_i.y / 2.0};
}

static int op_create(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, mbem_op **out,
                     bool dense = true) {
    if (!p || !out) { set_error("null argument"); return MBEM_EINVAL; }
    // parameters first (host only), so that a bad one is named even without a mesh
    if (!std::isfinite(p->eps_r_re) || !std::isfinite(p->eps_r_im) || !std::isfinite(p->mu_r_re) ||
        !std::isfinite(p->mu_r_im) || !std::isfinite(p->near_radius)) {
        set_error("material parameters or near radius not finite");
        return MBEM_EINVAL;
    }
    if (!(p->k0 > 0) || !std::isfinite(p->k0)) { set_error("k0 must be positive and finite"); return MBEM_EINVAL; }
    if (!mesh) { set_error("null argument"); return MBEM_EINVAL; }
    if (p->precision != MBEM_FP64 && p->precision != MBEM_MIXED) { set_error("bad precision"); return MBEM_EINVAL; }
    if (p->ssq_order < 0 || p->ssq_order > kMaxSSQ) { set_error("ssq_order out of range"); return MBEM_EINVAL; }
    if (p->quadrature != MBEM_QUAD_DEFAULT && p->quadrature != MBEM_QUAD_PAPER) {
        set_error("unknown quadrature scheme");
        return MBEM_EINVAL;
    }
    if (p->frame != MBEM_FRAME_INTERPOLATED && p->frame != MBEM_FRAME_NODAL) {
        set_error("unknown tangential frame");
        return MBEM_EINVAL;
    }
    if (p->near_store != 0 && p->near_store != 1) { set_error("near_store must be 0 or 1"); return MBEM_EINVAL; }
    if (p->near_store && p->precision == MBEM_MIXED &&
        (p->quadrature != MBEM_QUAD_DEFAULT || p->frame != MBEM_FRAME_INTERPOLATED)) {
        set_error("the FP64 near store is built for the default quadrature and the interpolated frame");
        return MBEM_EINVAL;
    }
    MBEM_TRY(set_device(ctx));
    mbem_op *op = new (std::nothrow) mbem_op;
    if (!op) { set_error("host allocation"); return MBEM_ENOMEM; }
    op->ctx = ctx;
    op->mesh = mesh;
    op->prec = p->precision;
    op->n2 = 2 * mesh->nn;
    op_set_material(op, p);
    const size_t esz = op->prec == MBEM_FP64 ? 16 : 8;
    int st = MBEM_OK;
    for (int o = 0; o < 3 && st == MBEM_OK && dense; ++o) {
        hipError_t e = hipMalloc(&op->K[o], esz * op->n2 * op->n2);
        if (e != hipSuccess) { set_error(std::string("operator allocation: ") + hipGetErrorString(e)); st = MBEM_ENOMEM; }
    }
    if (st == MBEM_OK) st = dalloc(&op->d_mval, 4 * mesh->m_col.size());   // 2 x 2 per node pair
    if (st != MBEM_OK) { op_free_device(op); delete op; return st; }
    *out = op;
    return MBEM_OK;
}

static int op_fill(mbem_ctx *ctx, mbem_op *op, bool deriv, mbem_stats *stats) {
    Timer t;
    t.start(ctx->stream);
    int st = fill_run(op, ctx->stream, deriv);
    const double ms = t.stop(ctx->stream);
    if (st == MBEM_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) { set_error("fill failed"); st = MBEM_EDEVICE; }
    if (st == MBEM_OK && stats) {
        const mbem_mesh *mesh = op->mesh;
        stats->t_fill_ms = ms;
        stats->n_near_pairs = op->n_near;
        stats->t_geom_ms = op->t_phase[0];
        stats->t_regular_ms = op->t_phase[1];
        stats->t_near_ms = op->t_phase[2];
        stats->t_ssq_ms = op->t_phase[3];
        stats->t_mass_ms = op->t_phase[4];
        stats->n_regular_pairs = mesh->nt * mesh->nt - mesh->n_spairs;
    }
    return st;
}

int mbem_fill(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, mbem_op **out,
              mbem_stats *stats) {
    mbem_op *op = nullptr;
    MBEM_TRY(op_create(ctx, mesh, p, &op));
    const int st = op_fill(ctx, op, false, stats);
    if (st != MBEM_OK) { op_free_device(op); delete op; return st; }
    *out = op;
    return MBEM_OK;
}

int mbem_fill_compressed(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, const mbem_blr_opts *o,
                         mbem_op **out, mbem_stats *stats, mbem_blr_stats *bstats) {
    if (!mesh || !p || !o || !out) { set_error("null argument"); return MBEM_EINVAL; }
    if (p->precision != MBEM_FP64 || p->quadrature != MBEM_QUAD_DEFAULT) {
        set_error("the block low-rank operator is built for FP64 and the default quadrature");
        return MBEM_EINVAL;
    }
    if (o->cluster < 1 || o->cluster > 2048 || !(o->eta > 0) || !(o->eps > 0 && o->eps < 1) || o->rmax < 1 ||
        o->rmax > 128 || o->band < 0) {
        set_error("block low-rank options out of range (cluster 1..2048, eta > 0, 0 < eps < 1, rmax 1..128, "
                  "band >= 0)");
        return MBEM_EINVAL;
    }
    mbem_op *op = nullptr;
    MBEM_TRY(op_create(ctx, mesh, p, &op, false));
    Timer t;
    t.start(ctx->stream);
    mbem_blr_stats bs{};
    int st = blr_fill_run(op, o, &bs, ctx->stream);
    const double ms = t.stop(ctx->stream);
    if (st == MBEM_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) { set_error("fill failed"); st = MBEM_EDEVICE; }
    if (st != MBEM_OK) { mbem_op_destroy(op); return st; }
    bs.t_total_ms = ms;
    if (bstats) *bstats = bs;
    if (stats) {
        *stats = mbem_stats{};
        stats->t_fill_ms = ms;
        stats->t_regular_ms = bs.t_fill_ms;
        stats->n_regular_pairs = mesh->nt * mesh->nt - mesh->n_spairs;
    }
    *out = op;
    return MBEM_OK;
}

void mbem_op_destroy(mbem_op *op) {
    if (!op) return;
    if (op->ctx) { (void)hipSetDevice(op->ctx->device); (void)hipStreamSynchronize(op->ctx->stream); }
    op_free_device(op);
    delete op;
}

int mbem_op_export_blocks(mbem_ctx *ctx, const mbem_op *op, mbem_c128 *K1, mbem_c128 *K2e, mbem_c128 *K2m) {
    if (!op) { set_error("null operator"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    return export_blocks_run(op, (double2 *)K1, (double2 *)K2e, (double2 *)K2m, ctx->stream);
}

int mbem_op_export_dense(mbem_ctx *ctx, const mbem_op *op, mbem_c128 *Z) {
    if (!op || !Z) { set_error("null argument"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    return export_dense_run(op, (double2 *)Z, ctx->stream);
}

int mbem_matvec(mbem_ctx *ctx, const mbem_op *op, const mbem_c128 *x, int32_t nrhs, mbem_c128 *y) {
    if (!op || !x || !y || nrhs < 1) { set_error("bad argument"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    double2 *tmp = nullptr;
    MBEM_TRY(dalloc(&tmp, 4 * op->n2));
    const int64_t N = 2 * op->n2;
    int st = MBEM_OK;
    for (int r = 0; r < nrhs && st == MBEM_OK; ++r)
        st = matvec_run(op, (const double2 *)x + r * N, (double2 *)y + r * N, tmp, ctx->stream);
    (void)hipStreamSynchronize(ctx->stream);
    dfree(tmp);
    return st;
}

int mbem_precond_setup(mbem_ctx *ctx, mbem_op *op, int32_t block, mbem_stats *stats) {
    if (!op) { set_error("null operator"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    Timer t;
    t.start(ctx->stream);
    int st = mbj_setup_run(op, block, ctx->stream);
    const double ms = t.stop(ctx->stream);
    if (stats) stats->t_setup_ms = ms;
    return st;
}

int mbem_precond_apply(mbem_ctx *ctx, const mbem_op *op, const mbem_c128 *v, mbem_c128 *z) {
    if (!op || !v || !z) { set_error("null argument"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    return mbj_apply_run(op, (const double2 *)v, (double2 *)z, ctx->stream);
}

int mbem_rhs_planewave(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, const double *khat,
                       const mbem_c128 *pol, int32_t nrhs, mbem_c128 *b) {
    if (!mesh || !p || !khat || !pol || !b || nrhs < 1) { set_error("bad argument"); return MBEM_EINVAL; }
    MBEM_TRY(check_frame(p));
    MBEM_TRY(set_device(ctx));
    double *dk = nullptr;
    double2 *dp = nullptr;
    MBEM_TRY(dalloc(&dk, 3 * nrhs));
    MBEM_TRY(dalloc(&dp, 3 * nrhs));
    const hipStream_t s = ctx->stream;
    MBEM_HIP(hipMemcpyAsync(dk, khat, sizeof(double) * 3 * nrhs, hipMemcpyHostToDevice, s));
    MBEM_HIP(hipMemcpyAsync(dp, pol, sizeof(double2) * 3 * nrhs, hipMemcpyHostToDevice, s));
    int st = rhs_run(mesh, p, dk, dp, nrhs, (double2 *)b, s);
    (void)hipStreamSynchronize(s);
    dfree(dk);
    dfree(dp);
    return st;
}

// r_ws, d_ws: optional device vectors of N elements (residual and
// correction); allocated here when null.
static int solve_impl(mbem_ctx *ctx, mbem_op *op, const mbem_c128 *b, int32_t nrhs, const mbem_solve_opts *o,
                      mbem_c128 *x, mbem_stats *stats, bool trans, double2 *r_ws = nullptr,
                      double2 *d_ws = nullptr) {
    if (!op || !b || !x || !o || nrhs < 1 || o->maxit < 1 || !(o->tol > 0)) {
        set_error("bad argument");
        return MBEM_EINVAL;
    }
    MBEM_TRY(set_device(ctx));
    const hipStream_t s = ctx->stream;
    if (trans) MBEM_TRY(mbj_transpose_run(op, s));
    Gmres g;
    g.trans = trans;
    MBEM_TRY(gmres_alloc(g, op, o->maxit, s));
    const int64_t N = g.N;
    double2 *r = r_ws, *d = d_ws;
    Owned own_r, own_d;
    if (!r_ws) { MBEM_TRY(dalloc(&r, N)); own_r.p = r; }
    if (!d_ws) { MBEM_TRY(dalloc(&d, N)); own_d.p = d; }
    Timer t;
    t.start(s);
    int total_it = 0, sweeps = 0, status = MBEM_OK;
    double worst = 0.0;
    // every column must be finite before anything is solved
    std::vector<double> bnorm(nrhs);
    for (int c = 0; c < nrhs; ++c) {
        MBEM_TRY(vec_norm2((const double2 *)b + c * N, N, g.ndev, s));
        MBEM_HIP(hipMemcpyAsync(&bnorm[c], g.ndev, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    MBEM_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < nrhs; ++c)
        if (!std::isfinite(bnorm[c])) {
            set_error("right-hand side column " + std::to_string(c) + " is not finite");
            return MBEM_EINVAL;
        }
    // Residual of the solution of the GMRES run just made on right-hand side
    // rhs with it steps: r = rhs - Z u for its solution u = P^-1 V y, formed
    // as rhs - sum_j y_j (Z z_j) from the steps' products Z z_j (z_j =
    // P^-1 V_j; r may be rhs), which are products with the operator, not
    // the Arnoldi recurrence, in place of one more product.  Returns |r|.
    auto residual = [&](const double2 *rhs, int it, double *rn) -> int {
        MBEM_TRY(vec_resid_products(r, rhs, g.W, N, it, g.hdev, N, s));
        MBEM_TRY(vec_norm2(r, N, g.ndev, s));
        MBEM_HIP(hipMemcpyAsync(rn, g.ndev, sizeof(double), hipMemcpyDeviceToHost, s));
        MBEM_HIP(hipStreamSynchronize(s));
        return MBEM_OK;
    };
    for (int c = 0; c < nrhs; ++c) {
        const double2 *bc = (const double2 *)b + c * N;
        double2 *xc = (double2 *)x + c * N;
        const double bn = bnorm[c];
        double rn = 0;
        int it = 0;
        double est = 0;
        if (op->prec == MBEM_FP64) {
            // GMRES on b; if its Arnoldi estimate met tol but the explicit
            // residual (rounding drift of the long recurrence) did not, one
            // more GMRES from the explicit residual corrects x
            const int maxref = o->max_refine > 0 ? o->max_refine : 3;
            int st = gmres_solve(g, bc, bn, o->tol, xc, &it, &est);
            if (st != MBEM_OK && st != MBEM_ENOCONV) return st;
            total_it += it;
            sweeps += 1;
            MBEM_TRY(residual(bc, it, &rn));
            for (int sw = 1; sw < maxref && st == MBEM_OK && bn > 0 && !(rn <= o->tol * bn) &&
                             std::isfinite(rn); ++sw) {
                st = gmres_solve(g, r, rn, o->tol * bn / rn, d, &it, &est);
                if (st != MBEM_OK && st != MBEM_ENOCONV) return st;
                total_it += it;
                sweeps += 1;
                MBEM_TRY(vec_axpy(xc, d, double2{1.0, 0.0}, N, s));
                MBEM_TRY(residual(r, it, &rn));   // r - Z d
            }
        } else {
            // iterative refinement: x += GMRES(Z, b - Z x), residual in FP64.
            // By default the first sweep aims at tol itself (floored at 1e-8,
            // about where the complex64 products stop reducing the Arnoldi
            // residual): one longer Krylov space costs fewer products than
            // restarting from the refined residual.
            const int maxref = o->max_refine > 0 ? o->max_refine : 8;
            const double itol = o->inner_tol > 0 ? o->inner_tol : std::max(o->tol, 1e-8);
            MBEM_HIP(hipMemsetAsync(xc, 0, sizeof(double2) * N, s));
            MBEM_HIP(hipMemcpyAsync(r, bc, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
            rn = bn;
            for (int sw = 0; sw < maxref && bn > 0 && !(rn <= o->tol * bn) && std::isfinite(rn); ++sw) {
                int st = gmres_solve(g, r, rn, std::max(itol, o->tol * bn / rn), d, &it, &est);
                if (st != MBEM_OK && st != MBEM_ENOCONV) return st;
                total_it += it;
                sweeps += 1;
                MBEM_TRY(vec_axpy(xc, d, double2{1.0, 0.0}, N, s));
                MBEM_TRY(residual(r, it, &rn));   // r - Z d
            }
        }
        // the iterate is accepted only if its explicit residual meets tol
        const double rel = bn > 0 ? rn / bn : 0.0;
        worst = std::max(worst, rel);
        if (!(rel <= o->tol)) status = MBEM_ENOCONV;
    }
    const double ms = t.stop(s);
    if (stats) {
        stats->iters = total_it;
        stats->outer_iters = sweeps;
        stats->rel_resid = worst;
        stats->t_solve_ms = ms;
        stats->t_matvec_ms = g.t_matvec;
        stats->n_matvec = g.n_matvec;
    }
    if (status == MBEM_ENOCONV) set_error("GMRES did not reach the tolerance");
    return status;
}

int mbem_solve(mbem_ctx *ctx, mbem_op *op, const mbem_c128 *b, int32_t nrhs, const mbem_solve_opts *o,
               mbem_c128 *x, mbem_stats *stats) {
    return solve_impl(ctx, op, b, nrhs, o, x, stats, false);
}

int mbem_solve_adjoint(mbem_ctx *ctx, mbem_op *op, const mbem_c128 *g, int32_t nrhs, const mbem_solve_opts *o,
                       mbem_c128 *lambda, mbem_stats *stats) {
    if (op && op->blr) { set_error("the transposed solve needs a dense operator"); return MBEM_EINVAL; }
    return solve_impl(ctx, op, g, nrhs, o, lambda, stats, true);
}

int mbem_fill_deps(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, mbem_op **out, mbem_stats *stats) {
    if (!p) { set_error("null argument"); return MBEM_EINVAL; }
    if (p->quadrature != MBEM_QUAD_DEFAULT) {
        set_error("the eps derivative is built for the default quadrature only");
        return MBEM_EINVAL;
    }
    mbem_params q = *p;
    q.precision = MBEM_FP64;
    mbem_op *op = nullptr;
    MBEM_TRY(op_create(ctx, mesh, &q, &op));
    const int st = op_fill(ctx, op, true, stats);
    if (st != MBEM_OK) { op_free_device(op); delete op; return st; }
    op->ce = {0.5, 0.0};   // d((eps_i + 1) / 2) / deps_i; the mass matrix itself is fixed
    op->cm = {0.0, 0.0};
    *out = op;
    return MBEM_OK;
}

int mbem_farfield_functional(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, const double *rhat,
                             const mbem_c128 *e, mbem_c128 *g) {
    if (!mesh || !p || !rhat || !e || !g) { set_error("null argument"); return MBEM_EINVAL; }
    MBEM_TRY(check_frame(p));
    MBEM_TRY(set_device(ctx));
    int st = ff_functional_run(mesh, p, rhat, (const double2 *)e, (double2 *)g, ctx->stream);
    (void)hipStreamSynchronize(ctx->stream);
    return st;
}

int mbem_grad_sigma_ext(mbem_ctx *ctx, mbem_op *op, const mbem_mesh *mesh, const mbem_params *p,
                        const mbem_c128 *x, const double *khat, const mbem_c128 *pol, const double *disp_dir,
                        const mbem_solve_opts *o, double *out, mbem_c128 *lambda_out, double *dsig_dnode,
                        double *dsig_dx, mbem_stats *stats) {
    if (!op || !mesh || !p || !x || !khat || !pol || !o || !out) { set_error("null argument"); return MBEM_EINVAL; }
    if (op->blr) { set_error("the gradient needs a dense operator"); return MBEM_EINVAL; }
    if (p->quadrature != MBEM_QUAD_DEFAULT || op->p.quadrature != MBEM_QUAD_DEFAULT) {
        set_error("the gradient is built for the default quadrature only");
        return MBEM_EINVAL;
    }
    if (p->frame != op->p.frame) { set_error("the parameters' frame differs from the operator's"); return MBEM_EINVAL; }
    if (mesh != op->mesh) { set_error("the mesh is not the operator's"); return MBEM_EINVAL; }
    if (disp_dir)
        for (int64_t i = 0; i < 3 * mesh->nn; ++i)
            if (!std::isfinite(disp_dir[i])) { set_error("displacement directions are not finite"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    const hipStream_t s = ctx->stream;
    const int64_t N = 2 * op->n2;
    double2 *g = nullptr, *lam = nullptr, *y = nullptr, *dots = nullptr;
    double *ddir = nullptr;
    Owned own_dir;
    if (disp_dir && dsig_dnode) {
        MBEM_TRY(dalloc(&ddir, 3 * mesh->nn));
        own_dir.p = ddir;
        MBEM_HIP(hipMemcpyAsync(ddir, disp_dir, sizeof(double) * 3 * mesh->nn, hipMemcpyHostToDevice, s));
    }
    MBEM_TRY(dalloc(&g, N));
    int st = dalloc(&lam, N);
    if (st == MBEM_OK) st = dalloc(&y, N);
    if (st == MBEM_OK) st = dalloc(&dots, 2);
    mbem_op *dop = nullptr;
    mbem_stats sst{};
    double2 hd[2] = {{0, 0}, {0, 0}};
    if (st == MBEM_OK) {
        const mbem_c128 ec[3] = {{pol[0].re, -pol[0].im}, {pol[1].re, -pol[1].im}, {pol[2].re, -pol[2].im}};
        st = ff_functional_run(mesh, p, khat, (const double2 *)ec, g, s);
    }
    Timer tm;
    double t_adj = 0, t_deps = 0, t_shape = 0;
    tm.start(s);
    if (st == MBEM_OK) st = solve_impl(ctx, op, (const mbem_c128 *)g, 1, o, (mbem_c128 *)lam, &sst, true);
    t_adj = tm.stop(s);
    tm.start(s);
    if (st == MBEM_OK) st = mbem_fill_deps(ctx, mesh, p, &dop, nullptr);
    if (st == MBEM_OK) {
        double2 *tmp = nullptr;
        st = dalloc(&tmp, 4 * op->n2);
        if (st == MBEM_OK) st = matvec_run(dop, (const double2 *)x, y, tmp, s);
        if (st == MBEM_OK) st = dotu_run(g, (const double2 *)x, N, dots, s);
        if (st == MBEM_OK) st = dotu_run(lam, y, N, dots + 1, s);
        if (st == MBEM_OK && hipMemcpyAsync(hd, dots, sizeof(hd), hipMemcpyDeviceToHost, s) != hipSuccess) st = MBEM_EDEVICE;
        (void)hipStreamSynchronize(s);
        dfree(tmp);
    }
    t_deps = tm.stop(s);
    if (st == MBEM_OK && lambda_out)
        if (hipMemcpy(lambda_out, lam, sizeof(double2) * N, hipMemcpyDeviceToDevice) != hipSuccess) st = MBEM_EDEVICE;
    tm.start(s);
    if (st == MBEM_OK && (dsig_dnode || dsig_dx))
        st = shape_grad_run(op, p, (const double2 *)x, lam, khat, (const double2 *)pol, ddir, dsig_dnode, dsig_dx,
                            s);
    t_shape = tm.stop(s);
    sst.t_adjoint_ms = t_adj;
    sst.t_deps_ms = t_deps;
    sst.t_shape_ms = t_shape;
    if (dop) mbem_op_destroy(dop);
    dfree(g); dfree(lam); dfree(y); dfree(dots);
    if (st != MBEM_OK) return st;
    // C = (4 pi / k) Im(g^T x);  dC/deps = (4 pi / k) Im(s'), s' = -lambda^T (dZ/deps) x,
    // holomorphic in eps: d/dRe = Im(s'), d/dIm = Im(i s') = Re(s')
    const double c = 4.0 * 3.14159265358979323846 / p->k0;
    out[0] = c * hd[0].y;
    out[1] = c * (-hd[1].y);
    out[2] = c * (-hd[1].x);
    if (stats) *stats = sst;
    return MBEM_OK;
}

int mbem_solve_block(mbem_ctx *ctx, mbem_op *op, const mbem_c128 *b, int32_t nrhs, const mbem_block_opts *o,
                     mbem_c128 *x, mbem_block_stats *stats) {
    if (!op || !b || !x || !o || nrhs < 1 || o->maxit < 0 || o->max_refine < 0 || !(o->tol > 0)) {
        set_error("bad argument");
        return MBEM_EINVAL;
    }
    if (op->blr) { set_error("the block solve needs a dense operator"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    Timer t;
    t.start(ctx->stream);
    const int st = block_solve_run(op, (const double2 *)b, nrhs, o, (double2 *)x, stats, ctx->stream);
    const double ms = t.stop(ctx->stream);
    if (stats) stats->t_solve_ms = ms;
    return st;
}

int mbem_gemm_autotune(mbem_ctx *ctx, mbem_op *op, int32_t nrhs, int32_t reps, float *ms, int32_t *best) {
    if (!op || nrhs < 1 || !best) { set_error("bad argument"); return MBEM_EINVAL; }
    if (op->blr) { set_error("the block product needs a dense operator"); return MBEM_EINVAL; }
    if (op->near_on) {
        MBEM_TRY(set_device(ctx));
        MBEM_TRY(near_fold_run(op, ctx->stream));
    }
    MBEM_TRY(set_device(ctx));
    const hipStream_t s = ctx->stream;
    MBEM_TRY(ensure_c64_copy(op, s));
    const int64_t n2 = op->n2, N = 2 * n2;
    float2 *X = nullptr, *T = nullptr;
    MBEM_TRY(dalloc(&X, (size_t)nrhs * N));
    int st = dalloc(&T, (size_t)4 * nrhs * n2);
    if (st == MBEM_OK) {
        MBEM_HIP(hipMemsetAsync(X, 0, sizeof(float2) * nrhs * N, s));
        CgemmList L;
        L.np = 3;
        for (int q = 0; q < 3; ++q) {
            CgemmProb &P = L.p[q];
            P.A = op->prec == MBEM_MIXED ? op->K[q] : op->K32[q];
            P.lda = n2; P.M = n2; P.K = n2; P.ldc = n2; P.batch = 1;
        }
        L.p[0].B = X; L.p[0].ldb = n2; L.p[0].Nb = 2 * nrhs; L.p[0].C = T;
        L.p[1].B = X + n2; L.p[1].ldb = N; L.p[1].Nb = nrhs; L.p[1].C = T + 2 * nrhs * n2;
        L.p[2].B = X; L.p[2].ldb = N; L.p[2].Nb = nrhs; L.p[2].C = T + 3 * nrhs * n2;
        int b = 0;
        st = cgemm_f32_autotune(L, s, std::max(1, (int)reps), ms, &b);
        if (st == MBEM_OK) { ctx->tuned_n2 = n2; ctx->tuned_ncol = nrhs; ctx->tuned_cfg = b; *best = b; }
    }
    (void)hipStreamSynchronize(s);
    dfree(X);
    dfree(T);
    return st;
}

int mbem_cgemm(mbem_ctx *ctx, int32_t dtype, int32_t conj_a, int64_t M, int64_t Nb, int64_t K, const void *A,
               int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc, int32_t config) {
    if (dtype < 0 || dtype > 2 || M < 0 || Nb < 0 || K < 0 || (dtype == 0 && conj_a)) {
        set_error("bad argument");
        return MBEM_EINVAL;
    }
    MBEM_TRY(set_device(ctx));
    CgemmList L;
    L.np = 1;
    CgemmProb &P = L.p[0];
    P.A = A; P.B = B; P.C = C; P.lda = lda; P.ldb = ldb; P.ldc = ldc; P.M = M; P.Nb = Nb; P.K = K;
    P.batch = 1;
    if (!cgemm_list_valid(L, dtype == 1 ? 16 : 8, dtype == 0 ? 8 : 16)) {
        set_error("GEMM operands: null pointer, leading dimension or alignment");
        return MBEM_EINVAL;
    }
    if (M == 0 || Nb == 0) return MBEM_OK;
    int st;
    if (dtype == 0) {
        if (config < 0 || config >= kGemmConfigs) { set_error("unknown GEMM configuration"); return MBEM_EINVAL; }
        st = cgemm_f32_run(L, config, ctx->stream);
    } else {
        st = cgemm_f64_run(L, dtype == 2, conj_a != 0, 1, nullptr, ctx->stream);
    }
    if (st == MBEM_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) { set_error("GEMM failed"); st = MBEM_EDEVICE; }
    return st;
}

int mbem_farfield(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, const mbem_c128 *x,
                  int32_t nrhs, const double *rhat, int64_t ndir, mbem_c128 *F) {
    if (!mesh || !p || !x || !rhat || !F || nrhs < 1 || ndir < 1) { set_error("bad argument"); return MBEM_EINVAL; }
    MBEM_TRY(check_frame(p));
    MBEM_TRY(set_device(ctx));
    int st = farfield_run(mesh, p, (const double2 *)x, nrhs, rhat, ndir, (double2 *)F, ctx->stream);
    (void)hipStreamSynchronize(ctx->stream);
    return st;
}

int mbem_spectrum(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, int32_t npts, const double *k0,
                  const mbem_c128 *eps_r, const mbem_c128 *mu_r, const double *khat, const mbem_c128 *pol,
                  int32_t block, const mbem_solve_opts *o, int32_t ntheta, double *sigma, int32_t *iters,
                  mbem_stats *stats) {
    if (!mesh || !p || !k0 || !eps_r || !khat || !pol || !o || !sigma || npts < 1) {
        set_error("bad argument");
        return MBEM_EINVAL;
    }
    if (o->maxit < 1 || !(o->tol > 0)) { set_error("bad solve options"); return MBEM_EINVAL; }
    if (block > kMaxBlock) { set_error("preconditioner block above 512 is not supported"); return MBEM_EINVAL; }
    for (int32_t i = 0; i < npts; ++i)
        if (!(k0[i] > 0)) { set_error("k0 must be positive at every point"); return MBEM_EINVAL; }
    MBEM_TRY(set_device(ctx));
    const hipStream_t s = ctx->stream;
    auto point = [&](int32_t i) {
        mbem_params q = *p;
        q.k0 = k0[i];
        q.eps_r_re = eps_r[i].re;
        q.eps_r_im = eps_r[i].im;
        q.mu_r_re = mu_r ? mu_r[i].re : 1.0;
        q.mu_r_im = mu_r ? mu_r[i].im : 0.0;
        return q;
    };
    mbem_params q = point(0);
    mbem_op *op = nullptr;
    MBEM_TRY(op_create(ctx, mesh, &q, &op));
    struct OpRelease {
        mbem_op *op;
        ~OpRelease() { mbem_op_destroy(op); }
    } release{op};
    // one allocation for b, x, the residual and the correction
    const int64_t N = 2 * op->n2;
    double2 *vec = nullptr;
    MBEM_TRY(dalloc(&vec, 4 * N + 3));
    Owned own_vec;
    own_vec.p = vec;
    double2 *b = vec, *x = vec + N, *r = vec + 2 * N, *d = vec + 3 * N, *dpol = vec + 4 * N;
    double *dk = nullptr;
    MBEM_TRY(dalloc(&dk, 3));
    Owned own_dk;
    own_dk.p = dk;
    MBEM_HIP(hipMemcpyAsync(dk, khat, sizeof(double) * 3, hipMemcpyHostToDevice, s));
    MBEM_HIP(hipMemcpyAsync(dpol, pol, sizeof(double2) * 3, hipMemcpyHostToDevice, s));
    CsWork cw;
    mbem_stats tot{};
    int status = MBEM_OK;
    for (int32_t i = 0; i < npts; ++i) {
        q = point(i);
        op_set_material(op, &q);
        double tf = 0.0;
        MBEM_TRY(fill_enqueue(op, s, false, i == 0));   // the geometry tables once
        MBEM_TRY(fill_collect(op, &tf));
        tot.t_fill_ms += tf;
        if (i == 0) tot.t_geom_ms = op->t_phase[0];
        tot.t_regular_ms += op->t_phase[1];
        tot.t_near_ms += op->t_phase[2];
        tot.t_ssq_ms += op->t_phase[3];
        tot.t_mass_ms += op->t_phase[4];
        tot.n_near_pairs += op->n_near;
        Timer t;
        t.start(s);
        MBEM_TRY(mbj_setup_run(op, block, s, true));
        tot.t_setup_ms += t.stop(s);
        MBEM_TRY(rhs_run(mesh, &q, dk, dpol, 1, b, s));
        mbem_stats ss{};
        const int st = solve_impl(ctx, op, (const mbem_c128 *)b, 1, o, (mbem_c128 *)x, &ss, false, r, d);
        if (st != MBEM_OK && st != MBEM_ENOCONV) return st;
        if (st == MBEM_ENOCONV) status = MBEM_ENOCONV;
        tot.iters += ss.iters;
        tot.outer_iters += ss.outer_iters;
        tot.rel_resid = std::max(tot.rel_resid, ss.rel_resid);
        tot.t_solve_ms += ss.t_solve_ms;
        tot.t_matvec_ms += ss.t_matvec_ms;
        tot.n_matvec += ss.n_matvec;
        if (iters) iters[i] = ss.iters;
        MBEM_TRY(cross_sections_impl(ctx, mesh, &q, x, khat, pol, ntheta, sigma + 3 * (int64_t)i, cw));
    }
    tot.n_regular_pairs = mesh->nt * mesh->nt - mesh->n_spairs;
    if (stats) *stats = tot;
    if (status == MBEM_ENOCONV) set_error("GMRES did not reach the tolerance at some point of the sweep");
    return status;
}

int mbem_cross_sections(mbem_ctx *ctx, const mbem_mesh *mesh, const mbem_params *p, const mbem_c128 *x,
                        const double *khat, const mbem_c128 *pol, int32_t ntheta, double *out) {
    if (!mesh || !p || !x || !khat || !pol || !out) { set_error("null argument"); return MBEM_EINVAL; }
    MBEM_TRY(check_frame(p));
    MBEM_TRY(set_device(ctx));
    CsWork w;
    return cross_sections_impl(ctx, mesh, p, (const double2 *)x, khat, pol, ntheta, out, w);
}

}  // extern "C"
