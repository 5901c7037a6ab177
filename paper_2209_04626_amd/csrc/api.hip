// Host orchestration of svd_plain (Algorithm 2 + Algorithm 1) and svd_mixed
// (Algorithm 4 with the pivots of Algorithm 5), and the C ABI.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../include/mpjsvd.h"
#include "common.hpp"
#include "internal.hpp"

using namespace mpj;

namespace mpj {
static thread_local char g_last_error[256] = "";
void note_hip_error(hipError_t e, const char *where) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
}
void note_error_text(const char *msg) { snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }
} // namespace mpj

extern "C" const char *svd_last_error(void) { return mpj::g_last_error; }

extern "C" void svd_default_opts(svd_opts *o, int mixed) {
    memset(o, 0, sizeof(*o));
    o->tol_alg = 1e-2;
    o->tol_orth = 1e-5;
    o->tol_cond_coef = 1.5;
    o->small_col_rel = ldexp(1.0, -53);
    o->small_col_frac = 0.25;
    o->eps_work = 0.0;
    o->eps_low = 0.0;
    o->maxsweep_low = 30;
    o->maxsweep_work = 30;
    o->want_u = 1;
    o->want_v = 1;
    o->branch = SVD_BRANCH_AUTO;
    o->switch_method = 1;
    o->pivot_precision = mixed ? 32 : 64;
    o->sign_normalize = 1;
    o->block_cols = 0;
    o->inner_sweeps = 0;
    o->kernel_timing = 0;
    o->low_stop_off = 0.0;
    o->block_cols_low = 0;
    o->block_cols_work = 0;
    o->v_method = mixed ? 1 : 0;
    o->diagnostics = 0;
    o->tol_vsolve = 0.0;
    o->inner_pairs = 0;
    o->tol_cluster = 0.0;
    o->y2_safeguard = 1;
    o->tol_y2 = 0.0;
    o->kernel_timing_every = 1;
    o->wait_polls = 0;
    o->fused_rounds = 0;
    o->capture = 0;
    // measured at n = 4096: four BF16-Gram sweeps then FP32 sweeps beat
    // FP32 sweeps alone; more BF16 sweeps do not shorten the FP32 ones
    o->half_sweeps = 4;
    o->half_stop_off = 0.0;
    o->half_storage = 0;
}

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    int m, n, N, b32, b64;
    size_t off_atall, off_tau0, off_t0, off_a1, off_wp, off_nrm2, off_piv, off_a1p, off_tau1,
        off_t1, off_rt, off_tau2, off_t2, off_x, off_y, off_vacc, off_y32, off_xt, off_ulow, off_bm,
        off_tau3, off_t3, off_ux, off_vx, off_sig, off_rank, off_nrmx, off_small, off_qr, off_jac,
        off_v32, off_v2, off_idx, off_y16, off_ydiag, total;
};

// Whether the FP32 stage asks for the fused round (it still falls back to
// the separate kernels where the grid does not fit the device).
bool fused_low(int n, const svd_opts &o) {
    if (o.fused_rounds < 0 || o.switch_method != 1) return false;
    // measured: at n = 2048 the separate 16-column kernels are faster (the
    // fused round's inner solve dominates a round there), at n = 4096 the
    // fused round is
    return o.fused_rounds > 0 || n > 2048;
}

// Jacobi block width per stage: the FP32 stage is bound by the latency of
// the inner 2b x 2b solves (b = 16 keeps them short), the FP64 stage with V by
// the traffic of the block updates (b = 32 halves the rounds per sweep).
int pick_b(int n, const svd_opts &o, bool low) {
    auto ok = [](int b) { return b == 16 || b == 32; };
    const int stage = low ? o.block_cols_low : o.block_cols_work;
    if (ok(stage)) return stage;
    if (ok(o.block_cols)) return o.block_cols;
    // the fused FP32 round works on 32-column blocks
    if (low && fused_low(n, o)) return 32;
    const int t = tuned_block_cols(n, low);
    if (ok(t)) return t;
    if (low) return 16;
    return n >= 512 ? 32 : 16;
}

Layout layout(int m, int n, const svd_opts &o) {
    Layout L;
    L.m = m; L.n = n;
    L.N = ((n + 63) / 64) * 64;
    if (L.N == 0) L.N = 64;
    L.b32 = pick_b(n, o, true);
    L.b64 = pick_b(n, o, false);
    const size_t d = sizeof(double), f = sizeof(float);
    const size_t nn = (size_t)n * n, NN = (size_t)L.N * L.N;
    const size_t nblk = qr_t_doubles(n);
    size_t p = 0;
    auto take = [&](size_t bytes) { size_t o_ = p; p += al256(bytes); return o_; };
    L.off_atall = take(m > n ? (size_t)m * n * d : 0);
    L.off_tau0 = take((size_t)n * d);
    L.off_t0 = take(nblk * d);
    L.off_a1 = take(nn * d);
    L.off_wp = take(nn * d);
    L.off_nrm2 = take(qrcp_scratch_bytes(n, (int)d));
    L.off_piv = take((size_t)n * sizeof(int));
    L.off_a1p = take(nn * d);
    L.off_tau1 = take((size_t)n * d);
    L.off_t1 = take(nblk * d);
    L.off_rt = take(nn * d);
    L.off_tau2 = take((size_t)n * d);
    L.off_t2 = take(nblk * d);
    L.off_x = take(NN * d);
    L.off_y = take(NN * d);
    L.off_vacc = take(NN * d);
    L.off_y32 = take(NN * f);
    L.off_v32 = take(o.switch_method >= 2 ? NN * f : 0);   // V_low for switch methods 2 and 3
    L.off_y16 = take(o.half_sweeps > 0 && o.half_storage ? NN * 2 : 0);   // BF16 Y (half_storage)
    L.off_ydiag = take(o.diagnostics == 2 ? NN * d : 0);     // copy of Y for the switch study
    L.off_xt = take(nn * f);
    L.off_ulow = take(NN * d);
    L.off_bm = take(nn * d);
    L.off_tau3 = take((size_t)n * d);
    L.off_t3 = take(nblk * d);
    L.off_ux = take(nn * d);
    L.off_vx = take(nn * d);
    L.off_sig = take((size_t)n * d);
    L.off_rank = take((size_t)n * sizeof(int));
    L.off_nrmx = take((size_t)n * d);
    L.off_small = take(4096);
    L.off_v2 = take(o.y2_safeguard ? NN * d : 0);           // V columns of Y2
    L.off_idx = take((size_t)n * sizeof(int) + (size_t)n * sizeof(float));
    L.off_qr = take(qr_scratch_doubles(m > n ? m : n, n, nullptr) * d);
    {
        const size_t j32 = jacobi_scratch_bytes(L.N, L.b32, (int)f);
        const size_t j64 = jacobi_scratch_bytes(L.N, L.b64, (int)d);
        L.off_jac = take(j32 > j64 ? j32 : j64);
    }
    L.total = p;
    return L;
}

// layout of the small-scalar block
struct Small {
    int nonfinite, nzero, nsmall, pad0;
    double cond;
    float orth;
    float orthv, orthy;
    int err_wait;        // a bounded cross-workgroup wait ran out
    int nonfinite_out;   // a singular value came out NaN or Inf
    int pad1;
    double condl;        // max|l_ii| / min|l_ii| of X = L (before the solve for V)
    double pivscale;     // power of two for the FP32 copy of A1 (pivots)
    double lowscale;     // power of two for the FP32 copy of X (FP32 stage)
    // stream-ordered mode (svd_opts.capture): decisions taken on the device
    int branch;          // SVD_BRANCH_LOW or SVD_BRANCH_SKIP
    int vtaken;          // v_method 1: 1 solve accepted, 3 rejected
    SweepCtl ctl_low, ctl_work, ctl_half;
};
static_assert(sizeof(Small) <= 4096, "small-scalar block");

inline dim3 grid_n(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

__global__ void k_zero_words(int *p, int n) {
    for (int i = threadIdx.x; i < n; i += 256) p[i] = 0;
}

// Section 3.5's three tests on the device: skip the FP32 stage when
// max|r_ii| / min|r_ii| <= tol_cond, when at least nsmall_min trailing
// columns of X are small, or when max|X_t^T X_t - I| <= tol_orth; a forced
// branch overrides them.  A skip switches the FP32 stage's sweeps off.
__global__ void k_branch_decide(Small *sm, double tol_cond, int nsmall_min, double tol_orth,
                                int forced) {
    if (threadIdx.x != 0) return;
    bool skip = sm->cond <= tol_cond || sm->nsmall >= nsmall_min || (double)sm->orth <= tol_orth;
    if (forced == SVD_BRANCH_LOW) skip = false;
    if (forced == SVD_BRANCH_SKIP) skip = true;
    sm->branch = skip ? SVD_BRANCH_SKIP : SVD_BRANCH_LOW;
    sm->ctl_low.stop = skip ? 1 : 0;
    sm->ctl_half.stop = skip ? 1 : 0;
}

// Skip branch in the stream-ordered mode: the switch ran on the unrotated
// FP32 copy, and its result is replaced by Q = I: Y = X (and V_acc = I
// when V is accumulated).
__global__ void k_select_skip(const Small *sm, int N, const double *X, double *Y, double *Vacc) {
    if (sm->branch != SVD_BRANCH_SKIP) return;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)N * N) return;
    Y[e] = X[e];
    if (Vacc) Vacc[e] = (e % (size_t)N == e / (size_t)N) ? 1.0 : 0.0;
}

// v_method 1's acceptance test on the device (the same rule as on the host).
__global__ void k_vsolve_decide(Small *sm, double tol_v) {
    if (threadIdx.x != 0) return;
    sm->vtaken = ((double)sm->orthv <= tol_v && sm->condl < INFINITY) ? 1 : 3;
}

// svd_info of a stream-ordered call, written by its last kernel.
__global__ void k_write_info(const Small *sm, svd_info *info, int mixed, int want_v, int vsolve,
                             int diagnostics) {
    if (threadIdx.x != 0) return;
    svd_info r;
    memset(&r, 0, sizeof(r));
    if (!sm) {   // n = 0
        r.orth = -1.0;
        r.orth_vx = -1.0;
        r.orth_y = -1.0;
        r.v_method_taken = want_v ? 0 : -1;
        *info = r;
        return;
    }
    const bool low = mixed && sm->branch == SVD_BRANCH_LOW;
    r.branch_taken = mixed ? sm->branch : SVD_BRANCH_SKIP;
    r.sweeps_low = low ? sm->ctl_low.sweeps : 0;
    r.sweeps_work = sm->ctl_work.sweeps;
    r.n_small = mixed ? sm->nsmall : 0;
    r.orth = mixed ? (double)sm->orth : -1.0;
    r.cond_r = mixed ? sm->cond : 0.0;
    for (int i = 0; i < 32; ++i) {
        r.off_low[i] = (low && i < sm->ctl_low.sweeps) ? sm->ctl_low.off[i] : 0.f;
        r.off_work[i] = i < sm->ctl_work.sweeps ? sm->ctl_work.off[i] : 0.f;
    }
    r.v_method_taken = !want_v ? -1 : (vsolve ? sm->vtaken : 0);
    r.orth_vx = vsolve ? (double)sm->orthv : -1.0;
    r.orth_y = diagnostics ? (double)sm->orthy : -1.0;
    r.fused_fallback = (low && (sm->ctl_low.timeout || sm->ctl_half.timeout)) ? 2 : 0;
    r.sweeps_half = low ? sm->ctl_half.sweeps : 0;
    int st = SVD_OK;
    if (!sm->ctl_work.conv) st = SVD_WARN_NOCONV;
    if (sm->nzero) st = SVD_WARN_RANK_DEFICIENT;
    if (vsolve && sm->vtaken == 3) st = SVD_WARN_VSOLVE;
    if (sm->nonfinite_out) st = SVD_ERR_BREAKDOWN;
    if (sm->err_wait || sm->ctl_work.timeout) st = SVD_ERR_WAIT_TIMEOUT;
    if (sm->nonfinite) st = SVD_ERR_NONFINITE;
    r.status = st;
    *info = r;
}

// Per-stage HIP events; a failed event call leaves stage_ms at 0 instead of
// failing the SVD.
struct Timer {
    hipEvent_t ev[9] = {};
    bool ok = false;
    hipStream_t s;
    int last = 0;
    Timer(hipStream_t st, bool on) : s(st) {
        if (!on) return;
        ok = true;
        for (int i = 0; i < 9; ++i)
            if (hipEventCreate(&ev[i]) != hipSuccess) { ev[i] = nullptr; ok = false; }
        if (ok && hipEventRecord(ev[0], s) != hipSuccess) ok = false;
    }
    void mark(int stage) {  // end of stage `stage` (0..7); skipped stages get 0 ms
        if (!ok) return;
        for (int k = last + 1; k <= stage + 1; ++k)
            if (hipEventRecord(ev[k], s) != hipSuccess) { ok = false; return; }
        last = stage + 1;
    }
    void fill(svd_info *info) {
        if (!ok) return;
        mark(7);
        if (!ok || hipEventSynchronize(ev[8]) != hipSuccess) return;
        for (int i = 0; i < 8; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) ms = 0.f;
            if (info) info->stage_ms[i] = ms;
        }
    }
    ~Timer() {
        for (int i = 0; i < 9; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
};

int read_back(hipStream_t s, void *host, const void *dev, size_t bytes) {
    hipError_t e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        note_hip_error(e, "read_back");
        return -1;
    }
    return 0;
}

int run_svd(bool mixed, int m, int n, const double *A, int lda, double *S, double *U, int ldu,
            double *V, int ldv, void *work, size_t work_bytes, const svd_opts *op, svd_info *info,
            void *stream) {
    svd_opts o;
    if (op) o = *op; else svd_default_opts(&o, mixed ? 1 : 0);
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (n > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (n > 0 && !S) return -5;
    if (o.want_u && n > 0 && !U) return -6;
    if (o.want_u && ldu < (m > 1 ? m : 1)) return -7;
    if (o.want_v && n > 0 && !V) return -8;
    if (o.want_v && ldv < (n > 1 ? n : 1)) return -9;
    if (n > 8192) return -2;
    if (o.pivot_precision != 32 && o.pivot_precision != 64) return -12;
    if (o.v_method != 0 && o.v_method != 1) return -12;
    if (o.switch_method < 1 || o.switch_method > 3) return -12;
    if (o.inner_pairs != 0 && o.inner_pairs != 1) return -12;
    if (o.y2_safeguard != 0 && o.y2_safeguard != 1) return -12;
    if (o.kernel_timing_every < 0) return -12;
    if (o.wait_polls < -1) return -12;
    if (o.fused_rounds < -1 || o.fused_rounds > 1) return -12;
    if (o.capture != 0 && o.capture != 1) return -12;
    if (o.half_sweeps < 0 || o.half_stop_off < 0.0) return -12;
    if (o.half_storage != 0 && o.half_storage != 1) return -12;
    if (o.diagnostics < 0 || o.diagnostics > 2) return -12;
    const bool cap = o.capture != 0;
    // the stream-ordered mode has no host-side clock, and Algorithm 3's
    // route (no triangular factor for V) needs the branch known on the host
    if (cap && o.kernel_timing != 0) return -12;
    if (cap && mixed && o.switch_method == 3 && o.branch != SVD_BRANCH_LOW) return -12;
    if (cap) {
        // info is device memory, written by the call's last kernel
        if (n == 0 && info)
            hipLaunchKernelGGL(k_write_info, dim3(1), dim3(64), 0, (hipStream_t)stream,
                               (const Small *)nullptr, info, mixed ? 1 : 0, o.want_v, 0, 0);
        if (n == 0) return hipGetLastError() == hipSuccess ? 0 : SVD_ERR_HIP;
    } else if (info) {
        memset(info, 0, sizeof(*info));
        info->orth = -1.0;
        info->orth_vx = -1.0;
        info->orth_y = -1.0;
        info->v_method_taken = o.want_v ? 0 : -1;
    }
    if (n == 0) return 0;
    mpj::g_last_error[0] = 0;
    (void)hipGetLastError();  // drop a stale error left by an earlier, unrelated call
    const Layout L = layout(m, n, o);
    if (!work) return -10;
    if (work_bytes < L.total) return -11;

    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)work;
    auto D = [&](size_t off) { return (double *)(w + off); };
    double *Atall = D(L.off_atall), *tau0 = D(L.off_tau0), *T0 = D(L.off_t0);
    double *A1 = D(L.off_a1), *A1P = D(L.off_a1p), *tau1 = D(L.off_tau1), *T1 = D(L.off_t1);
    double *Rt = D(L.off_rt), *tau2 = D(L.off_tau2), *T2 = D(L.off_t2);
    double *X = D(L.off_x), *Y = D(L.off_y), *Vacc = D(L.off_vacc);
    float *Y32 = (float *)(w + L.off_y32), *Xt = (float *)(w + L.off_xt);
    double *Ulow = D(L.off_ulow), *Bm = D(L.off_bm), *tau3 = D(L.off_tau3), *T3 = D(L.off_t3);
    double *UX = D(L.off_ux), *VX = D(L.off_vx), *sig = D(L.off_sig), *nrmX = D(L.off_nrmx);
    int *piv = (int *)(w + L.off_piv), *rank = (int *)(w + L.off_rank);
    Small *sm = (Small *)(w + L.off_small);
    const int N = L.N;
    const int inner = o.inner_sweeps > 0 ? o.inner_sweeps : 1;

    QRScratch q;
    qr_scratch_carve(q, D(L.off_qr), m > n ? m : n, n);
    q.err = &sm->err_wait;
    q.spin = o.wait_polls;
    JacobiWork jw;
    int hflag[3] = {0, 0, 0};
    jw.hflag = hflag;
    jw.n_real = n;
    jw.cross_pairs = o.inner_pairs == 0 ? 1 : 0;
    KernelClock kclock;
    kclock.on = o.kernel_timing != 0;
    if (o.kernel_timing >= 100) kclock.only = o.kernel_timing - 100;
    if (o.kernel_timing_every > 1) kclock.every = o.kernel_timing_every;
    jw.kc = o.kernel_timing >= 2 ? &kclock : nullptr;
    q.kc = jw.kc;
    float off_low[32] = {0}, off_work[32] = {0};

    Timer tm(s, !cap);
    Small hs;
    memset(&hs, 0, sizeof(hs));
    // (a kernel, not a memset: the call may be captured in a graph)
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, (int *)sm, (int)(sizeof(Small) / 4));
    if (cap) jw.off_hist = nullptr;

    // a0: ingest (A is const) and non-finite scan; non-finite entries are
    // copied as 0 so that the stream-ordered mode runs on finite data (its
    // status then reports SVD_ERR_NONFINITE)
    double *Ain = (m > n) ? Atall : A1;
    const int ldin = (m > n) ? m : n;
    copy_scan(s, m, n, A, lda, Ain, ldin, &sm->nonfinite);
    MPJ_CHECK(hipGetLastError());
    if (!cap && read_back(s, &hs, sm, sizeof(Small))) return SVD_ERR_HIP;
    if (hs.nonfinite) {
        if (info) info->status = SVD_ERR_NONFINITE;
        return 0;
    }
    // a1: tall reduction A = Q0 R1
    if (m > n) {
        qr_factor(s, m, n, Atall, m, tau0, T0, q);
        copy_upper(s, n, Atall, m, A1, n);
    }
    tm.mark(0);
    // a2: pivots (Algorithm 5 in FP32, or FP64)
    // kernel_timing 1: the pass is one interval of n back-to-back step launches
    if (o.kernel_timing == 1)
        kclock.begin(s, SVD_K_QRCP, 0.0);
    int piv_launches;
    if (o.pivot_precision == 32) {
        // the FP32 copy of A1 is scaled by a power of two so that squared
        // column norms of graded inputs stay inside the FP32 range
        col_norms(s, n, n, A1, n, nrmX);
        pow2_scale(s, n, nrmX, &sm->pivscale);
        piv_launches = qrcp_pivots<float>(s, n, A1, n, (float *)D(L.off_wp), w + L.off_nrm2, piv,
                                          jw.kc, &sm->pivscale, o.wait_polls,
                                          cap ? &sm->err_wait : nullptr);
    } else {
        piv_launches = qrcp_pivots<double>(s, n, A1, n, D(L.off_wp), w + L.off_nrm2, piv, jw.kc,
                                           nullptr, o.wait_polls);
    }
    if (o.kernel_timing == 1) {
        kclock.end(s);
        // launches and algorithmic work of the whole pass (see qrcp_pivots)
        const int es = o.pivot_precision == 32 ? 4 : 8;
        kclock.bytes[0] = qrcp_pass_bytes(n, es);
        kclock.flops[0] = qrcp_pass_flops(n);
        kclock.pass_calls = piv_launches;
    }
    tm.mark(1);
    // a3: FP64 QR of A1 P
    gather_cols(s, n, n, A1, n, piv, A1P, n);
    qr_factor(s, n, n, A1P, n, tau1, T1, q);
    tm.mark(2);
    // a4: R = L Q2 via the QR of R^T; X = L (zero padded to N x N)
    transpose_upper_to_lower(s, n, A1P, n, Rt, n, n);
    qr_factor(s, n, n, Rt, n, tau2, T2, q);
    transpose_upper_to_lower(s, n, Rt, n, X, N, N);
    tm.mark(3);
    MPJ_CHECK(hipGetLastError());

    // a5: special cases of Section 3.5
    int branch = SVD_BRANCH_SKIP;
    double cond = 0.0, orth = -1.0;
    int nsmall = 0;
    if (mixed) {
        diag_cond(s, n, A1P, n, &sm->cond);
        col_norms(s, n, n, X, N, nrmX);
        count_small(s, n, nrmX, o.small_col_rel, &sm->nsmall);
        pow2_scale(s, n, nrmX, &sm->lowscale);
        if (cap) {
            // every test measured, the branch taken on the device
            make_xt32(s, n, X, N, Xt, n);
            gemm_orth_maxdev(s, n, Xt, n, &sm->orth);
            hipLaunchKernelGGL(k_branch_decide, dim3(1), dim3(64), 0, s, sm,
                               o.tol_cond_coef * pow((double)n, 0.25),
                               (int)ceil(o.small_col_frac * n), o.tol_orth, o.branch);
            MPJ_CHECK(hipGetLastError());
            // the host enqueues the FP32 stage and the switch; with a skip
            // the stage's sweeps exit at once and k_select_skip sets Y = X
            branch = SVD_BRANCH_LOW;
        }
    }
    if (mixed && !cap) {
        if (read_back(s, &hs, sm, sizeof(Small))) return SVD_ERR_HIP;
        cond = hs.cond;
        nsmall = hs.nsmall;
        const bool small_cond = cond <= o.tol_cond_coef * pow((double)n, 0.25);
        const bool many_small = nsmall >= (int)ceil(o.small_col_frac * n);
        bool skip = small_cond || many_small;
        if (!skip || o.branch != SVD_BRANCH_AUTO) {
            make_xt32(s, n, X, N, Xt, n);
            gemm_orth_maxdev(s, n, Xt, n, &sm->orth);
            if (read_back(s, &hs, sm, sizeof(Small))) return SVD_ERR_HIP;
            orth = hs.orth;
            if (orth <= o.tol_orth) skip = true;
        }
        if (o.branch == SVD_BRANCH_LOW) skip = false;
        if (o.branch == SVD_BRANCH_SKIP) skip = true;
        branch = skip ? SVD_BRANCH_SKIP : SVD_BRANCH_LOW;
    }
    tm.mark(4);

    const double eps_low = o.eps_low > 0 ? o.eps_low : sqrt((double)n) * ldexp(1.0, -24);
    const double eps_work = o.eps_work > 0 ? o.eps_work : sqrt((double)n) * ldexp(1.0, -53);
    int sweeps_low = 0, conv_low = 1, fused_fallback = 0, sweeps_half = 0;
    if (branch == SVD_BRANCH_LOW) {
        // a6: FP32 one-sided Jacobi on low(X) (Section 3.2); V_low is only
        // accumulated for switch methods 2 and 3
        const bool vlow = o.switch_method >= 2;
        float *V32 = vlow ? (float *)(w + L.off_v32) : nullptr;
        // low(X) times a power of two (exact): squared norms and dot
        // products of graded columns stay inside the FP32 range, and every
        // quantity the stage hands on (angles, normalised columns) is
        // invariant under the scale
        // three-precision variant (fused round only): the first sweeps form
        // their Gram blocks on the BF16 matrix cores from Y rounded to BF16
        // (half_storage 0: Y itself stays FP32), or keep Y in BF16 as well
        // (half_storage 1: Y widened to FP32 afterwards); then FP32 sweeps
        const int hmode = o.half_sweeps > 0 ? (o.half_storage ? 2 : 1) : 0;
        const bool use_half = hmode > 0 && !vlow && fused_low(n, o) && L.b32 == 32 &&
                              jacobi_fused_ok(N, hmode);
        unsigned short *Y16 = (unsigned short *)(w + L.off_y16);
        if (hmode == 2 && use_half)
            convert_f64_bf16(s, N, N, X, N, Y16, N, &sm->lowscale);
        else
            convert_f64_f32(s, N, N, X, N, Y32, N, &sm->lowscale);
        if (use_half) {
            jacobi_carve(jw, w + L.off_jac, N, L.b32, (int)sizeof(float));
            jw.half = hmode;
            jw.fused = 1;
            jw.spin = o.wait_polls;
            jw.off_hist = nullptr;
            jw.ctl = cap ? &sm->ctl_half : nullptr;
            jw.stop_off = o.half_stop_off > 0 ? o.half_stop_off : ldexp(1.0, -6);
            int conv_half = 0;
            // rotate where the cosine of the columns exceeds the BF16 unit
            sweeps_half = jacobi_sweeps<float>(s, N, L.b32, hmode == 2 ? (float *)Y16 : Y32, nullptr,
                                               ldexp(1.0, -8), o.half_sweeps, inner, jw, &conv_half);
            jw.half = 0;
            jw.ctl = nullptr;
            if (sweeps_half == -2) {
                // a wait ran out: the stage starts from low(X) in FP32 instead
                (void)hipGetLastError();
                mpj::g_last_error[0] = 0;
                fused_fallback = 1;
                sweeps_half = 0;
                convert_f64_f32(s, N, N, X, N, Y32, N, &sm->lowscale);
            } else if (sweeps_half < 0) {
                return SVD_ERR_HIP;
            } else if (hmode == 2) {
                widen_bf16_f32(s, N, N, Y16, N, Y32, N);
            }
        }
        if (vlow) {
            set_identity(s, N, Ulow, N);
            convert_f64_f32(s, N, N, Ulow, N, V32, N);
        }
        jacobi_carve(jw, w + L.off_jac, N, L.b32, (int)sizeof(float));
        jw.off_hist = cap ? nullptr : off_low;
        jw.ctl = cap ? &sm->ctl_low : nullptr;
        jw.stop_off = o.low_stop_off > 0 ? o.low_stop_off
                                         : (o.low_stop_off == 0 ? sqrt((double)n) * eps_low : 0.0);
        jw.fused = fused_low(n, o) ? 1 : 0;
        jw.spin = o.wait_polls;
        sweeps_low = jacobi_sweeps<float>(s, N, L.b32, Y32, V32, eps_low, o.maxsweep_low, inner,
                                          jw, &conv_low);
        if (sweeps_low == -2) {
            // a fused round gave up waiting (another stream held compute
            // units): the stage starts again from low(X) with separate kernels
            (void)hipGetLastError();
            mpj::g_last_error[0] = 0;
            fused_fallback = 1;
            convert_f64_f32(s, N, N, X, N, Y32, N, &sm->lowscale);
            jw.fused = 0;
            for (int i = 0; i < 32; ++i) off_low[i] = 0.f;
            sweeps_low = jacobi_sweeps<float>(s, N, L.b32, Y32, V32, eps_low, o.maxsweep_low, inner,
                                              jw, &conv_low);
        }
        jw.fused = 0;
        jw.stop_off = 0.0;
        jw.ctl = nullptr;
        if (sweeps_low < 0) return SVD_ERR_HIP;
        tm.mark(5);
        // a7: switch (Section 3.3).  Method 1 (Algorithm 4): B = X^T U_low;
        // method 2: B = fp64(V_low); then B = Q R2, Y = X Q.  Method 3
        // (Algorithm 3): B = V_s = P Q2^T fp64(V_low), the right vectors of
        // A itself, and Y = A1 Q with no preconditioning of the FP64 stage.
        if (o.switch_method == 3) {
            convert_f32_f64(s, n, n, V32, N, UX, n);
            qr_apply_left(s, false, n, n, Rt, n, T2, n, UX, n, q);
            permute_rows_v(s, n, UX, n, piv, Bm, n);
        } else if (vlow) {
            convert_f32_f64(s, n, n, V32, N, Bm, n);
        } else {
            normalize_f32_to_f64(s, N, N, Y32, N, Ulow, N);
            gemm<double>(s, true, false, n, n, n, 1.0, X, N, Ulow, N, 0.0, Bm, n, q.split,
                         q.split_elems, jw.kc);
        }
        qr_factor(s, n, n, Bm, n, tau3, T3, q);
        const bool q_implicit = (!o.want_v || o.v_method == 1) && o.switch_method != 3;
        if (q_implicit) {
            // V is formed after the sweeps (Section 3.4) or not at all, so Q
            // itself is not needed: Y = X Q = (Q^T X^T)^T, the reflectors
            // applied to X^T (U_low's buffer is free once B is formed)
            transpose64(s, n, n, X, N, Ulow, N);
            qr_apply_left(s, true, n, n, Bm, n, T3, n, Ulow, N, q);
            zero_pad_fill(s, N, N, Y, N);
            transpose64(s, n, n, Ulow, N, Y, N);
        } else {
            set_identity(s, N, Vacc, N);
            qr_apply_left(s, false, n, n, Bm, n, T3, n, Vacc, N, q);
            zero_pad_fill(s, N, N, Y, N);
            gemm<double>(s, false, false, n, n, n, 1.0, o.switch_method == 3 ? A1 : X,
                         o.switch_method == 3 ? n : N, Vacc, N, 0.0, Y, N, q.split, q.split_elems,
                         jw.kc);
        }
        if (cap) {
            hipLaunchKernelGGL(k_select_skip, grid_n((size_t)N * N), dim3(256), 0, s,
                               (const Small *)sm, N, (const double *)X, Y,
                               q_implicit ? (double *)nullptr : Vacc);
        }
        tm.mark(6);
    } else {
        MPJ_CHECK(hipMemcpyAsync(Y, X, (size_t)N * N * sizeof(double), hipMemcpyDeviceToDevice, s));
        set_identity(s, N, Vacc, N);
        tm.mark(6);
    }
    MPJ_CHECK(hipGetLastError());
    // Algorithm 3's Y = A1 Q has no triangular factor to solve with: V is
    // accumulated there
    const bool alg3 = branch == SVD_BRANCH_LOW && o.switch_method == 3;
    const bool vsolve = o.want_v && o.v_method == 1 && !alg3;
    double orth_y = -1.0;
    int n_y2 = 0, sweeps_y2 = 0;
    // (the safeguard picks Y2 on the host: not in the stream-ordered mode)
    const bool y2check = o.y2_safeguard && branch == SVD_BRANCH_LOW && n >= 2 && !cap;
    if (o.diagnostics == 2)
        MPJ_CHECK(hipMemcpyAsync(w + L.off_ydiag, Y, (size_t)N * N * sizeof(double),
                                 hipMemcpyDeviceToDevice, s));
    if (o.diagnostics && !y2check) {
        // how far the columns of Y are from orthogonal when the FP64 sweeps start
        normalize_cols64(s, n, n, Y, N, Ulow, N);
        gemm_orth_maxdev64(s, n, Ulow, N, &sm->orthy);
        if (!cap) {
            if (read_back(s, &hs, sm, sizeof(Small))) return SVD_ERR_HIP;
            orth_y = hs.orthy;
        }
    }
    if (y2check) {
        // Section 3.4's safeguard: C = D^-1 Y^T Y D^-1; the columns whose
        // off-diagonal max|c_ij| is well above the FP32 level form Y2, and
        // FP64 sweeps run on Y2 alone before the sweeps over all of Y
        int *idx = (int *)(w + L.off_idx);
        float *dev = (float *)(idx + n);
        normalize_cols64(s, n, n, Y, N, Ulow, N);
        gram_colmax_offdiag64(s, n, Ulow, N, dev);
        std::vector<float> hdev(n);
        if (read_back(s, hdev.data(), dev, (size_t)n * sizeof(float))) return SVD_ERR_HIP;
        float dmax = 0.f;
        for (int j = 0; j < n; ++j) dmax = fmaxf(dmax, hdev[j]);
        if (o.diagnostics) orth_y = dmax;
        const double tol2 = o.tol_y2 > 0 ? o.tol_y2 : 64.0 * sqrt((double)n) * ldexp(1.0, -24);
        std::vector<int> y2;
        for (int j = 0; j < n; ++j)
            if ((double)hdev[j] > tol2) y2.push_back(j);
        const int k = (int)y2.size();
        if (k >= 2) {
            const int K = cdiv(k, 2 * L.b64) * 2 * L.b64;   // Y2's columns, zero padded
            double *Y2 = Ulow, *V2 = (o.want_v && !vsolve) ? D(L.off_v2) : nullptr;
            MPJ_CHECK(hipMemcpyAsync(idx, y2.data(), (size_t)k * sizeof(int), hipMemcpyHostToDevice, s));
            zero_pad_fill(s, N, K, Y2, N);
            gather_cols(s, N, k, Y, N, idx, Y2, N);
            if (V2) {
                zero_pad_fill(s, N, K, V2, N);
                gather_cols(s, N, k, Vacc, N, idx, V2, N);
            }
            jacobi_carve(jw, w + L.off_jac, N, L.b64, (int)sizeof(double));
            jw.off_hist = nullptr;
            jw.n_real = k;
            int conv_y2 = 0;
            sweeps_y2 = jacobi_sweeps_cols<double>(s, N, K, L.b64, Y2, V2, eps_work, o.maxsweep_work,
                                                   inner, jw, &conv_y2);
            jw.n_real = n;
            if (sweeps_y2 < 0) return SVD_ERR_HIP;
            scatter_cols(s, N, k, Y2, N, idx, Y, N);
            if (V2) scatter_cols(s, N, k, V2, N, idx, Vacc, N);
            MPJ_CHECK(hipGetLastError());
            n_y2 = k;
        }
    }

    // a8: FP64 one-sided Jacobi (Algorithm 1); V_X accumulated from Q
    // (v_method 0) or formed afterwards (v_method 1, Section 3.4)

    int conv_work = 0;
    jacobi_carve(jw, w + L.off_jac, N, L.b64, (int)sizeof(double));
    jw.off_hist = cap ? nullptr : off_work;
    jw.ctl = cap ? &sm->ctl_work : nullptr;
    const int sweeps_work = jacobi_sweeps<double>(s, N, L.b64, Y, (o.want_v && !vsolve) ? Vacc : nullptr,
                                                  eps_work, o.maxsweep_work, inner, jw, &conv_work);
    if (sweeps_work < 0) return SVD_ERR_HIP;
    int v_taken = o.want_v ? 0 : -1, sweeps_vfix = 0;
    double orth_vx = -1.0;
    if (vsolve) {
        // Y = X V_X = U_X Sigma, so V_X = X^{-1} Y with X = L lower triangular
        MPJ_CHECK(hipMemcpyAsync(Vacc, Y, (size_t)N * N * sizeof(double), hipMemcpyDeviceToDevice, s));
        diag_cond(s, n, X, N, &sm->condl);
        trsm_lower(s, n, n, X, N, Vacc, N, jw.kc);
        gemm_orth_maxdev64(s, n, Vacc, N, &sm->orthv);
        const double tol_v = o.tol_vsolve > 0 ? o.tol_vsolve : n * ldexp(1.0, -50);
        if (cap) {
            // accepted or not, V_X stays the solve's (the fallback below
            // needs the host); a rejection is reported in the status
            hipLaunchKernelGGL(k_vsolve_decide, dim3(1), dim3(64), 0, s, sm, tol_v);
        } else if (read_back(s, &hs, sm, sizeof(Small))) {
            return SVD_ERR_HIP;
        }
        orth_vx = hs.orthv;
        // default: n 2^-50 = 8 n u, the size of the rounding error that the
        // accumulated rotations of a few sweeps leave in V_X.  A zero on the
        // diagonal of L (rank-deficient X) makes the solve meaningless, and a
        // NaN from it reads as an infinite deviation: both take the other
        // route of Section 3.4.
        if (cap) {
            v_taken = 1;
        } else if (orth_vx <= tol_v && hs.condl < INFINITY) {
            v_taken = 1;
        } else {
            // not accurate enough: V_X from the QR of X^T U_X (U_X = the
            // normalised columns of Y), then sweeps with accumulation on X Q
            normalize_cols64(s, n, n, Y, N, Ulow, N);
            gemm<double>(s, true, false, n, n, n, 1.0, X, N, Ulow, N, 0.0, Bm, n, q.split,
                         q.split_elems, jw.kc);
            qr_factor(s, n, n, Bm, n, tau3, T3, q);
            set_identity(s, N, Vacc, N);
            qr_apply_left(s, false, n, n, Bm, n, T3, n, Vacc, N, q);
            zero_pad_fill(s, N, N, Y, N);
            gemm<double>(s, false, false, n, n, n, 1.0, X, N, Vacc, N, 0.0, Y, N, q.split,
                         q.split_elems, jw.kc);
            int conv_fix = 0;
            jw.off_hist = nullptr;
            sweeps_vfix = jacobi_sweeps<double>(s, N, L.b64, Y, Vacc, eps_work, o.maxsweep_work,
                                                inner, jw, &conv_fix);
            if (sweeps_vfix < 0) return SVD_ERR_HIP;
            conv_work = conv_work && conv_fix;
            v_taken = 2;
        }
    }

    // a9: sigma, U_X, V_X sorted; U = Q0 Q1 U_X, V = P Q2^T V_X
    finalize_sort(s, n, N, Y, Vacc, sig, rank, UX, VX, S, &sm->nzero, &sm->nonfinite_out,
                  o.want_v != 0);
    if (o.want_u) {
        if (!alg3) qr_apply_left(s, false, n, n, A1P, n, T1, n, UX, n, q);
        place_u(s, m, n, UX, n, U, ldu);
        if (m > n) qr_apply_left(s, false, m, n, Atall, m, T0, n, U, ldu, q);
    }
    if (o.want_v) {
        if (!alg3) {
            qr_apply_left(s, false, n, n, Rt, n, T2, n, VX, n, q);
            permute_rows_v(s, n, VX, n, piv, V, ldv);
        } else {
            MPJ_CHECK(hipMemcpy2DAsync(V, (size_t)ldv * sizeof(double), VX, (size_t)n * sizeof(double),
                                       (size_t)n * sizeof(double), n, hipMemcpyDeviceToDevice, s));
        }
        if (o.sign_normalize) sign_normalize(s, m, n, U, ldu, o.want_u != 0, V, ldv);
    }
    MPJ_CHECK(hipGetLastError());
    if (cap) {
        if (info)
            hipLaunchKernelGGL(k_write_info, dim3(1), dim3(64), 0, s, (const Small *)sm, info,
                               mixed ? 1 : 0, o.want_v, vsolve ? 1 : 0, o.diagnostics);
        MPJ_CHECK(hipGetLastError());
        return 0;
    }
    tm.mark(7);
    if (read_back(s, &hs, sm, sizeof(Small))) return SVD_ERR_HIP;
    kclock.collect();
    if (info) {
        for (int c = 0; c < SVD_K_NCLASS; ++c) {
            info->kern_ms[c] = kclock.ms[c];
            info->kern_calls[c] = kclock.calls[c];
            info->kern_bytes[c] = kclock.tot_bytes[c];
            info->kern_flops[c] = kclock.tot_flops[c];
        }
        if (o.kernel_timing == 1) info->kern_calls[SVD_K_QRCP] = kclock.pass_calls;
        for (int i = 0; i < 32; ++i) { info->off_low[i] = off_low[i]; info->off_work[i] = off_work[i]; }
        tm.fill(info);
        info->branch_taken = branch;
        info->sweeps_low = sweeps_low;
        info->sweeps_work = sweeps_work;
        info->n_small = nsmall;
        info->orth = orth;
        info->cond_r = mixed ? cond : 0.0;
        info->v_method_taken = v_taken;
        info->sweeps_vfix = sweeps_vfix;
        info->orth_vx = orth_vx;
        info->orth_y = orth_y;
        info->n_y2 = n_y2;
        info->sweeps_y2 = sweeps_y2;
        info->fused_fallback = fused_fallback;
        info->sweeps_half = sweeps_half;
        int st = SVD_OK;
        if (!conv_work) st = SVD_WARN_NOCONV;
        if (hs.nzero) st = SVD_WARN_RANK_DEFICIENT;
        if (hs.nonfinite_out) st = SVD_ERR_BREAKDOWN;
        if (hs.err_wait) st = SVD_ERR_WAIT_TIMEOUT;
        info->status = st;
    }
    return 0;
}

} // namespace

extern "C" size_t svd_diag_y_offset(int m, int n, const svd_opts *op) {
    if (!op || op->diagnostics != 2 || m < 0 || n <= 0 || n > m) return 0;
    return layout(m, n, *op).off_ydiag;
}

extern "C" size_t svd_workspace_size(int m, int n, const svd_opts *op) {
    if (m < 0 || n < 0 || n > m) return 0;
    svd_opts o;
    if (op) o = *op; else svd_default_opts(&o, 1);
    if (n == 0) return 256;
    return layout(m, n, o).total;
}

extern "C" int svd_plain(int m, int n, const double *A, int lda, double *S, double *U, int ldu,
                         double *V, int ldv, void *work, size_t work_bytes, const svd_opts *o,
                         svd_info *info, void *stream) {
    return run_svd(false, m, n, A, lda, S, U, ldu, V, ldv, work, work_bytes, o, info, stream);
}

extern "C" int svd_mixed(int m, int n, const double *A, int lda, double *S, double *U, int ldu,
                         double *V, int ldv, void *work, size_t work_bytes, const svd_opts *o,
                         svd_info *info, void *stream) {
    return run_svd(true, m, n, A, lda, S, U, ldu, V, ldv, work, work_bytes, o, info, stream);
}

extern "C" const char *svd_status_string(int code) {
    switch (code) {
    case SVD_OK: return "ok";
    case SVD_WARN_NOCONV: return "warning: a Jacobi phase reached its sweep cap";
    case SVD_ERR_NONFINITE: return "error: input holds NaN or Inf";
    case SVD_WARN_RANK_DEFICIENT: return "warning: zero singular value(s)";
    case EIG_ERR_CLUSTER: return "error: a block of equal |eigenvalue| larger than 64";
    case SVD_ERR_WAIT_TIMEOUT: return "error: a bounded cross-workgroup wait ran out; outputs undefined";
    case SVD_ERR_BREAKDOWN: return "error: a non-finite singular value from finite input; outputs undefined";
    case SVD_ERR_HIP: return "error: HIP runtime failure";
    case SVD_ERR_SCRATCH_LIMIT: return "error: the problem needs more scratch than the fixed array holds";
    default: return code < 0 ? "error: invalid argument" : "unknown status";
    }
}
