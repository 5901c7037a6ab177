// Host-side declarations shared by the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <vector>

namespace mpj {

// Per-launch HIP event timing for a kernel class (opt-in).  Pairs of events
// are taken from a pool, recorded around each launch and read after the
// caller synchronises.
struct KernelClock {
    static constexpr int NC = 12;
    std::vector<hipEvent_t> ev;
    std::vector<int> cls;
    std::vector<double> bytes, flops;
    size_t used = 0;
    bool on = false;
    int only = -1;          // >= 0: bracket only the launches of this class
    int every = 1;          // clock every `every`-th launch of a class (slot())
    int seen[NC] = {0};
    bool skipping = false;
    float ms[NC] = {0};
    int calls[NC] = {0};
    int pass_calls = 0;
    double tot_bytes[NC] = {0};
    double tot_flops[NC] = {0};
    // The clock is optional: an event call that fails switches it off
    // (the timings are then absent) instead of failing the computation.
    bool grow(int c, double b, double f) {
        if (used + 2 <= ev.size()) return true;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess) { on = false; return false; }
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            on = false;
            return false;
        }
        ev.push_back(e0);
        ev.push_back(e1);
        cls.push_back(c);
        bytes.push_back(b);
        flops.push_back(f);
        return true;
    }
    void begin(hipStream_t s, int c, double b, double f = 0.0) {
        if (!on) return;
        skipping = (only >= 0 && c != only) || (seen[c]++ % every != 0);
        if (skipping) return;
        if (!grow(c, b, f)) return;
        cls[used / 2] = c;
        bytes[used / 2] = b;
        flops[used / 2] = f;
        if (hipEventRecord(ev[used], s) != hipSuccess) on = false;
    }
    // The events of one launch of class c that the dispatch itself records
    // (hipExtLaunchKernelGGL): no marker packets around the kernel, so short
    // launches are timed as the trace sees them.  False when c is not
    // clocked.
    bool slot(int c, double b, double f, hipEvent_t *e0, hipEvent_t *e1) {
        if (!on || (only >= 0 && c != only)) return false;
        if (seen[c]++ % every != 0) return false;
        if (!grow(c, b, f)) return false;
        cls[used / 2] = c;
        bytes[used / 2] = b;
        flops[used / 2] = f;
        *e0 = ev[used];
        *e1 = ev[used + 1];
        used += 2;
        return true;
    }
    void end(hipStream_t s) {
        if (!on || skipping) return;
        if (hipEventRecord(ev[used + 1], s) != hipSuccess) { on = false; return; }
        used += 2;
    }
    // call after the stream has been synchronised
    void collect() {
        if (!on) return;
        for (size_t i = 0; i < used; i += 2) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) continue;
            ms[cls[i / 2]] += t;
            calls[cls[i / 2]] += 1;
            tot_bytes[cls[i / 2]] += bytes[i / 2];
            tot_flops[cls[i / 2]] += flops[i / 2];
        }
        used = 0;
    }
    ~KernelClock() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

// ---------------------------------------------------------------- tuning
// Entries of the loaded tuning table for size n (0 = none).
int tuned_block_cols(int n, bool low);
int tuned_wg_per_cu(int nmax);

// ---------------------------------------------------------------- GEMM
// C (M x N, column-major, ldc) = alpha op(A) op(B) + beta C, op = transpose
// when ta / tb.  `split` (may be NULL) is scratch for split-K partial
// products: split_elems doubles (or floats); without it no split is used.
template <typename T>
void gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, T alpha,
          const T *A, int lda, const T *B, int ldb, T beta, T *C, int ldc,
          T *split, size_t split_elems, KernelClock *kc = nullptr);

// maxdev = max_{i,j < n} |(X^T X)_ij - delta_ij| for the n x n FP32 matrix
// X (ld ldx), accumulated into *maxdev (float bits, caller zeroes it).
void gemm_orth_maxdev(hipStream_t s, int n, const float *X, int ldx, float *maxdev);
void gemm_orth_maxdev64(hipStream_t s, int n, const double *X, int ldx, float *maxdev);
void trsm_lower(hipStream_t s, int n, int nrhs, const double *L, int ldl, double *B, int ldb,
                KernelClock *kc);
void normalize_cols64(hipStream_t s, int rows, int cols, const double *Y, int ldy, double *U,
                      int ldu);

// ---------------------------------------------------------------- QR
constexpr int QR_NB = 32;    // panel width of the blocked Householder QR
constexpr int QR_NBO = 128;  // outer block of the QR: trailing updates and Q applications
constexpr int QR_RC = 256;   // rows per workgroup in the panel kernels

struct QRScratch {
    double *part;   // 2 * max_groups * QR_NB
    double *head;   // 2 * QR_NB
    unsigned long long *tpart;   // one-launch panel: tagged sums, 2 * 2 * max_groups * QR_NB words
    unsigned long long *thead;   // and the tagged head row, 2 * 2 * QR_NB words
    unsigned long long *tw1 = nullptr;   // one-launch in-block update: tagged partials
    unsigned long long *tw2 = nullptr;   // and the tagged entries of V^T C (right after tw1)
    int tw_words = 0;                    // words of both
    double *vtv;    // max_groups * QR_NB * QR_NB
    double *vb;     // m * QR_NB     (explicit unit-lower block of reflectors)
    double *vbo;    // m * QR_NBO    (the same for an outer block)
    double *go;     // QR_NBO * QR_NBO  (V^T V of an outer block)
    double *tp;     // QR_NB * QR_NB    (T of the current panel)
    double *w1;     // QR_NBO * ncols_max
    double *w2;     // QR_NBO * ncols_max
    double *split;  // split-K scratch
    size_t split_elems;
    int *flags;     // max_groups step flags of the one-launch panel
    int *err = nullptr;          // device word set to 1 when a bounded wait of the
                                 // one-launch panel runs out (the factors are then
                                 // invalid); NULL: not reported
    int spin = 0;                // polls of a bounded wait before it gives up; 0 =
                                 // the default, < 0 = give up at once (testing)
    KernelClock *kc = nullptr;   // optional per-launch timing
};
size_t qr_scratch_doubles(int m, int ncols_max, size_t *split_elems);
void qr_scratch_carve(QRScratch &q, double *base, int m, int ncols_max);

// Doubles of the block factors T of an n-column QR: ceil(n / QR_NBO) blocks
// of QR_NBO x QR_NBO.
size_t qr_t_doubles(int n);
// Householder QR of the m x n matrix A (m >= n): R in the upper triangle,
// reflectors below, tau[n], block factors T of each outer block of QR_NBO
// columns (QR_NBO x QR_NBO, ld QR_NBO, upper triangular) in Tall.
void qr_factor(hipStream_t s, int m, int n, double *A, int lda, double *tau,
               double *Tall, QRScratch &q);
// C (m x ncol) <- Q C (trans = false) or Q^T C (trans = true), Q from
// qr_factor of an m x k matrix.
void qr_apply_left(hipStream_t s, bool trans, int m, int k, const double *Qf,
                   int ldq, const double *Tall, int ncol, double *C, int ldc,
                   QRScratch &q);

// ---------------------------------------------------------------- QRCP
// Businger-Golub pivot selection on a working copy of the n x n matrix A1:
// piv[k] = column chosen at step k.  W holds n*n elements of T; scratch holds
// qrcp_scratch_bytes(n, sizeof(T)) bytes.  Returns the number of launches
// the pass took (1 for the one-launch FP32 pass, else n).
size_t qrcp_scratch_bytes(int n, int elem);
double qrcp_step_bytes(int n, int k, int elem);
double qrcp_step_flops(int n, int k);
double qrcp_pass_bytes(int n, int elem);
double qrcp_pass_flops(int n);
// scale (device, may be NULL): a power of two applied to A1 before it is
// rounded to T (pivots are invariant under it); spin: polls of the one-launch
// pass's bounded waits (0 = default, < 0 = give up at once, which sends the
// pass to the step-by-step fallback).  err_out (device, may be NULL): the
// stream-ordered mode; the one-launch pass then sets *err_out when a wait ran
// out instead of being checked from the host, and nothing falls back.
template <typename T>
int qrcp_pivots(hipStream_t s, int n, const double *A1, int lda, T *W,
                 void *scratch, int *piv, KernelClock *kc = nullptr,
                 const double *scale = nullptr, int spin = 0, int *err_out = nullptr);

// ---------------------------------------------------------------- Jacobi
// Device-side state of one Jacobi stage in the stream-ordered mode (all
// sweeps enqueued, stopping decided on the device).  Zero before the stage,
// except `stop`, which may start at 1 to switch the whole stage off.
struct SweepCtl {
    int stop;       // 1: the enqueued sweeps that remain exit at once
    int sweeps;     // sweeps run
    int conv;       // 1: a stopping rule fired (not only the cap)
    int timeout;    // a bounded wait of a fused round ran out (Y invalid)
    float off[32];  // per sweep: max relative off-diagonal
};

struct JacobiWork {
    void *gram;      // partial Gram blocks
    void *wmat;      // per-pair rotation blocks
    int *skip;       // per-pair "nothing to rotate" flags
    int *flag;       // device: [0] any rotation this sweep, [1] a fused
                     // round's wait ran out
    int *hflag;      // host copy of flag[0..2]
    float *offp;     // device, per pair slot: max relative off-diagonal
                     // |g_pq| / sqrt(g_pp g_qq) seen this sweep
    float *smxp;     // device, per pair slot: max |sin| applied this sweep
    int n_real = 0;  // columns of the problem (before padding)
    KernelClock *kc = nullptr;
    float *off_hist = nullptr;  // per-sweep max relative off-diagonal (host, 32)
    double stop_off = 0.0;      // also stop once a sweep starts with off <= this
    int cross_pairs = 0;        // 1: after a sweep's first round, rotate only the
                                // pairs between the two blocks of each block pair
    int *rotmap = nullptr;      // device: per round and pair slot, 1 if rotated
    float *gpart = nullptr;     // device: partial Gram blocks of the fused FP32 round
    int *gflag = nullptr;       // device: their flags
    int fused = 0;              // 1: FP32 sweeps without V may use the fused round
    int spin = 0;               // polls of the fused round's wait (0 = default,
                                // < 0 = give up at once, a test hook)
    SweepCtl *ctl = nullptr;    // device: stream-ordered mode (see SweepCtl)
    int half = 0;               // fused round only: 1 = Gram products on the BF16
                                // matrix cores; 2 = that, and Y stored in BF16
                                // (the float pointer passed in is the BF16 array)
};
// Whether the fused FP32 round (half: its BF16 variant 1 or 2) runs for N
// rows and columns on the current device.
bool jacobi_fused_ok(int N, int half);
size_t jacobi_scratch_bytes(int N, int b, int elem);
void jacobi_carve(JacobiWork &j, char *base, int N, int b, int elem);
// One-sided block-Jacobi sweeps on Y (N x N padded, ld N) with optional V
// accumulation (V: N x N, ld N).  Returns the number of sweeps run (-1 on a
// HIP error, -2 when a bounded wait of the fused FP32 round ran out, which
// leaves Y invalid); *conv set to 1 if the last sweep rotated nothing.
template <typename T>
int jacobi_sweeps(hipStream_t s, int N, int b, T *Y, T *V, double eps,
                  int maxsweep, int max_inner, JacobiWork &jw, int *conv);
// The same on the first ncols columns of Y and V only (ncols a multiple of 2b).
template <typename T>
int jacobi_sweeps_cols(hipStream_t s, int N, int ncols, int b, T *Y, T *V, double eps,
                       int maxsweep, int max_inner, JacobiWork &jw, int *conv);
void scatter_cols(hipStream_t s, int rows, int n, const double *D, int ldd, const int *idx, double *A,
                  int lda);
void gram_colmax_offdiag64(hipStream_t s, int n, const double *X, int ldx, float *dev);

// ---------------------------------------------------------------- misc
void copy_scan(hipStream_t s, int m, int n, const double *A, int lda,
               double *D, int ldd, int *nonfinite);
void copy_upper(hipStream_t s, int n, const double *R, int ldr, double *D, int ldd);
void gather_cols(hipStream_t s, int rows, int n, const double *A, int lda,
                 const int *piv, double *D, int ldd);
void transpose_upper_to_lower(hipStream_t s, int n, const double *R, int ldr,
                              double *L, int ldl, int Npad);
void set_identity(hipStream_t s, int N, double *V, int ldv);
void zero_pad_fill(hipStream_t s, int rows, int cols, double *D, int ldd);
// B (cols x rows) = A^T (A rows x cols).
void transpose64(hipStream_t s, int rows, int cols, const double *A, int lda, double *B, int ldb);
void diag_cond(hipStream_t s, int n, const double *R, int ldr, double *out);
void col_norms(hipStream_t s, int rows, int n, const double *X, int ldx, double *nrm);
void count_small(hipStream_t s, int n, const double *nrm, double rel, int *out);
void make_xt32(hipStream_t s, int n, const double *X, int ldx, float *Xt, int ldt);
// Y = fp32(X * scale[0]) (scale: device pointer, NULL = 1)
void convert_f64_f32(hipStream_t s, int rows, int cols, const double *X, int ldx, float *Y, int ldy,
                     const double *scale = nullptr);
// scale[0] = the power of two that brings the largest of the n norms nrm[]
// to about 2^56 (range guard for FP32 copies; see misc.hip)
void pow2_scale(hipStream_t s, int n, const double *nrm, double *scale);
void convert_f32_f64(hipStream_t s, int rows, int cols, const float *X, int ldx, double *Y, int ldy);
// Y16 = bf16(X * scale[0]) (round to nearest even; scale: device, NULL = 1),
// and Y = fp32(Y16) (exact)
void convert_f64_bf16(hipStream_t s, int rows, int cols, const double *X, int ldx,
                      unsigned short *Y, int ldy, const double *scale);
void widen_bf16_f32(hipStream_t s, int rows, int cols, const unsigned short *Y16, int ld16,
                    float *Y, int ldy);
void normalize_f32_to_f64(hipStream_t s, int rows, int cols, const float *Y, int ldy, double *U, int ldu);
void finalize_sort(hipStream_t s, int n, int N, const double *Y, const double *V,
                   double *sig, int *rank, double *UX, double *VX, double *S, int *nzero,
                   int *nonfinite, bool want_v);
void place_u(hipStream_t s, int m, int n, const double *W, int ldw, double *U, int ldu);
void permute_rows_v(hipStream_t s, int n, const double *T, int ldt, const int *piv,
                    double *V, int ldv);
void sign_normalize(hipStream_t s, int m, int n, double *U, int ldu, bool have_u,
                    double *V, int ldv);

} // namespace mpj

namespace mpj {
// Records the first HIP failure of the current call (thread-local) so that
// svd_last_error() can report it.
void note_hip_error(hipError_t e, const char *where);
// Records a message (no HIP error behind it) for svd_last_error().
void note_error_text(const char *msg);
}

#define MPJ_CHECK(x)                                                        \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) {                                             \
            mpj::note_hip_error(e_, #x);                                    \
            return SVD_ERR_HIP;                                             \
        }                                                                   \
    } while (0)
