// Adjoint of the SVD for a strided batch of equal shapes (not part of the
// paper's method; the standard result for distinct singular values).
//
// With J = U^T gU, K = V^T gV and F_ij = d / (d^2 + eta^2), d = s_j^2 - s_i^2
// (F_ii = 0), the cotangent of A is
//   gA = (U M + gU S^-1) V^T,
//   M  = (F o (J - J^T)) S + diag(gS) + S (F o (K - K^T)) - J S^-1 [m > n],
// where the last term and gU S^-1 together are (I - U U^T) gU S^-1 V^T.
// One workgroup per matrix; the products run on the FP64 matrix cores with
// 64 x 64 output tiles staged through LDS; J, K, M, Z live in the workspace.
#include <stdio.h>

#include <mutex>

#include "../../include/mpjsvd.h"
#include "common.hpp"
#include "internal.hpp"
#include "wg_gemm.hpp"

namespace mpj {

constexpr int BW_NT = WG_NT;

__global__ __launch_bounds__(BW_NT) void k_svd_backward(
    int m, int n, const double *U, long long sU, const double *S, long long sS, const double *V,
    long long sV, const double *gU, const double *gS, const double *gV, double *gA, long long sA,
    double eps_deg, double *work) {
    __shared__ double As[1][16][65];
    __shared__ double Bs[1][16][65];
    const int bidx = blockIdx.x, tid = threadIdx.x;
    const double *u = U + bidx * sU, *s = S + bidx * sS, *v = V + bidx * sV;
    const double *gu = gU ? gU + bidx * sU : nullptr;
    const double *gs = gS ? gS + bidx * sS : nullptr;
    const double *gv = gV ? gV + bidx * sV : nullptr;
    double *ga = gA + bidx * sA;
    const size_t nn = (size_t)n * n;
    double *Jw = work + (size_t)bidx * (3 * nn + (size_t)m * n);
    double *Kw = Jw + nn, *Mw = Kw + nn, *Zw = Mw + nn;

    if (gu) wg_gemm<true, false>(n, n, m, u, m, gu, m, Jw, n, false, As, Bs);
    if (gv) wg_gemm<true, false>(n, n, n, v, n, gv, n, Kw, n, false, As, Bs);
    double s1 = 0.0;
    for (int i = 0; i < n; ++i) s1 = fmax(s1, s[i]);
    const double eta = eps_deg * s1 * s1;
    for (size_t e = tid; e < nn; e += BW_NT) {
        const int i = (int)(e % n), j = (int)(e / n);
        double mij = 0.0;
        if (i == j) {
            if (gs) mij = gs[i];
        } else {
            const double d = s[j] * s[j] - s[i] * s[i];
            const double den = d * d + eta * eta;
            const double f = den > 0.0 ? d / den : 0.0;
            if (gu) mij += f * (Jw[(size_t)j * n + i] - Jw[(size_t)i * n + j]) * s[j];
            if (gv) mij += s[i] * f * (Kw[(size_t)j * n + i] - Kw[(size_t)i * n + j]);
        }
        if (gu && m > n) mij -= s[j] > 0.0 ? Jw[(size_t)j * n + i] / s[j] : 0.0;
        Mw[e] = mij;
    }
    __syncthreads();
    // Z = U M (+ gU S^-1 when m > n)
    if (gu && m > n) {
        for (size_t e = tid; e < (size_t)m * n; e += BW_NT) {
            const int j = (int)(e / m);
            Zw[e] = s[j] > 0.0 ? gu[e] / s[j] : 0.0;
        }
        __syncthreads();
        wg_gemm<false, false>(m, n, n, u, m, Mw, n, Zw, m, true, As, Bs);
    } else {
        wg_gemm<false, false>(m, n, n, u, m, Mw, n, Zw, m, false, As, Bs);
    }
    // gA = Z V^T
    wg_gemm<false, true>(m, n, n, Zw, m, v, n, ga, m, false, As, Bs);
}

// Scratch of svd_backward_noalloc: a fixed device array in place of the
// caller's workspace.  Each GPU the library runs on holds its own copy from
// the load of the code object until the process ends.  Host code never uses
// the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[SVD_BACKWARD_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int BW_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[BW_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).  0, or SVD_ERR_HIP with svd_last_error() set.
int scratch_address(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { note_hip_error(e, "svd_backward_noalloc: hipGetDevice"); return SVD_ERR_HIP; }
    if (dev < 0 || dev >= BW_MAX_DEVICES) {
        note_hip_error(hipErrorInvalidDevice, "svd_backward_noalloc: device index");
        return SVD_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            note_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                           "svd_backward_noalloc: hipGetSymbolAddress(scratch)");
            return SVD_ERR_HIP;
        }
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return 0;
}
} // namespace

} // namespace mpj

using namespace mpj;

extern "C" size_t svd_backward_workspace_size(int batch, int m, int n) {
    if (batch < 0 || m < n || n < 1) return 0;
    return (size_t)batch * (3 * (size_t)n * n + (size_t)m * n) * sizeof(double) + 256;
}

// Arguments 1-14 and 16 (stream) as for svd_backward; nothing is allocated.
static int check_backward_args(int batch, int m, int n, const double *U, long long sU,
                               const double *S, long long sS, const double *V, long long sV,
                               double *gA, long long sA) {
    if (batch < 0) return -1;
    if (m < 1 || m < n) return -2;
    if (n < 1) return -3;
    if (!U) return -4;
    if (sU < (long long)m * n && batch > 1) return -5;
    if (!S) return -6;
    if (sS < n && batch > 1) return -7;
    if (!V) return -8;
    if (sV < (long long)n * n && batch > 1) return -9;
    if (!gA) return -13;
    if (sA < (long long)m * n && batch > 1) return -14;
    return 0;
}

extern "C" int svd_backward(int batch, int m, int n, const double *U, long long sU, const double *S,
                            long long sS, const double *V, long long sV, const double *gU,
                            const double *gS, const double *gV, double *gA, long long sA,
                            double eps_deg, void *work, size_t work_bytes, void *stream) {
    const int rc = check_backward_args(batch, m, n, U, sU, S, sS, V, sV, gA, sA);
    if (rc) return rc;
    if (batch == 0) return 0;
    if (!work) return -16;
    if (work_bytes < svd_backward_workspace_size(batch, m, n)) return -17;
    if (!(eps_deg > 0.0)) eps_deg = 1e-12;
    hipLaunchKernelGGL(k_svd_backward, dim3(batch), dim3(BW_NT), 0, (hipStream_t)stream, m, n, U, sU,
                       S, sS, V, sV, gU, gS, gV, gA, sA, eps_deg, (double *)work);
    return hipGetLastError() == hipSuccess ? 0 : SVD_ERR_HIP;
}

extern "C" int svd_backward_noalloc(int batch, int m, int n, const double *U, long long sU,
                                    const double *S, long long sS, const double *V, long long sV,
                                    const double *gU, const double *gS, const double *gV, double *gA,
                                    long long sA, double eps_deg, void *stream) {
    const int rc = check_backward_args(batch, m, n, U, sU, S, sS, V, sV, gA, sA);
    if (rc) return rc;
    if (batch == 0) return 0;
    const size_t need = svd_backward_workspace_size(batch, m, n);
    if (need > SVD_BACKWARD_NOALLOC_SCRATCH_BYTES) {
        char msg[160];
        snprintf(msg, sizeof(msg), "svd_backward_noalloc: %zu bytes of scratch needed, the fixed "
                 "array holds %zu", need, (size_t)SVD_BACKWARD_NOALLOC_SCRATCH_BYTES);
        note_error_text(msg);
        return SVD_ERR_SCRATCH_LIMIT;
    }
    double *work = nullptr;
    const int ra = scratch_address(&work);
    if (ra) return ra;
    if (!(eps_deg > 0.0)) eps_deg = 1e-12;
    // every word of the scratch the kernel reads it writes first (J, K, M, Z
    // per matrix), so the previous call's contents need no clearing
    hipLaunchKernelGGL(k_svd_backward, dim3(batch), dim3(BW_NT), 0, (hipStream_t)stream, m, n, U, sU,
                       S, sS, V, sV, gU, gS, gV, gA, sA, eps_deg, work);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { note_hip_error(e, "svd_backward_noalloc launch"); return SVD_ERR_HIP; }
    return 0;
}
