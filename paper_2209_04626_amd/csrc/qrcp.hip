// Pivot selection of Businger-Golub QR with column pivoting (the RRQR of
// Section 2.2), run in FP32 for Algorithm 5 (only the permutation P is kept;
// the FP64 QR of A1 P follows) or in FP64 for the plain path.
//
// Per-step form (fallback): one launch per elimination step k.  Every
// workgroup redundantly picks the
// pivot (largest remaining trailing column norm, ties to the smallest column
// index), builds the Householder reflector of that column from its trailing
// part, applies it to the columns it owns and writes their new trailing
// norms, recomputed from the updated entries rather than downdated.  Norms are
// double-buffered between launches so that the pivot every workgroup reads
// is the one all of them read.  Columns stay in place; a used column is
// marked by a norm of -1.
#include "common.hpp"
#include "internal.hpp"


namespace mpj {

constexpr int CP_NT = 256;       // threads per workgroup (4 wavefronts)
constexpr int CP_CPW = 16;       // columns per workgroup (4 per wavefront)
constexpr int CP_MAXN = 8192;    // pivot column cached in LDS

template <typename T>
__global__ __launch_bounds__(CP_NT) void qrcp_init(int n, const double *A1, int lda, T *W,
                                                   T *nrm) {
    // one wavefront per column: convert and take the full column norm
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * (CP_NT / 64) + (threadIdx.x >> 6);
    if (j >= n) return;
    T s = 0;
    for (int i = lane; i < n; i += 64) {
        const T v = (T)A1[(size_t)j * lda + i];
        W[(size_t)j * n + i] = v;
        s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) nrm[j] = tsqrt(s);
}

template <typename T>
__global__ __launch_bounds__(CP_NT) void qrcp_step(int k, int n, T *W, const T *nin, T *nout,
                                                   int *piv) {
    __shared__ T pc[CP_MAXN];
    __shared__ T rv[CP_NT / 64];
    __shared__ int ri[CP_NT / 64];
    __shared__ T red[CP_NT / 64];
    __shared__ T prm[3];
    __shared__ int psh;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;

    // 1. pivot: argmax of the remaining norms, ties to the smallest index
    T best = -2;
    int bi = n;
    for (int j = t; j < n; j += CP_NT) {
        const T v = nin[j];
        if (v > best) { best = v; bi = j; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T ov = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { rv[w] = best; ri[w] = bi; }
    __syncthreads();
    if (t == 0) {
        T b = rv[0];
        int i = ri[0];
        for (int q = 1; q < CP_NT / 64; ++q)
            if (rv[q] > b || (rv[q] == b && ri[q] < i)) { b = rv[q]; i = ri[q]; }
        psh = i;
        if (blockIdx.x == 0) piv[k] = i;
    }
    __syncthreads();
    const int p = psh;

    // 2. reflector of the pivot column from rows k..n-1
    T s = 0;
    for (int i = k + t; i < n; i += CP_NT) {
        const T v = W[(size_t)p * n + i];
        pc[i] = v;
        if (i > k) s += v * v;
    }
    s = block_sum<CP_NT>(s, red);
    if (t == 0) {
        const T x0 = pc[k];
        const T xn = tsqrt(s);
        T tau = 0, scale = 0;
        if (xn != T(0)) {
            const T beta = -copysign(tsqrt(x0 * x0 + s), x0);
            tau = (beta - x0) / beta;
            scale = T(1) / (x0 - beta);
        }
        prm[1] = tau; prm[2] = scale;
    }
    __syncthreads();
    const T tau = prm[1], scale = prm[2];

    // 3. update the owned columns and recompute their trailing norms
    for (int c = w; c < CP_CPW; c += CP_NT / 64) {
        const int j = blockIdx.x * CP_CPW + c;
        if (j >= n) break;
        const T nj = nin[j];
        if (j == p || nj < T(0)) {
            if (lane == 0) nout[j] = T(-1);
            continue;
        }
        T* col = W + (size_t)j * n;
        T d = 0;
        for (int i = k + 1 + lane; i < n; i += 64) d += pc[i] * col[i];
        d = wave_sum(d);
        const T wv = tau * (col[k] + scale * d);
        T ns = 0;
        for (int i = k + 1 + lane; i < n; i += 64) {
            const T v = col[i] - wv * scale * pc[i];
            col[i] = v;
            ns += v * v;
        }
        ns = wave_sum(ns);
        if (lane == 0) {
            col[k] -= wv;
            nout[j] = tsqrt(ns);
        }
    }
}


// Register-cached step: one wavefront per owned column, the column's rows
// k..n-1 are loaded into registers with all loads in flight, then the dot
// product, the update and the new trailing norm are computed from registers
// and the column is stored once.  Requires n <= 64 * RPL.
constexpr int CR_NT = 512;            // 8 wavefronts = 8 columns per workgroup
constexpr int CR_W = CR_NT / 64;

template <typename T, int RPL>
__global__ __launch_bounds__(CR_NT) void qrcp_step_reg(int k, int n, T *W, const T *nin, T *nout,
                                                       int *piv) {
    __shared__ T pc[CP_MAXN];
    __shared__ T rv[CR_W];
    __shared__ int ri[CR_W];
    __shared__ T red[CR_W];
    __shared__ T prm[2];
    __shared__ int psh;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int j = blockIdx.x * CR_W + w;

    // the owned column: start its loads before the pivot search
    T x[RPL];
    const bool live = j < n && nin[j] >= T(0);
    if (live) {
        const T *col = W + (size_t)j * n;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            x[r] = (i >= k && i < n) ? col[i] : T(0);
        }
    }

    // 1. pivot: argmax of the remaining norms, ties to the smallest index
    T best = -2;
    int bi = n;
    for (int q = t; q < n; q += CR_NT) {
        const T v = nin[q];
        if (v > best) { best = v; bi = q; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T ov = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { rv[w] = best; ri[w] = bi; }
    __syncthreads();
    if (t == 0) {
        T b = rv[0];
        int i = ri[0];
        for (int q = 1; q < CR_W; ++q)
            if (rv[q] > b || (rv[q] == b && ri[q] < i)) { b = rv[q]; i = ri[q]; }
        psh = i;
        if (blockIdx.x == 0) piv[k] = i;
    }
    __syncthreads();
    const int p = psh;

    // 2. reflector of the pivot column from rows k..n-1
    T s = 0;
    for (int i = k + t; i < n; i += CR_NT) {
        const T v = W[(size_t)p * n + i];
        pc[i] = v;
        if (i > k) s += v * v;
    }
    s = block_sum<CR_NT>(s, red);
    if (t == 0) {
        const T x0 = pc[k];
        T tau = 0, scale = 0;
        if (s != T(0)) {
            const T beta = -copysign(tsqrt(x0 * x0 + s), x0);
            tau = (beta - x0) / beta;
            scale = T(1) / (x0 - beta);
        }
        prm[0] = tau; prm[1] = scale;
    }
    __syncthreads();
    if (j >= n) return;
    if (!live || j == p) {
        if (lane == 0) nout[j] = T(-1);
        return;
    }
    const T tau = prm[0], scale = prm[1];

    // 3. update the owned column from registers, store once
    T d = 0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i > k && i < n) d += pc[i] * x[r];
    }
    d = wave_sum(d);
    const int qk = k / 64, rk = k % 64;
    T xk = 0;
#pragma unroll
    for (int r = 0; r < RPL; ++r)
        if (r == qk) xk = x[r];
    xk = __shfl(xk, rk, 64);
    const T wv = tau * (xk + scale * d);
    T ns = 0;
    T *col = W + (size_t)j * n;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i > k && i < n) {
            const T v = x[r] - wv * scale * pc[i];
            col[i] = v;
            ns += v * v;
        } else if (i == k) {
            col[i] = x[r] - wv;
        }
    }
    ns = wave_sum(ns);
    if (lane == 0) nout[j] = tsqrt(ns);
}

template <typename T>
void qrcp_pivots(hipStream_t s, int n, const double *A1, int lda, T *W, T *norms2, int *piv,
                 KernelClock *kc) {
    if (n <= 0) return;
    hipLaunchKernelGGL((qrcp_init<T>), dim3(cdiv(n, CP_NT / 64)), dim3(CP_NT), 0, s, n, A1, lda, W,
                       norms2);
    for (int k = 0; k < n; ++k) {
        const T *nin = norms2 + (size_t)(k & 1) * n;
        T *nout = norms2 + (size_t)((k + 1) & 1) * n;
        const dim3 g(cdiv(n, CR_W));
        // algorithmic bytes of step k: the active trailing block (rows k..n-1
        // of the n-k-1 remaining columns) read and written once, the pivot
        // column read once
        const double m = n - k;
        if (kc) kc->begin(s, 6, (2.0 * m * (m - 1) + m) * sizeof(T));
        if (n <= 64 * 16)
            hipLaunchKernelGGL((qrcp_step_reg<T, 16>), g, dim3(CR_NT), 0, s, k, n, W, nin, nout, piv);
        else if (n <= 64 * 32)
            hipLaunchKernelGGL((qrcp_step_reg<T, 32>), g, dim3(CR_NT), 0, s, k, n, W, nin, nout, piv);
        else if (n <= 64 * 64)
            hipLaunchKernelGGL((qrcp_step_reg<T, 64>), g, dim3(CR_NT), 0, s, k, n, W, nin, nout, piv);
        else
            hipLaunchKernelGGL((qrcp_step<T>), dim3(cdiv(n, CP_CPW)), dim3(CP_NT), 0, s, k, n, W, nin,
                               nout, piv);
        if (kc) kc->end(s);
    }
}

template void qrcp_pivots<float>(hipStream_t, int, const double *, int, float *, float *, int *,
                                 KernelClock *);
template void qrcp_pivots<double>(hipStream_t, int, const double *, int, double *, double *, int *,
                                  KernelClock *);

} // namespace mpj
