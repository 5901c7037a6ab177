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
#include <climits>

#include "../../include/mpjsvd.h"
#include "common.hpp"
#include "internal.hpp"


namespace mpj {

constexpr int CP_NT = 256;       // threads per workgroup (4 wavefronts)
constexpr int CP_CPW = 16;       // columns per workgroup (4 per wavefront)
constexpr int CP_MAXN = 8192;    // pivot column cached in LDS

template <typename T>
__global__ __launch_bounds__(CP_NT) void qrcp_init(int n, const double *A1, int lda, T *W,
                                                   T *nrm, const double *scale) {
    // one wavefront per column: convert and take the full column norm
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * (CP_NT / 64) + (threadIdx.x >> 6);
    if (j >= n) return;
    const double f = scale ? *scale : 1.0;
    T s = 0;
    for (int i = lane; i < n; i += 64) {
        const T v = (T)(A1[(size_t)j * lda + i] * f);
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


// Register-cached step with column compaction (n <= 64 * RPL).
//
// Before step k the live positions are k..n-1; position j holds the data of
// working column perm[j] (columns never move; perm is the indirection).  Step
// k takes the pivot position p from the per-workgroup candidates of step k-1
// (largest trailing norm, ties to the smallest column index), exchanges
// positions k and p (position p now refers to the column that sat at k), and
// updates the live positions k+1..n-1 with the reflector of the pivot column.
// One wavefront owns one position: its column's rows k..n-1 are held in
// registers (row k + lane + 64 r in x[r]), loaded before the pivot is known,
// and stored once.  The reflector needs only the pivot's row-k entry and its
// trailing norm (carried in the candidate), so the pivot column is staged in
// LDS only for the dot products.  Each workgroup leaves the best of its new
// trailing norms (rows k+1..n-1) as the candidate for step k+1.
constexpr int Q2_NT = 512;            // 8 wavefronts = 8 positions per workgroup
constexpr int Q2_W = Q2_NT / 64;

template <typename T>
struct Cand {
    T v;
    int pos, col;
};

template <typename T>
__device__ __forceinline__ bool cand_better(T v, int c, T bv, int bc) {
    return v > bv || (v == bv && c < bc);
}

template <typename T>
__global__ __launch_bounds__(Q2_NT) void qrcp_init2(int n, const double *A1, int lda, T *W,
                                                    int *perm, Cand<T> *cout,
                                                    const double *scale) {
    __shared__ T cv[Q2_W];
    __shared__ int cc[Q2_W];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * Q2_W + w;
    const double f = scale ? *scale : 1.0;
    T s = 0;
    if (j < n) {
        for (int i = lane; i < n; i += 64) {
            const T v = (T)(A1[(size_t)j * lda + i] * f);
            W[(size_t)j * n + i] = v;
            s += v * v;
        }
    }
    s = wave_sum(s);
    if (lane == 0) {
        cv[w] = j < n ? tsqrt(s) : T(-1);
        cc[w] = j < n ? j : INT_MAX;
        if (j < n) perm[j] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        T bv = cv[0];
        int bc = cc[0];
        for (int q = 1; q < Q2_W; ++q)
            if (cand_better(cv[q], cc[q], bv, bc)) { bv = cv[q]; bc = cc[q]; }
        cout[blockIdx.x] = Cand<T>{bv, bc, bc};
    }
}

template <typename T, int RPL>
__global__ __launch_bounds__(Q2_NT) void qrcp_step2(int k, int n, T *__restrict__ W,
                                                    int *__restrict__ perm,
                                                    const Cand<T> *__restrict__ cin, int ncin,
                                                    Cand<T> *__restrict__ cout,
                                                    int *__restrict__ piv) {
    __shared__ T pc[64 * RPL];
    __shared__ T rv[Q2_W];
    __shared__ int rp[Q2_W], rc[Q2_W];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int j = k + 1 + blockIdx.x * Q2_W + w;
    const bool live = j < n;
    const int m = n - k;                      // rows k..n-1

    // the owned position's column, loaded before the pivot is known
    int col = live ? perm[j] : 0;
    T x[RPL];
    auto load = [&](int c) {
        const T *src = W + (size_t)c * n + k;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            x[r] = i < m ? src[i] : T(0);
        }
    };
    if (live) load(col);

    // 1. pivot: best of the previous step's candidates
    T bv = T(-2);
    int bp = -1, bc = INT_MAX;
    if (t < ncin) {
        const Cand<T> c = cin[t];
        bv = c.v; bp = c.pos; bc = c.col;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T ov = __shfl_xor(bv, o, 64);
        const int op = __shfl_xor(bp, o, 64);
        const int oc = __shfl_xor(bc, o, 64);
        if (cand_better(ov, oc, bv, bc)) { bv = ov; bp = op; bc = oc; }
    }
    if (lane == 0) { rv[w] = bv; rp[w] = bp; rc[w] = bc; }
    __syncthreads();
    bv = rv[0]; bp = rp[0]; bc = rc[0];
#pragma unroll
    for (int q = 1; q < Q2_W; ++q)
        if (cand_better(rv[q], rc[q], bv, bc)) { bv = rv[q]; bp = rp[q]; bc = rc[q]; }
    const int p = bp, pcol = bc;
    const T pnorm = bv;

    // 2. stage the pivot column (rows k..n-1); position p takes over the
    // column that sat at position k
    {
        const T *src = W + (size_t)pcol * n + k;
        for (int i = t; i < m; i += Q2_NT) pc[i] = src[i];
    }
    if (blockIdx.x == 0 && t == 0) piv[k] = pcol;
    if (live && j == p) {
        col = perm[k];
        load(col);
        if (lane == 0) perm[p] = col;
    }
    __syncthreads();

    // 3. reflector H = I - tau v v^T with v = [1; x(k+1:)/(x_k - beta)]
    T tau = 0, scale = 0;
    {
        const T x0 = pc[0];
        if (pnorm > T(0)) {
            const T beta = -copysign(pnorm, x0);
            tau = (beta - x0) / beta;
            scale = T(1) / (x0 - beta);
        }
    }

    // 4. apply it to the owned column, store rows k+1..n-1, new trailing norm
    T nv = T(-1);
    if (live) {
        T d = 0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            if (i >= 1 && i < m) d += pc[i] * x[r];
        }
        d = wave_sum(d);
        const T xk = __shfl(x[0], 0, 64);
        const T wv = tau * (xk + scale * d);
        const T f = wv * scale;
        T ns = 0;
        T *dst = W + (size_t)col * n + k;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            if (i >= 1 && i < m) {
                const T v = x[r] - f * pc[i];
                dst[i] = v;
                ns += v * v;
            }
        }
        nv = tsqrt(wave_sum(ns));
    }

    // 5. this workgroup's candidate for step k+1
    __syncthreads();   // rv/rp/rc are reused
    if (lane == 0) { rv[w] = nv; rp[w] = live ? j : -1; rc[w] = live ? col : INT_MAX; }
    __syncthreads();
    if (t == 0) {
        T cv = rv[0];
        int cp = rp[0], cc = rc[0];
        for (int q = 1; q < Q2_W; ++q)
            if (cand_better(rv[q], rc[q], cv, cc)) { cv = rv[q]; cp = rp[q]; cc = rc[q]; }
        cout[blockIdx.x] = Cand<T>{cv, cp, cc};
    }
}

// Whole pass in one launch (FP32, n <= 4096): the working matrix never
// leaves registers.  Wavefront w of workgroup b owns column 16 b + w for the
// whole pass (rows lane + 64 r in x[r]); used columns drop out.  Step k:
//   1. each workgroup takes its best live column (largest trailing norm, ties
//      to the smallest index) as its candidate, publishes that column's rows
//      k..n-1 (double-buffered by step parity) with device-coherent stores,
//      waits for them to complete, then publishes its candidate as one
//      64-bit key: step k + 1 | norm bits | 8191 - column (0 for none), so
//      that the largest key of a step is the pivot with the tie rule;
//   2. it polls, with a bound, until every key of the step is in, takes the
//      largest, and reads the pivot column from its owner's slot;
//   3. it applies the reflector to its live columns and recomputes their
//      trailing norms (rows k+1..n-1).
// A wait that runs out sets *err and the host redoes the pass step by step.
// Requires all workgroups resident at once: one per compute unit, launched
// only when the device has a unit for each.
constexpr int QP_NT = 1024;
constexpr int QP_W = QP_NT / 64;
constexpr int QP_SPIN = 1 << 22;
constexpr int QP_TAG = 45;            // key bits [45, 64): step tag

__device__ __forceinline__ unsigned long long qp_key(int step, float v, int col) {
    if (!(v >= 0.f)) return (unsigned long long)step << QP_TAG;
    return ((unsigned long long)step << QP_TAG) |
           ((unsigned long long)__float_as_uint(v) << 13) | (unsigned long long)(8191 - col);
}

template <int RPL>
__global__ __launch_bounds__(QP_NT) void qrcp_persist(int n, const double *__restrict__ A1,
                                                     int lda, float *__restrict__ cbuf,
                                                     unsigned long long *__restrict__ keys,
                                                     int *err, int *__restrict__ piv,
                                                     const double *ascale, int spin) {
    typedef float T;
    // The step's pivot column in LDS, lane-major: row lane + 64 r of the
    // column sits at pc[lane * PL + r], so a lane reads the entries of its
    // own rows four at a time (128-bit reads; the row pad of 4 entries puts
    // the lanes of each read on distinct banks).
    constexpr int NP = 64 * RPL;          // candidate slot length in cbuf (rows >= n unused)
    constexpr int PL = RPL + 4;
    __shared__ __align__(16) T pc[64 * PL];
    __shared__ unsigned long long rk[QP_W];
    __shared__ int bad;
    const int nwg = gridDim.x;
    const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int j = b * QP_W + w;
    bool live = j < n;
    T x[RPL];
    T nv;
    {
        const double f = ascale ? *ascale : 1.0;
        T ns = 0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            x[r] = (live && i < n) ? (T)(A1[(size_t)j * lda + i] * f) : T(0);
            ns += x[r] * x[r];
        }
        nv = live ? tsqrt(wave_sum(ns)) : T(-1);
    }
    for (int i = t; i < 64 * PL; i += QP_NT) pc[i] = T(0);
    auto pidx = [](int i) { return (i & 63) * PL + (i >> 6); };
    if (t == 0) bad = 0;
    for (int k = 0; k < n; ++k) {
        const int buf = k & 1;
        const int r0 = k >> 6, kl = k & 63;
        // 1. this workgroup's candidate, its rows k..n-1, then its key
        if (lane == 0) rk[w] = live ? qp_key(k + 1, nv, j) : qp_key(k + 1, -1.f, 0);
        __syncthreads();
        unsigned long long bk = lane < QP_W ? rk[lane] : 0ull;
        int bw = lane;
#pragma unroll
        for (int o = QP_W / 2; o > 0; o >>= 1) {
            const unsigned long long ok = __shfl_xor(bk, o, 64);
            const int ow = __shfl_xor(bw, o, 64);
            if (ok > bk) { bk = ok; bw = ow; }
        }
        bk = __shfl(bk, 0, 64); bw = __shfl(bw, 0, 64);
        const bool any = (bk & ((1ull << QP_TAG) - 1)) != 0;
        if (w == bw && any) {
#pragma unroll
            for (int r = 0; r < RPL; r += 4)
                *reinterpret_cast<flt4 *>(pc + lane * PL + r) = flt4{x[r], x[r + 1], x[r + 2], x[r + 3]};
        }
        __syncthreads();
        if (any) {
            T *cb = cbuf + ((size_t)buf * nwg + b) * NP;
            for (int i = k + t; i < n; i += QP_NT) coh_store(cb + i, pc[pidx(i)]);
        }
        // every wavefront's stores are complete before the key goes out
        publish_fence();
        __syncthreads();
        if (t == 0) coh_store(keys + (size_t)buf * nwg + b, bk);
        // 2. every workgroup's key of step k; the largest is the pivot
        unsigned long long gk = 0ull;
        if (t < nwg) {
            int it = 0;
            for (;;) {
                gk = coh_load(keys + (size_t)buf * nwg + t);
                if ((int)(gk >> QP_TAG) == k + 1 && spin >= 0) break;
                if (spin < 0 || ++it > spin) { bad = 1; gk = 0ull; break; }
                __builtin_amdgcn_s_sleep(1);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long ok = __shfl_xor(gk, o, 64);
            if (ok > gk) gk = ok;
        }
        if (lane == 0) rk[w] = gk;   // rk was last read before the previous barrier
        __syncthreads();
        gk = lane < QP_W ? rk[lane] : 0ull;
#pragma unroll
        for (int o = QP_W / 2; o > 0; o >>= 1) {
            const unsigned long long ok = __shfl_xor(gk, o, 64);
            if (ok > gk) gk = ok;
        }
        gk = __shfl(gk, 0, 64);
        const int p = min(max(8191 - (int)(gk & 8191ull), 0), n - 1);
        const T pnorm = __uint_as_float((unsigned)((gk >> 13) & 0xffffffffull));
        {
            const T *src = cbuf + ((size_t)buf * nwg + p / QP_W) * NP;
            for (int i = k + t; i < n; i += QP_NT) pc[pidx(i)] = coh_load(src + i);
        }
        if (b == 0 && t == 0) {
            piv[k] = p;
            if (bad) *err = 1;
        }
        __syncthreads();
        // 3. reflector H = I - tau v v^T, v = [1; x(k+1:)/(x_k - beta)], and update
        T tau = 0, scale = 0;
        {
            const T x0 = pc[pidx(k)];
            if (pnorm > T(0)) {
                const T beta = -copysign(pnorm, x0);
                tau = (beta - x0) / beta;
                scale = T(1) / (x0 - beta);
            }
        }
        if (live && j == p) {
            live = false;
            nv = T(-1);
        } else if (live) {
            // (groups of 8 registers: the empty asm statements keep the
            // compiler from holding RPL staged pivot entries live at once)
            // Groups of 8 rows wholly above the pivot row are skipped.
            T d = 0, xk = 0;
            const T *pl = pc + lane * PL;
#pragma unroll
            for (int rg = 0; rg < RPL; rg += 8) {
                if (rg + 7 >= r0) {
                    const flt4 v0 = *reinterpret_cast<const flt4 *>(pl + rg);
                    const flt4 v1 = *reinterpret_cast<const flt4 *>(pl + rg + 4);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int r = rg + e;
                        const T pv = e < 4 ? v0[e & 3] : v1[e & 3];
                        if (r > r0) {
                            d += pv * x[r];
                        } else if (r == r0) {
                            xk = x[r];
                            if (lane > kl) d += pv * x[r];
                        }
                    }
                }
                __asm__ volatile("" ::: "memory");
            }
            d = wave_sum(d);
            xk = __shfl(xk, kl, 64);
            const T f = tau * (xk + scale * d) * scale;
            T ns = 0;
#pragma unroll
            for (int rg = 0; rg < RPL; rg += 8) {
                if (rg + 7 >= r0) {
                    const flt4 v0 = *reinterpret_cast<const flt4 *>(pl + rg);
                    const flt4 v1 = *reinterpret_cast<const flt4 *>(pl + rg + 4);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int r = rg + e;
                        const T pv = e < 4 ? v0[e & 3] : v1[e & 3];
                        if (r > r0 || (r == r0 && lane > kl)) {
                            x[r] -= f * pv;
                            ns += x[r] * x[r];
                        }
                    }
                }
                __asm__ volatile("" ::: "memory");
            }
            nv = tsqrt(wave_sum(ns));
        }
    }
}

__global__ void qrcp_persist_reset(int nkeys, unsigned long long *keys, int *err) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nkeys) keys[e] = 0ull;
    if (e == 0) *err = 0;
}

// Algorithmic work of pivot step k (the trailing-matrix pass of Businger-
// Golub QRCP): the m x (m-1) trailing block read once (m = n - k), and
// 4 m (m-1) flops (the dot products and the rank-one update).
double qrcp_step_bytes(int n, int k, int elem) {
    const double m = n - k;
    return m * (m - 1) * elem;
}
double qrcp_step_flops(int n, int k) {
    const double m = n - k;
    return 4.0 * m * (m - 1);
}
double qrcp_pass_bytes(int n, int elem) {
    double b = 0.0;
    for (int k = 0; k < n; ++k) b += qrcp_step_bytes(n, k, elem);
    return b;
}
double qrcp_pass_flops(int n) {
    double f = 0.0;
    for (int k = 0; k < n; ++k) f += qrcp_step_flops(n, k);
    return f;
}

size_t qrcp_scratch_bytes(int n, int elem) {
    // fallback: two norm vectors; compacted step: perm + two candidate arrays
    const size_t a = (size_t)2 * n * elem;
    const size_t ncand = (size_t)cdiv(n, Q2_W) + 1;
    const size_t b = (size_t)n * sizeof(int) + 64 + 2 * ncand * sizeof(Cand<double>);
    const size_t nwg = (size_t)cdiv(n, QP_W);
    const size_t c = 2 * nwg * sizeof(unsigned long long) + 256;
    size_t m = a > b ? a : b;
    return m > c ? m : c;
}

// A wait of the one-launch pass that ran out, passed on to *out (OR).
__global__ void qrcp_err_out(const int *err, int *out) {
    if (threadIdx.x == 0 && *err) *out = 1;
}

// The one-launch FP32 pass; false when it does not apply or could not run
// (then nothing observable has changed and the caller takes the step path).
// err_out set (stream-ordered mode): the pass's time-out flag is passed on
// to *err_out on the device instead of being read back, and there is no
// fallback (the pivots are then a clamped, possibly repeating, column list).
static bool qrcp_persist_pass(hipStream_t s, int n, const double *A1, int lda, float *W,
                              void *scratch, int *piv, KernelClock *kc, const double *scale,
                              int spin, int *err_out) {
    const int sp = spin == 0 ? QP_SPIN : spin;
    if (n < 128 || n > 64 * 64) return false;
    const int nwg = cdiv(n, QP_W);
    unsigned long long *keys = (unsigned long long *)scratch;
    int *err = (int *)(keys + 2 * (size_t)nwg);
    float *cbuf = W;   // 2 * nwg * 64 RPL floats <= n * n doubles (the working copy is not needed)
    const void *fn;
    if (n <= 64 * 16) fn = (const void *)qrcp_persist<16>;
    else if (n <= 64 * 32) fn = (const void *)qrcp_persist<32>;
    else fn = (const void *)qrcp_persist<64>;
    // every workgroup must be resident at once: at most one per compute unit
    // here, and only if the kernel fits one per unit
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, QP_NT, 0) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (per_cu < 1 || nwg > ncu) return false;
    hipLaunchKernelGGL(qrcp_persist_reset, dim3(cdiv(2 * nwg, 256)), dim3(256), 0, s, 2 * nwg, keys,
                       err);
    if (kc) kc->begin(s, SVD_K_QRCP, qrcp_pass_bytes(n, sizeof(float)), qrcp_pass_flops(n));
    if (n <= 64 * 16)
        hipLaunchKernelGGL((qrcp_persist<16>), dim3(nwg), dim3(QP_NT), 0, s, n, A1, lda, cbuf, keys,
                           err, piv, scale, sp);
    else if (n <= 64 * 32)
        hipLaunchKernelGGL((qrcp_persist<32>), dim3(nwg), dim3(QP_NT), 0, s, n, A1, lda, cbuf, keys,
                           err, piv, scale, sp);
    else
        hipLaunchKernelGGL((qrcp_persist<64>), dim3(nwg), dim3(QP_NT), 0, s, n, A1, lda, cbuf, keys,
                           err, piv, scale, sp);
    if (kc) kc->end(s);
    if (hipGetLastError() != hipSuccess) return false;
    if (err_out) {
        hipLaunchKernelGGL(qrcp_err_out, dim3(1), dim3(64), 0, s, (const int *)err, err_out);
        return hipGetLastError() == hipSuccess;
    }
    int h_err = 1;
    if (hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return h_err == 0;
}

template <typename T>
int qrcp_pivots(hipStream_t s, int n, const double *A1, int lda, T *W, void *scratch, int *piv,
                KernelClock *kc, const double *scale, int spin, int *err_out) {
    if (n <= 0) return 0;
    if (n > 64 * 64) {
        T *norms2 = (T *)scratch;
        hipLaunchKernelGGL((qrcp_init<T>), dim3(cdiv(n, CP_NT / 64)), dim3(CP_NT), 0, s, n, A1, lda,
                           W, norms2, scale);
        for (int k = 0; k < n; ++k) {
            const T *nin = norms2 + (size_t)(k & 1) * n;
            T *nout = norms2 + (size_t)((k + 1) & 1) * n;
            if (kc) kc->begin(s, SVD_K_QRCP, qrcp_step_bytes(n, k, sizeof(T)), qrcp_step_flops(n, k));
            hipLaunchKernelGGL((qrcp_step<T>), dim3(cdiv(n, CP_CPW)), dim3(CP_NT), 0, s, k, n, W, nin,
                               nout, piv);
            if (kc) kc->end(s);
        }
        return n;
    }
    if (sizeof(T) == 4 &&
        qrcp_persist_pass(s, n, A1, lda, (float *)W, scratch, piv, kc, scale, spin, err_out))
        return 1;
    int *perm = (int *)scratch;
    const size_t ncand = (size_t)cdiv(n, Q2_W) + 1;
    Cand<T> *cand = (Cand<T> *)((char *)scratch + (((size_t)n * sizeof(int) + 63) / 64) * 64);
    hipLaunchKernelGGL((qrcp_init2<T>), dim3(cdiv(n, Q2_W)), dim3(Q2_NT), 0, s, n, A1, lda, W, perm,
                       cand, scale);
    for (int k = 0; k < n; ++k) {
        const Cand<T> *cin = cand + (size_t)(k & 1) * ncand;
        Cand<T> *cout = cand + (size_t)((k + 1) & 1) * ncand;
        const int ncin = cdiv(n - k, Q2_W);
        const int nwg = n - k - 1 > 0 ? cdiv(n - k - 1, Q2_W) : 1;
        if (kc) kc->begin(s, SVD_K_QRCP, qrcp_step_bytes(n, k, sizeof(T)), qrcp_step_flops(n, k));
        if (n <= 64 * 16)
            hipLaunchKernelGGL((qrcp_step2<T, 16>), dim3(nwg), dim3(Q2_NT), 0, s, k, n, W, perm, cin,
                               ncin, cout, piv);
        else if (n <= 64 * 32)
            hipLaunchKernelGGL((qrcp_step2<T, 32>), dim3(nwg), dim3(Q2_NT), 0, s, k, n, W, perm, cin,
                               ncin, cout, piv);
        else
            hipLaunchKernelGGL((qrcp_step2<T, 64>), dim3(nwg), dim3(Q2_NT), 0, s, k, n, W, perm, cin,
                               ncin, cout, piv);
        if (kc) kc->end(s);
    }
    return n;
}

template int qrcp_pivots<float>(hipStream_t, int, const double *, int, float *, void *, int *,
                                KernelClock *, const double *, int, int *);
template int qrcp_pivots<double>(hipStream_t, int, const double *, int, double *, void *, int *,
                                 KernelClock *, const double *, int, int *);

} // namespace mpj
