// Batched mixed-precision SVD of many small matrices of uneven size in one
// persistent-kernel launch (not in the paper: the batching layer around its
// Algorithm 4).
//
// Each 256-thread workgroup repeatedly takes the next matrix from a device
// work queue (matrices ordered longest first by an n^3 cost estimate, so the
// big ones start early) and runs the whole path on it with workgroup-level
// routines in its own slice of the workspace:
//   tall QR A = Q0 R1 (m > n), FP32 Businger-Golub pivots (Algorithm 5),
//   FP64 QR of A1 P, LQ step through the QR of R^T (X = L), the Section 3.5
//   tests, FP32 one-sided Jacobi without V, the switch X^T U_low = Q R2,
//   Y = X Q, FP64 one-sided Jacobi with V = Q, then the final step of
//   Algorithm 1, U = Q0 Q1 U_X, V = P Q2^T V_X and the sign rule.
// The one-sided Jacobi sweeps use the round-robin pair order, one wavefront
// per column pair, with the dot products reduced across the wavefront.
// Every wavefront reaches the queue-exhausted exit, so the grid drains.
#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/mpjsvd.h"
#include "common.hpp"
#include "internal.hpp"
#include "wg_gemm.hpp"

namespace mpj {

constexpr int BT_NT = 1024;            // 16 wavefronts: 16 column pairs at a time
constexpr int BT_W = BT_NT / 64;
constexpr int BT_MAXN = 256;

struct BatchMeta {                     // one entry per matrix
    int m, n;
    long long offA, offS, offV;
};

struct BatchParams {
    double tol_orth, tol_cond_coef, small_col_rel, small_col_frac;
    double eps_low_coef, eps_work_coef;  // eps = coef * sqrt(n) (0 -> fixed below)
    double eps_low_fixed, eps_work_fixed;
    int maxsweep_low, maxsweep_work, branch, sign_normalize;
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double bt_sum(double v, double *red) { return block_sum<BT_NT>(v, red); }

// Householder QR of the m x n (m >= n) matrix A in place; tau[n].
__device__ void wg_qr(int m, int n, double *A, int lda, double *tau, double *red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int k = 0; k < n; ++k) {
        double *x = A + (size_t)k * lda;
        double s = 0.0;
        for (int i = k + 1 + tid; i < m; i += BT_NT) s += x[i] * x[i];
        s = bt_sum(s, red);
        const double x0 = x[k];
        double beta = x0, tv = 0.0, scale = 0.0;
        if (s != 0.0) {
            beta = -copysign(sqrt(x0 * x0 + s), x0);
            tv = (beta - x0) / beta;
            scale = 1.0 / (x0 - beta);
        }
        for (int j = k + 1 + w; j < n; j += BT_W) {
            double *c = A + (size_t)j * lda;
            double d = 0.0;
            for (int i = k + 1 + lane; i < m; i += 64) d += x[i] * c[i];
            d = wave_sum(d);
            const double wv = tv * (c[k] + scale * d);
            for (int i = k + 1 + lane; i < m; i += 64) c[i] -= wv * scale * x[i];
            if (lane == 0) c[k] -= wv;
        }
        __syncthreads();
        for (int i = k + 1 + tid; i < m; i += BT_NT) x[i] *= scale;
        if (tid == 0) { x[k] = beta; tau[k] = tv; }
        __syncthreads();
    }
}

// C (m x ncol) <- Q C (trans = false) or Q^T C, Q = H_0 .. H_{k-1} from wg_qr.
__device__ void wg_apply_q(bool trans, int m, int k, const double *Qf, int ldq, const double *tau,
                           int ncol, double *C, int ldc) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int s = 0; s < k; ++s) {
        const int j = trans ? s : k - 1 - s;
        const double *v = Qf + (size_t)j * ldq;
        const double tj = tau[j];
        if (tj != 0.0) {
            for (int col = w; col < ncol; col += BT_W) {
                double *c = C + (size_t)col * ldc;
                double d = 0.0;
                for (int i = j + 1 + lane; i < m; i += 64) d += v[i] * c[i];
                d = tj * (wave_sum(d) + c[j]);
                for (int i = j + 1 + lane; i < m; i += 64) c[i] -= d * v[i];
                if (lane == 0) c[j] -= d;
            }
        }
        __syncthreads();
    }
}

// Businger-Golub pivots in precision T on a copy W (n x n, ld n) of A1
// (ld lda; only its upper triangle when `upper`, i.e. when A1 is the R1 of
// the tall QR with reflectors below the diagonal); ties go to the smallest
// column index.
template <typename T>
__device__ void wg_qrcp(int n, const double *A1, int lda, bool upper, T *W, T *nrm, int *piv,
                        double *red, int *ish) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int e = tid; e < n * n; e += BT_NT) {
        const int i = e % n, j = e / n;
        W[e] = (!upper || i <= j) ? (T)A1[(size_t)j * lda + i] : T(0);
    }
    __syncthreads();
    for (int j = w; j < n; j += BT_W) {
        T s = 0;
        for (int i = lane; i < n; i += 64) s += W[(size_t)j * n + i] * W[(size_t)j * n + i];
        s = wave_sum(s);
        if (lane == 0) nrm[j] = tsqrt(s);
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (w == 0) {
            T bv = T(-2);
            int bi = n;
            for (int j = lane; j < n; j += 64) {
                const T v = nrm[j];
                if (v > bv) { bv = v; bi = j; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const T ov = __shfl_xor(bv, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { ish[0] = bi; piv[k] = bi; }
        }
        __syncthreads();
        const int p = ish[0];
        const T *x = W + (size_t)p * n;
        T s = 0;
        for (int i = k + 1 + tid; i < n; i += BT_NT) s += x[i] * x[i];
        s = (T)bt_sum((double)s, red);
        const T x0 = x[k];
        T tv = 0, scale = 0;
        if (s != T(0)) {
            const T beta = -copysign(tsqrt(x0 * x0 + s), x0);
            tv = (beta - x0) / beta;
            scale = T(1) / (x0 - beta);
        }
        for (int j = w; j < n; j += BT_W) {
            if (j == p || nrm[j] < T(0)) continue;
            T *c = W + (size_t)j * n;
            T d = 0;
            for (int i = k + 1 + lane; i < n; i += 64) d += x[i] * c[i];
            d = wave_sum(d);
            const T wv = tv * (c[k] + scale * d);
            T ns = 0;
            for (int i = k + 1 + lane; i < n; i += 64) {
                const T v = c[i] - wv * scale * x[i];
                c[i] = v;
                ns += v * v;
            }
            ns = wave_sum(ns);
            if (lane == 0) { c[k] -= wv; nrm[j] = tsqrt(ns); }
        }
        __syncthreads();
        if (tid == 0) nrm[p] = T(-1);
        __syncthreads();
    }
}

// One-sided Jacobi (Algorithm 1) on the n columns of Y (rows x n, ld ldy),
// accumulating into V (n x n, ld ldv) when given; round-robin pair order,
// one wavefront per pair.  Angles and tests in FP64.  Returns the sweeps run;
// *conv = 1 if the last sweep rotated nothing.
template <typename T>
__device__ int wg_jacobi(int rows, int n, T *Y, int ldy, double *V, int ldv, double eps,
                         int maxsweep, int *conv, int *flag) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nn = n + (n & 1);
    const double eps2 = eps * eps;
    *conv = 0;
    int sw = 0;
    for (; sw < maxsweep; ++sw) {
        __syncthreads();
        if (tid == 0) *flag = 0;
        __syncthreads();
        for (int r = 0; r < nn - 1; ++r) {
            for (int k = w; k < nn / 2; k += BT_W) {
                int p, q;
                rr_slot(nn, r, k, &p, &q);
                if (q >= n) continue;
                T *yp = Y + (size_t)p * ldy, *yq = Y + (size_t)q * ldy;
                T a = 0, b = 0, g = 0;
                for (int i = lane; i < rows; i += 64) {
                    const T u = yp[i], v = yq[i];
                    a += u * u; b += v * v; g += u * v;
                }
                const double al = (double)wave_sum(a), be = (double)wave_sum(b);
                const double ga = (double)wave_sum(g);
                if (!(ga * ga > eps2 * al * be)) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double sg = zeta >= 0.0 ? 1.0 : -1.0;
                const double az = fabs(zeta);
                const double root = az > 1e150 ? az : sqrt(1.0 + az * az);
                const double t = sg / (az + root);
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                const T cT = (T)c, sT = (T)s;
                for (int i = lane; i < rows; i += 64) {
                    const T u = yp[i], v = yq[i];
                    yp[i] = cT * u - sT * v;
                    yq[i] = sT * u + cT * v;
                }
                if (V) {
                    double *vp = V + (size_t)p * ldv, *vq = V + (size_t)q * ldv;
                    for (int i = lane; i < n; i += 64) {
                        const double u = vp[i], v = vq[i];
                        vp[i] = c * u - s * v;
                        vq[i] = s * u + c * v;
                    }
                }
                if (lane == 0) *flag = 1;
            }
            __syncthreads();
        }
        if (*flag == 0) { *conv = 1; ++sw; break; }
    }
    return sw;
}

// Per-workgroup scratch, in doubles, for matrices up to M x N.
struct BtLayout {
    size_t abuf, a1p, rt, x, y, vacc, ulow, bm, ux, vx, w32, vec, total;
};
__host__ __device__ inline BtLayout bt_layout(int M, int N) {
    BtLayout L;
    const size_t nn = (size_t)N * N;
    size_t p = 0;
    L.abuf = p; p += (size_t)M * N;
    L.a1p = p; p += nn;
    L.rt = p; p += nn;
    L.x = p; p += nn;
    L.y = p; p += nn;
    L.vacc = p; p += nn;
    L.ulow = p; p += nn;
    L.bm = p; p += nn;
    L.ux = p; p += nn;
    L.vx = p; p += nn;
    L.w32 = p; p += (nn + 1) / 2;          // n x n floats
    L.vec = p; p += 12 * (size_t)N + 64;  // taus, sig, norms, piv, rank
    L.total = (p + 31) & ~(size_t)31;
    return L;
}

__global__ void bt_reset(int *counter) { *counter = 0; }

__global__ __launch_bounds__(BT_NT) void bt_svd(int batch, const BatchMeta *__restrict__ meta,
                                                const int *__restrict__ order, BatchParams prm,
                                                int M, int Nmax, const double *__restrict__ A_base,
                                                double *S_base, double *U_base, double *V_base,
                                                double *work, svd_batch_info *info, int *counter) {
    __shared__ double red[BT_W];
    __shared__ double As[BT_NT / 256][16][65];
    __shared__ double Bs[BT_NT / 256][16][65];
    __shared__ int ish[4];
    __shared__ int flag;
    __shared__ double dsh[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const BtLayout L = bt_layout(M, Nmax);
    double *base = work + (size_t)blockIdx.x * L.total;
    double *Ab = base + L.abuf, *A1P = base + L.a1p, *Rt = base + L.rt, *X = base + L.x;
    double *Y = base + L.y, *Vacc = base + L.vacc, *Ulow = base + L.ulow, *Bm = base + L.bm;
    double *UX = base + L.ux, *VX = base + L.vx;
    float *W32 = (float *)(base + L.w32);
    double *vec = base + L.vec;
    double *tau0 = vec, *tau1 = vec + Nmax, *tau2 = vec + 2 * Nmax, *tau3 = vec + 3 * Nmax;
    double *sig = vec + 4 * Nmax;
    float *nrm32 = (float *)(vec + 5 * Nmax);
    int *piv = (int *)(vec + 6 * Nmax), *rank = (int *)(vec + 7 * Nmax);

    for (;;) {
        if (tid == 0) ish[0] = atomicAdd(counter, 1);
        __syncthreads();
        const int qi = ish[0];
        __syncthreads();
        if (qi >= batch) break;
        const int jm = order[qi];
        const BatchMeta md = meta[jm];
        const int m = md.m, n = md.n;
        const double *A = A_base + md.offA;
        double *S = S_base + md.offS, *U = U_base + md.offA, *Vo = V_base + md.offV;

        // a0/a1: copy A; tall reduction A = Q0 R1
        for (int e = tid; e < m * n; e += BT_NT) Ab[e] = A[e];
        __syncthreads();
        if (m > n) wg_qr(m, n, Ab, m, tau0, red);
        // a2: FP32 pivots on A1 = upper triangle of Ab (ld m)
        const bool tall = m > n;
        wg_qrcp<float>(n, Ab, m, tall, W32, nrm32, piv, red, ish + 1);
        // a3: FP64 QR of A1 P
        for (int e = tid; e < n * n; e += BT_NT) {
            const int i = e % n, k = e / n, c = piv[k];
            A1P[e] = (!tall || i <= c) ? Ab[(size_t)c * m + i] : 0.0;
        }
        __syncthreads();
        wg_qr(n, n, A1P, n, tau1, red);
        // a4: R = L Q2 via the QR of R^T; X = L
        for (int e = tid; e < n * n; e += BT_NT) {
            const int i = e % n, j = e / n;
            Rt[e] = i >= j ? A1P[(size_t)i * n + j] : 0.0;
        }
        __syncthreads();
        wg_qr(n, n, Rt, n, tau2, red);
        for (int e = tid; e < n * n; e += BT_NT) {
            const int i = e % n, j = e / n;
            X[e] = i >= j ? Rt[(size_t)i * n + j] : 0.0;
        }
        __syncthreads();

        // a5: special cases of Section 3.5
        int branch = prm.branch;
        if (branch == SVD_BRANCH_AUTO) {
            // cond_R from the pivoted R, trailing small columns of X
            double mx = 0.0, mn = INFINITY;
            for (int i = tid; i < n; i += BT_NT) {
                const double d = fabs(A1P[(size_t)i * n + i]);
                mx = fmax(mx, d); mn = fmin(mn, d);
            }
            mx = wave_max(mx);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
            if (lane == 0) { red[w] = mx; }
            __syncthreads();
            if (tid == 0) { double a = 0; for (int q = 0; q < BT_W; ++q) a = fmax(a, red[q]); dsh[0] = a; }
            __syncthreads();
            if (lane == 0) red[w] = mn;
            __syncthreads();
            if (tid == 0) { double a = INFINITY; for (int q = 0; q < BT_W; ++q) a = fmin(a, red[q]); dsh[1] = a; }
            __syncthreads();
            const double cond = dsh[1] > 0.0 ? dsh[0] / dsh[1] : INFINITY;
            // column norms of X into sig (scratch)
            for (int j = w; j < n; j += BT_W) {
                double s2 = 0.0;
                for (int i = lane; i < n; i += 64) s2 += X[(size_t)j * n + i] * X[(size_t)j * n + i];
                s2 = wave_sum(s2);
                if (lane == 0) sig[j] = sqrt(s2);
            }
            __syncthreads();
            if (tid == 0) {
                double xm = 0.0;
                for (int j = 0; j < n; ++j) xm = fmax(xm, sig[j]);
                int ns = 0;
                for (int j = n - 1; j >= 0 && sig[j] <= prm.small_col_rel * xm; --j) ++ns;
                ish[2] = ns;
            }
            __syncthreads();
            const int nsmall = ish[2];
            bool skip = cond <= prm.tol_cond_coef * pow((double)n, 0.25) ||
                        nsmall >= (int)ceil(prm.small_col_frac * n);
            if (!skip) {
                // X_t = low(X) D^-1 (FP32 values), orth = max |X_t^T X_t - I|
                for (int j = w; j < n; j += BT_W) {
                    float s2 = 0.f;
                    for (int i = lane; i < n; i += 64) {
                        const float v = (float)X[(size_t)j * n + i];
                        s2 += v * v;
                    }
                    const float d = sqrtf(wave_sum(s2));
                    const float inv = d > 0.f ? 1.f / d : 0.f;
                    for (int i = lane; i < n; i += 64)
                        Ulow[(size_t)j * n + i] = (double)((float)X[(size_t)j * n + i] * inv);
                }
                __syncthreads();
                wg_gemm<true, false, BT_NT>(n, n, n, Ulow, n, Ulow, n, Bm, n, false, As, Bs);
                double dm = 0.0;
                for (int e = tid; e < n * n; e += BT_NT)
                    dm = fmax(dm, fabs(Bm[e] - ((e % n) == (e / n) ? 1.0 : 0.0)));
                dm = wave_max(dm);
                if (lane == 0) red[w] = dm;
                __syncthreads();
                double om = 0.0;
                for (int q = 0; q < BT_W; ++q) om = fmax(om, red[q]);
                __syncthreads();
                if (om <= prm.tol_orth) skip = true;
            }
            branch = skip ? SVD_BRANCH_SKIP : SVD_BRANCH_LOW;
        }

        int sweeps_low = 0, conv_low = 1;
        for (int e = tid; e < n * n; e += BT_NT) Vacc[e] = ((e % n) == (e / n)) ? 1.0 : 0.0;
        if (branch == SVD_BRANCH_LOW) {
            // a6: FP32 one-sided Jacobi on low(X), no V
            for (int e = tid; e < n * n; e += BT_NT) W32[e] = (float)X[e];
            __syncthreads();
            const double el = prm.eps_low_fixed > 0 ? prm.eps_low_fixed : prm.eps_low_coef * sqrt((double)n);
            sweeps_low = wg_jacobi<float>(n, n, W32, n, nullptr, n, el, prm.maxsweep_low, &ish[3], &flag);
            conv_low = ish[3];
            // U_low = Y_low D^-1 lifted to FP64
            for (int j = w; j < n; j += BT_W) {
                float s2 = 0.f;
                for (int i = lane; i < n; i += 64) s2 += W32[(size_t)j * n + i] * W32[(size_t)j * n + i];
                const float d = sqrtf(wave_sum(s2));
                for (int i = lane; i < n; i += 64)
                    Ulow[(size_t)j * n + i] = d > 0.f ? (double)(W32[(size_t)j * n + i] / d) : 0.0;
            }
            __syncthreads();
            // a7: X^T U_low = Q R2, Q formed explicitly, Y = X Q
            wg_gemm<true, false, BT_NT>(n, n, n, X, n, Ulow, n, Bm, n, false, As, Bs);
            wg_qr(n, n, Bm, n, tau3, red);
            wg_apply_q(false, n, n, Bm, n, tau3, n, Vacc, n);
            wg_gemm<false, false, BT_NT>(n, n, n, X, n, Vacc, n, Y, n, false, As, Bs);
        } else {
            for (int e = tid; e < n * n; e += BT_NT) Y[e] = X[e];
            __syncthreads();
        }

        // a8: FP64 one-sided Jacobi with V accumulated from Q
        const double ew = prm.eps_work_fixed > 0 ? prm.eps_work_fixed : prm.eps_work_coef * sqrt((double)n);
        const int sweeps_work = wg_jacobi<double>(n, n, Y, n, Vacc, n, ew, prm.maxsweep_work, &ish[3], &flag);
        const int conv_work = ish[3];

        // a9: sigma, stable descending order, U_X, V_X
        for (int j = w; j < n; j += BT_W) {
            double s2 = 0.0;
            for (int i = lane; i < n; i += 64) s2 += Y[(size_t)j * n + i] * Y[(size_t)j * n + i];
            s2 = wave_sum(s2);
            if (lane == 0) sig[j] = sqrt(s2);
        }
        __syncthreads();
        for (int j = tid; j < n; j += BT_NT) {
            const double sj = sig[j];
            int rk = 0;
            for (int i = 0; i < n; ++i) rk += (sig[i] > sj) || (sig[i] == sj && i < j);
            rank[j] = rk;
        }
        __syncthreads();
        int nzero = 0;
        for (int j = w; j < n; j += BT_W) {
            const int d = rank[j];
            const double sj = sig[j];
            const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
            for (int i = lane; i < n; i += 64) {
                UX[(size_t)d * n + i] = Y[(size_t)j * n + i] * inv;
                VX[(size_t)d * n + i] = Vacc[(size_t)j * n + i];
            }
            if (lane == 0) { S[d] = sj; if (sj == 0.0) nzero = 1; }
        }
        __syncthreads();
        // U = Q0 Q1 U_X
        wg_apply_q(false, n, n, A1P, n, tau1, n, UX, n);
        for (int e = tid; e < m * n; e += BT_NT) {
            const int i = e % m, j = e / m;
            U[e] = i < n ? UX[(size_t)j * n + i] : 0.0;
        }
        __syncthreads();
        if (m > n) wg_apply_q(false, m, n, Ab, m, tau0, n, U, m);
        // V = P Q2^T V_X
        wg_apply_q(false, n, n, Rt, n, tau2, n, VX, n);
        for (int e = tid; e < n * n; e += BT_NT) {
            const int k = e % n, j = e / n;
            Vo[(size_t)j * n + piv[k]] = VX[e];
        }
        __syncthreads();
        if (prm.sign_normalize) {
            for (int i = w; i < n; i += BT_W) {
                double best = -1.0;
                int bk = n;
                for (int k = lane; k < n; k += 64) {
                    const double a = fabs(Vo[(size_t)i * n + k]);
                    if (a > best) { best = a; bk = k; }
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const double ob = __shfl_xor(best, o, 64);
                    const int okk = __shfl_xor(bk, o, 64);
                    if (ob > best || (ob == best && okk < bk)) { best = ob; bk = okk; }
                }
                const bool neg = Vo[(size_t)i * n + bk] < 0.0;
                if (neg) {
                    for (int k = lane; k < n; k += 64) Vo[(size_t)i * n + k] = -Vo[(size_t)i * n + k];
                    for (int k = lane; k < m; k += 64) U[(size_t)i * m + k] = -U[(size_t)i * m + k];
                }
            }
        }
        // per-matrix result
        nzero = block_or<BT_NT>(nzero, (int *)red);
        if (tid == 0) {
            svd_batch_info r;
            r.status = SVD_OK;
            if (!conv_work || (branch == SVD_BRANCH_LOW && !conv_low)) r.status = SVD_WARN_NOCONV;
            if (nzero) r.status = SVD_WARN_RANK_DEFICIENT;
            r.branch_taken = branch;
            r.sweeps_low = sweeps_low;
            r.sweeps_work = sweeps_work;
            info[jm] = r;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- plan
struct BatchPlan {
    int batch = 0, maxm = 0, maxn = 0, nwg = 0;
    BatchMeta *d_meta = nullptr;   // device copy of the metadata
    int *d_order = nullptr;        // device copy of the LPT order
    BatchParams prm{};
    size_t work_bytes = 0;
    std::mutex mu;                 // guards the captured graph
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    const void *key[7] = {nullptr};
};

} // namespace mpj

using namespace mpj;

extern "C" int svd_batched_plan_create(int batch, const int *h_m, const int *h_n,
                                       const svd_opts *op, void **plan, size_t *work_bytes) {
    if (batch < 0) return -1;
    if (batch > 0 && (!h_m || !h_n)) return -2;
    if (!plan) return -5;
    svd_opts o;
    if (op) o = *op; else svd_default_opts(&o, 1);
    BatchPlan *P = new (std::nothrow) BatchPlan();
    if (!P) return SVD_ERR_HIP;
    std::vector<BatchMeta> meta(batch);
    long long a = 0, sofs = 0, v = 0;
    for (int j = 0; j < batch; ++j) {
        const int m = h_m[j], n = h_n[j];
        if (n < 1 || m < n || m > BT_MAXN) { delete P; return -3; }
        meta[j] = BatchMeta{m, n, a, sofs, v};
        a += (long long)m * n; sofs += n; v += (long long)n * n;
        P->maxm = std::max(P->maxm, m);
        P->maxn = std::max(P->maxn, n);
    }
    // longest-processing-time first: cost ~ n^3 (sweeps) + m n^2 (tall QR)
    std::vector<int> order(batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const double cx = (double)meta[x].n * meta[x].n * (meta[x].n * 8.0 + meta[x].m);
        const double cy = (double)meta[y].n * meta[y].n * (meta[y].n * 8.0 + meta[y].m);
        return cx > cy;
    });
    P->batch = batch;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete P;
        return SVD_ERR_HIP;
    }
    int wpc = tuned_wg_per_cu(P->maxn);
    if (wpc < 1) wpc = 2;
    P->nwg = std::max(1, std::min(batch, wpc * ncu));
    P->prm.tol_orth = o.tol_orth;
    P->prm.tol_cond_coef = o.tol_cond_coef;
    P->prm.small_col_rel = o.small_col_rel;
    P->prm.small_col_frac = o.small_col_frac;
    P->prm.eps_low_coef = ldexp(1.0, -24);
    P->prm.eps_work_coef = ldexp(1.0, -53);
    P->prm.eps_low_fixed = o.eps_low;
    P->prm.eps_work_fixed = o.eps_work;
    P->prm.maxsweep_low = o.maxsweep_low;
    P->prm.maxsweep_work = o.maxsweep_work;
    P->prm.branch = o.branch;
    P->prm.sign_normalize = o.sign_normalize;
    if (batch > 0) {
        const BtLayout L = bt_layout(P->maxm, P->maxn);
        P->work_bytes = (size_t)P->nwg * L.total * sizeof(double) + 256;
        // the plan's own device metadata (the compute call allocates nothing)
        if (hipMalloc(&P->d_meta, sizeof(BatchMeta) * batch) != hipSuccess ||
            hipMalloc(&P->d_order, sizeof(int) * batch) != hipSuccess ||
            hipMemcpy(P->d_meta, meta.data(), sizeof(BatchMeta) * batch, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(P->d_order, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(P->d_meta);
            (void)hipFree(P->d_order);
            delete P;
            return SVD_ERR_HIP;
        }
    } else {
        P->work_bytes = 256;
    }
    *plan = P;
    if (work_bytes) *work_bytes = P->work_bytes;
    return 0;
}

extern "C" void svd_batched_plan_destroy(void *plan) {
    BatchPlan *P = (BatchPlan *)plan;
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->cap) (void)hipStreamDestroy(P->cap);
    (void)hipFree(P->d_meta);
    (void)hipFree(P->d_order);
    delete P;
}

extern "C" int svd_batched(void *plan, const double *A_base, double *S_base, double *U_base,
                           double *V_base, void *work, size_t work_bytes, svd_batch_info *info,
                           void *stream) {
    BatchPlan *P = (BatchPlan *)plan;
    if (!P) return -1;
    if (P->batch == 0) return 0;
    if (!A_base) return -2;
    if (!S_base) return -3;
    if (!U_base) return -4;
    if (!V_base) return -5;
    if (!work) return -6;
    if (work_bytes < P->work_bytes) return -7;
    if (!info) return -8;
    hipStream_t s = (hipStream_t)stream;
    double *wk = (double *)work;
    // the queue counter sits past the per-workgroup slices
    const BtLayout L = bt_layout(P->maxm, P->maxn);
    int *counter = (int *)(wk + (size_t)P->nwg * L.total);
    std::lock_guard<std::mutex> lock(P->mu);
    const void *key[7] = {A_base, S_base, U_base, V_base, work, info, nullptr};
    bool same = P->exec != nullptr;
    for (int i = 0; i < 6 && same; ++i) same = P->key[i] == key[i];
    if (!same) {
        // capture [reset queue; persistent kernel] once per buffer set; the
        // counter is cleared by a kernel, not a memset node
        if (P->exec) { (void)hipGraphExecDestroy(P->exec); P->exec = nullptr; }
        if (!P->cap && hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess)
            return SVD_ERR_HIP;
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return SVD_ERR_HIP;
        hipLaunchKernelGGL(bt_reset, dim3(1), dim3(1), 0, P->cap, counter);
        hipLaunchKernelGGL(bt_svd, dim3(P->nwg), dim3(BT_NT), 0, P->cap, P->batch,
                           (const BatchMeta *)P->d_meta, (const int *)P->d_order, P->prm, P->maxm,
                           P->maxn, A_base, S_base, U_base, V_base, wk, info, counter);
        if (hipStreamEndCapture(P->cap, &g) != hipSuccess || !g) return SVD_ERR_HIP;
        hipError_t e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) { P->exec = nullptr; return SVD_ERR_HIP; }
        for (int i = 0; i < 7; ++i) P->key[i] = key[i];
    }
    if (hipGraphLaunch(P->exec, s) != hipSuccess) return SVD_ERR_HIP;
    return 0;
}
