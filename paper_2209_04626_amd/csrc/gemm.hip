// Dense GEMM on the matrix cores (MFMA 16x16x4, FP64 or FP32), used for the
// dense contractions of the path: blocked Householder updates (Section 3.1),
// the switch products X^T U_low and X Q (Section 3.3), the back-transforms
// U = Q0 Q1 U_X, V = P Q2^T V_X, and the FP32 orthogonality test
// max|X_t^T X_t - I| of Section 3.5.
//
// Tiling: 64 x 64 (or 32 x 64) output tile per 256-thread workgroup, K
// staged through LDS in slices of 32 with the next slice prefetched into
// registers.  Split-K writes partial products to scratch and a second kernel
// sums them in a fixed order (deterministic).
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace mpj {

constexpr int GBN = 64, GBK = 32;

// EPI_MAXDEV and EPI_COLMAX take C = A^T A (a Gram matrix, symmetric): only
// the tiles on or above the block diagonal are formed.
enum { EPI_STORE = 0, EPI_PART = 1, EPI_MAXDEV = 2, EPI_COLMAX = 3 };

// BM x 64 output tile per 256-thread workgroup (BM = 64: 2 x 2 wavefronts of
// 32 x 32; BM = 32, for the 32-row products of the blocked Householder
// updates: 1 x 4 wavefronts of 32 x 16).  K advances in slices of 32: the
// next slice is loaded into registers while the matrix cores work on the
// current one from LDS.
template <typename T, bool TA, bool TB, int EPI, int BM>
__global__ __launch_bounds__(256) void gemm_kernel(
    int M, int N, int K, T alpha, const T *__restrict__ A, int lda,
    const T *__restrict__ B, int ldb, T beta, T *C, int ldc, int kchunk,
    T *part, float *maxdev) {
    constexpr int WN = BM == 64 ? 2 : 4;           // wavefronts along N
    constexpr int TI = 2, TJ = BM == 64 ? 2 : 1;   // MFMA tiles per wavefront
    constexpr int PA = BM * GBK / 256, PB = GBK * GBN / 256;
    // LDS: the K slices of A and B, reused after the K loop for the output
    // tile so that C is read and written along its columns
    constexpr size_t SZ_AB = sizeof(T) * (GBK * (BM + 1) + GBK * (GBN + 1));
    constexpr size_t SZ_C = sizeof(T) * GBN * (BM + 1);
    __shared__ __align__(16) char smem[SZ_AB > SZ_C ? SZ_AB : SZ_C];
    T (*As)[BM + 1] = reinterpret_cast<T (*)[BM + 1]>(smem);
    T (*Bs)[GBN + 1] = reinterpret_cast<T (*)[GBN + 1]>(smem + sizeof(T) * GBK * (BM + 1));
    T (*Cs)[BM + 1] = reinterpret_cast<T (*)[BM + 1]>(smem);
    __shared__ float red[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / WN, wn = w % WN;
    const int i0 = blockIdx.x * BM, j0 = blockIdx.y * GBN;
    if ((EPI == EPI_MAXDEV || EPI == EPI_COLMAX) && i0 > j0) return;   // the mirror tile covers it
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    typedef typename acc4<T>::type V4;
    V4 acc[TI][TJ];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b) acc[a][b] = V4{0, 0, 0, 0};

    T ra[PA], rb[PB];
    auto load = [&](int k0) {
#pragma unroll
        for (int rep = 0; rep < PA; ++rep) {
            const int e = tid + 256 * rep;
            int i, k;
            if (!TA) { i = e % BM; k = e / BM; } else { k = e % GBK; i = e / GBK; }
            const int gi = i0 + i, gk = k0 + k;
            T v = 0;
            if (gi < M && gk < kend)
                v = TA ? A[(size_t)gi * lda + gk] : A[(size_t)gk * lda + gi];
            ra[rep] = v;
        }
#pragma unroll
        for (int rep = 0; rep < PB; ++rep) {
            const int e = tid + 256 * rep;
            int j, k;
            if (!TB) { k = e % GBK; j = e / GBK; } else { j = e % GBN; k = e / GBN; }
            const int gj = j0 + j, gk = k0 + k;
            T v = 0;
            if (gj < N && gk < kend)
                v = TB ? B[(size_t)gk * ldb + gj] : B[(size_t)gj * ldb + gk];
            rb[rep] = v;
        }
    };
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += GBK) {
        __syncthreads();
#pragma unroll
        for (int rep = 0; rep < PA; ++rep) {
            const int e = tid + 256 * rep;
            int i, k;
            if (!TA) { i = e % BM; k = e / BM; } else { k = e % GBK; i = e / GBK; }
            As[k][i] = ra[rep];
        }
#pragma unroll
        for (int rep = 0; rep < PB; ++rep) {
            const int e = tid + 256 * rep;
            int j, k;
            if (!TB) { k = e % GBK; j = e / GBK; } else { j = e % GBN; k = e / GBN; }
            Bs[k][j] = rb[rep];
        }
        __syncthreads();
        if (k0 + GBK < kend) load(k0 + GBK);
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 4) {
            T a[TI], b[TJ];
#pragma unroll
            for (int t = 0; t < TI; ++t) a[t] = As[kk + lane / 16][wm * 32 + t * 16 + lane % 16];
#pragma unroll
            for (int t = 0; t < TJ; ++t) b[t] = Bs[kk + lane / 16][wn * 16 * TJ + t * 16 + lane % 16];
#pragma unroll
            for (int ti = 0; ti < TI; ++ti)
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = mfma16(a[ti], b[tj], acc[ti][tj]);
        }
    }

    float dmax = 0.f;
    if (EPI == EPI_MAXDEV) {
#pragma unroll
        for (int ti = 0; ti < TI; ++ti)
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = i0 + wm * 32 + ti * 16 + mfma_row<T>(lane, r);
                    const int gj = j0 + wn * 16 * TJ + tj * 16 + lane % 16;
                    if (gi < M && gj < N) {
                        const T dv = alpha * acc[ti][tj][r] - (gi == gj ? T(1) : T(0));
                        float d = (float)(dv < T(0) ? -dv : dv);
                        // fmaxf drops a NaN operand: a NaN entry (a NaN in X)
                        // must read as the largest deviation instead
                        if (d != d) d = INFINITY;
                        dmax = fmaxf(dmax, d);
                    }
                }
    } else {
        __syncthreads();   // the last slice's reads of As / Bs are done
#pragma unroll
        for (int ti = 0; ti < TI; ++ti)
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Cs[wn * 16 * TJ + tj * 16 + lane % 16][wm * 32 + ti * 16 + mfma_row<T>(lane, r)] =
                        acc[ti][tj][r];
        __syncthreads();
        if constexpr (EPI == EPI_COLMAX) {
            // largest off-diagonal |c_ij| of each column j (and, through the
            // symmetry, of each row i) of the tile, into maxdev[] (zeroed
            // beforehand; non-negative floats order as their bit patterns).
            // A NaN entry is passed over, as fmaxf does.
            if (tid < 2 * GBN) {
                const bool colw = tid < GBN;
                const int x = tid % GBN;
                const int gx = colw ? j0 + x : i0 + x;
                float m = 0.f;
                if (gx < (colw ? N : M)) {
                    for (int y = 0; y < GBN; ++y) {
                        const int gi = colw ? i0 + y : gx, gj = colw ? gx : j0 + y;
                        if (gi < M && gj < N && gi != gj) {
                            const float d = (float)fabs(alpha * (colw ? Cs[x][y] : Cs[y][x]));
                            m = fmaxf(m, d);
                        }
                    }
                    atomicMax((unsigned int *)maxdev + gx, __float_as_uint(m));
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < BM * GBN / 256; ++q) {
                const int e = tid + 256 * q;
                const int i = e % BM, j = e / BM;
                const int gi = i0 + i, gj = j0 + j;
                if (gi < M && gj < N) {
                    const T v = alpha * Cs[j][i];
                    if (EPI == EPI_STORE) {
                        T *c = C + (size_t)gj * ldc + gi;
                        *c = (beta == T(0)) ? v : v + beta * (*c);
                    } else {
                        part[(size_t)blockIdx.z * M * N + (size_t)gj * M + gi] = v;
                    }
                }
            }
        }
    }
    if (EPI == EPI_MAXDEV) {
        dmax = wave_max(dmax);
        if (lane == 0) red[w] = dmax;
        __syncthreads();
        if (tid == 0) {
            const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
            atomicMax((unsigned int *)maxdev, __float_as_uint(m));
        }
    }
}

// FP64 products with a large output (C = alpha op(A) op(B) + beta C): a
// 128 x 128 tile per 256-thread workgroup, 2 x 2 wavefronts of 64 x 64 (4 x 4
// MFMA tiles each), so that each value staged in LDS feeds four times the
// products of the 64 x 64 kernel.  K advances in slices of 16, double-buffered
// in LDS: the next slice is loaded into registers while the matrix cores work
// on the current one, then written to the other buffer (one barrier per
// slice).  The operands go into the MFMA swapped (it forms the tile of C^T =
// op(B)^T op(A)^T), which leaves lane l of each 16 x 16 tile holding rows
// l % 16 of four columns of C: reads and writes of C cover 128 contiguous
// bytes of a column per 16 lanes, with no staging.
constexpr int G2M = 128, G2K = 16, G2LD = G2M + 1;
template <bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void gemm128_kernel(int M, int N, int K, double alpha,
                                                         const double *__restrict__ A, int lda,
                                                         const double *__restrict__ B, int ldb,
                                                         double beta, double *C, int ldc) {
    __shared__ double As[2][G2K][G2LD];
    __shared__ double Bs[2][G2K][G2LD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int i0 = blockIdx.x * G2M, j0 = blockIdx.y * G2M;
    constexpr int PL = G2M * G2K / 256;      // values of each operand per thread and slice
    double ra[PL], rb[PL];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PL; ++u) {
            int i, k;
            if (!TA) { i = tid % G2M; k = tid / G2M + 2 * u; } else { k = tid % G2K; i = tid / G2K + 16 * u; }
            const int gi = i0 + i, gk = k0 + k;
            ra[u] = (gi < M && gk < K) ? (TA ? A[(size_t)gi * lda + gk] : A[(size_t)gk * lda + gi]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PL; ++u) {
            int j, k;
            if (TB) { j = tid % G2M; k = tid / G2M + 2 * u; } else { k = tid % G2K; j = tid / G2K + 16 * u; }
            const int gj = j0 + j, gk = k0 + k;
            rb[u] = (gj < N && gk < K) ? (TB ? B[(size_t)gk * ldb + gj] : B[(size_t)gj * ldb + gk]) : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < PL; ++u) {
            int i, k;
            if (!TA) { i = tid % G2M; k = tid / G2M + 2 * u; } else { k = tid % G2K; i = tid / G2K + 16 * u; }
            As[buf][k][i] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < PL; ++u) {
            int j, k;
            if (TB) { j = tid % G2M; k = tid / G2M + 2 * u; } else { k = tid % G2K; j = tid / G2K + 16 * u; }
            Bs[buf][k][j] = rb[u];
        }
    };
    dbl4 acc[4][4];   // [tile along i][tile along j]
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = dbl4{0, 0, 0, 0};
    const int ns = cdiv(K, G2K);
    load(0);
    store(0);
    __syncthreads();
    for (int sl = 0; sl < ns; ++sl) {
        const int cur = sl & 1;
        if (sl + 1 < ns) load((sl + 1) * G2K);
#pragma unroll
        for (int kk = 0; kk < G2K; kk += 4) {
            double xa[4], xb[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                xa[t] = As[cur][kk + lane / 16][wm * 64 + 16 * t + lane % 16];
                xb[t] = Bs[cur][kk + lane / 16][wn * 64 + 16 * t + lane % 16];
            }
#pragma unroll
            for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = mfma16(xb[tj], xa[ti], acc[ti][tj]);
        }
        if (sl + 1 < ns) store(cur ^ 1);
        __syncthreads();
    }
    // lane l, element r of tile (ti, tj): C(i0 + 64 wm + 16 ti + l % 16, j0 + 64 wn + 16 tj + l / 16 + 4 r)
    const int gi_l = i0 + wm * 64 + lane % 16;
    const bool beta0 = beta == 0.0;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti) {
        const int gi = gi_l + 16 * ti;
        double cv[4][4];
        if (!beta0) {
#pragma unroll
            for (int tj = 0; tj < 4; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gj = j0 + wn * 64 + 16 * tj + lane / 16 + 4 * r;
                    cv[tj][r] = (gi < M && gj < N) ? C[(size_t)gj * ldc + gi] : 0.0;
                }
        }
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = j0 + wn * 64 + 16 * tj + lane / 16 + 4 * r;
                if (gi < M && gj < N) {
                    const double v = alpha * acc[ti][tj][r];
                    C[(size_t)gj * ldc + gi] = beta0 ? v : v + beta * cv[tj][r];
                }
            }
    }
}

// C = sum_z part[z] + beta C, summed in z order.
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce(int M, int N, int nz,
                                                     const T *__restrict__ part, T beta,
                                                     T *C, int ldc) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t MN = (size_t)M * N;
    if (e >= MN) return;
    const int i = (int)(e % M), j = (int)(e / M);
    T s = 0;
    for (int z = 0; z < nz; ++z) s += part[z * MN + e];
    T *c = C + (size_t)j * ldc + i;
    *c = (beta == T(0)) ? s : s + beta * (*c);
}

template <typename T, bool TA, bool TB, int BM>
static void gemm_launch_bm(hipStream_t s, int M, int N, int K, T alpha, const T *A, int lda,
                           const T *B, int ldb, T beta, T *C, int ldc, T *split,
                           size_t split_elems) {
    const int tm = cdiv(M, BM), tn = cdiv(N, GBN);
    const int tiles = tm * tn;
    int nz = 1;
    if (K <= 0) {
        // C = beta C
        hipLaunchKernelGGL((gemm_kernel<T, TA, TB, EPI_STORE, BM>), dim3(tm, tn, 1), dim3(256), 0, s,
                           M, N, 0, alpha, A, lda, B, ldb, beta, C, ldc, GBK, (T *)nullptr,
                           (float *)nullptr);
        return;
    }
    if (split && tiles < 512 && K >= 512) {
        nz = min(cdiv(K, 256), cdiv(1024, tiles));
        const size_t cap = split_elems / ((size_t)M * N);
        if ((size_t)nz > cap) nz = (int)cap;
        if (nz < 2) nz = 1;
    }
    int kchunk = cdiv(cdiv(K, nz), GBK) * GBK;
    nz = cdiv(K, kchunk);
    if constexpr (std::is_same<T, double>::value && BM == 64) {
        // enough 128 x 128 tiles to give every compute unit one
        if (nz == 1 && (long long)cdiv(M, G2M) * cdiv(N, G2M) >= 240) {
            hipLaunchKernelGGL((gemm128_kernel<TA, TB>), dim3(cdiv(M, G2M), cdiv(N, G2M)), dim3(256), 0, s,
                               M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
            return;
        }
    }
    if (nz == 1) {
        hipLaunchKernelGGL((gemm_kernel<T, TA, TB, EPI_STORE, BM>), dim3(tm, tn, 1), dim3(256), 0, s,
                           M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, (T *)nullptr,
                           (float *)nullptr);
    } else {
        hipLaunchKernelGGL((gemm_kernel<T, TA, TB, EPI_PART, BM>), dim3(tm, tn, nz), dim3(256), 0, s,
                           M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, split,
                           (float *)nullptr);
        const size_t MN = (size_t)M * N;
        hipLaunchKernelGGL((splitk_reduce<T>), dim3((unsigned)cdivl((long long)MN, 256)), dim3(256), 0, s,
                           M, N, nz, split, beta, C, ldc);
    }
}

template <typename T, bool TA, bool TB>
static void gemm_launch(hipStream_t s, int M, int N, int K, T alpha, const T *A, int lda,
                        const T *B, int ldb, T beta, T *C, int ldc, T *split,
                        size_t split_elems) {
    if (M <= 0 || N <= 0) return;
    if (M <= 32)
        gemm_launch_bm<T, TA, TB, 32>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, split, split_elems);
    else
        gemm_launch_bm<T, TA, TB, 64>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, split, split_elems);
}

template <typename T>
void gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, T alpha, const T *A, int lda,
          const T *B, int ldb, T beta, T *C, int ldc, T *split, size_t split_elems,
          KernelClock *kc) {
    // algorithmic work: 2MNK flops; A, B read once, C written (and read
    // when beta != 0)
    if (kc)
        kc->begin(s, 8, ((double)M * K + (double)K * N + (beta == T(0) ? 1.0 : 2.0) * M * N) * sizeof(T),
                  2.0 * M * N * K);
    if (!ta && !tb) gemm_launch<T, false, false>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, split, split_elems);
    else if (ta && !tb) gemm_launch<T, true, false>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, split, split_elems);
    else if (!ta && tb) gemm_launch<T, false, true>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, split, split_elems);
    else gemm_launch<T, true, true>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, split, split_elems);
    if (kc) kc->end(s);
}

template void gemm<double>(hipStream_t, bool, bool, int, int, int, double, const double *, int,
                           const double *, int, double, double *, int, double *, size_t,
                           KernelClock *);
template void gemm<float>(hipStream_t, bool, bool, int, int, int, float, const float *, int,
                          const float *, int, float, float *, int, float *, size_t, KernelClock *);

void gemm_orth_maxdev(hipStream_t s, int n, const float *X, int ldx, float *maxdev) {
    if (n <= 0) return;
    const int t = cdiv(n, 64);
    hipLaunchKernelGGL((gemm_kernel<float, true, false, EPI_MAXDEV, 64>), dim3(t, t, 1), dim3(256), 0, s,
                       n, n, n, 1.0f, X, ldx, X, ldx, 0.0f, (float *)nullptr, n, cdiv(n, GBK) * GBK,
                       (float *)nullptr, maxdev);
}

// Largest off-diagonal |c_ij| of each column of C = X^T X (n x n, FP64
// columns), into dev[0 .. n-1] (FP32), without storing C.
__global__ void k_zero_f32(int n, float *p) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0.f;
}
void gram_colmax_offdiag64(hipStream_t s, int n, const double *X, int ldx, float *dev) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_f32, dim3(cdiv(n, 256)), dim3(256), 0, s, n, dev);
    const int t = cdiv(n, 64);
    hipLaunchKernelGGL((gemm_kernel<double, true, false, EPI_COLMAX, 64>), dim3(t, t, 1), dim3(256), 0,
                       s, n, n, n, 1.0, X, ldx, X, ldx, 0.0, (double *)nullptr, n, cdiv(n, GBK) * GBK,
                       (double *)nullptr, dev);
}

// The same for FP64 columns (the deviation is formed in FP64, its maximum
// kept in FP32).
void gemm_orth_maxdev64(hipStream_t s, int n, const double *X, int ldx, float *maxdev) {
    if (n <= 0) return;
    const int t = cdiv(n, 64);
    hipLaunchKernelGGL((gemm_kernel<double, true, false, EPI_MAXDEV, 64>), dim3(t, t, 1), dim3(256), 0,
                       s, n, n, n, 1.0, X, ldx, X, ldx, 0.0, (double *)nullptr, n, cdiv(n, GBK) * GBK,
                       (double *)nullptr, maxdev);
}

} // namespace mpj
