// Workgroup-level FP64 GEMM on the matrix cores, used by kernels that run a
// whole small problem inside one workgroup (the SVD adjoint, the batched
// SVD): 64 x 64 output tiles, 4 wavefronts of 2 x 2 MFMA tiles per tile, K
// staged through LDS in slices of 16.
#pragma once
#include "common.hpp"

namespace mpj {

constexpr int WG_NT = 256;

// C (M x N) = op(A) op(B) (+ C when accumulate).  NT threads in groups of
// four wavefronts; each group computes its own 64 x 64 output tiles (tile
// g, g + NT/256, ...) and stages its K slices in As[g], Bs[g] (LDS).
template <bool TA, bool TB, int NT = WG_NT>
__device__ void wg_gemm(int M, int N, int K, const double *A, int lda, const double *B, int ldb,
                        double *C, int ldc, bool accumulate, double (*As)[16][65],
                        double (*Bs)[16][65]) {
    constexpr int NG = NT / 256;
    static_assert(NG * 256 == NT, "groups of 256 threads");
    const int tid = threadIdx.x, g = tid / 256, gt = tid % 256, lane = tid & 63, w = gt >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int tm = (M + 63) / 64, tn = (N + 63) / 64, ntile = tm * tn;
    for (int t0 = 0; t0 < ntile; t0 += NG) {
        const int tile = t0 + g;
        const bool act = tile < ntile;
        const int i0 = act ? (tile % tm) * 64 : 0, j0 = act ? (tile / tm) * 64 : 0;
        dbl4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0, 0, 0, 0};
        for (int k0 = 0; k0 < K; k0 += 16) {
            for (int e = gt; e < 64 * 16; e += 256) {
                int i, k;
                if (!TA) { i = e % 64; k = e / 64; } else { k = e % 16; i = e / 16; }
                const int gi = i0 + i, gk = k0 + k;
                double v = 0.0;
                if (act && gi < M && gk < K) v = TA ? A[(size_t)gi * lda + gk] : A[(size_t)gk * lda + gi];
                As[g][k][i] = v;
            }
            for (int e = gt; e < 64 * 16; e += 256) {
                int j, k;
                if (!TB) { k = e % 16; j = e / 16; } else { j = e % 64; k = e / 64; }
                const int gj = j0 + j, gk = k0 + k;
                double v = 0.0;
                if (act && gj < N && gk < K) v = TB ? B[(size_t)gk * ldb + gj] : B[(size_t)gj * ldb + gk];
                Bs[g][k][j] = v;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                double a[2], b[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    a[t] = As[g][kk + lane / 16][wm * 32 + t * 16 + lane % 16];
                    b[t] = Bs[g][kk + lane / 16][wn * 32 + t * 16 + lane % 16];
                }
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mfma16(a[ti], b[tj], acc[ti][tj]);
            }
            __syncthreads();
        }
        if (act) {
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int gi = i0 + wm * 32 + ti * 16 + mfma_row<double>(lane, r);
                        const int gj = j0 + wn * 32 + tj * 16 + lane % 16;
                        if (gi < M && gj < N) {
                            double *c = C + (size_t)gj * ldc + gi;
                            *c = accumulate ? *c + acc[ti][tj][r] : acc[ti][tj][r];
                        }
                    }
        }
    }
    __syncthreads();
}


} // namespace mpj
