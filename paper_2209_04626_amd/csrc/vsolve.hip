// Right singular vectors without accumulated rotations (Section 3.4).
//
// After the FP64 sweeps have run on Y without V, Y = X V_X holds U_X Sigma,
// so V_X = X^{-1} Y: one triangular solve with the lower triangular X = L of
// the LQ step.  Writing L = D_r Z_r (row scaling D_r), the solve's error
// depends on the conditioning of Z_r, not of L (Section 3.1), which the
// QRCP + LQ preconditioning keeps small.  The caller checks the result's
// orthogonality and falls back to the QR of X^T U_X followed by sweeps with
// accumulation when it is not good enough.
#include "../../include/mpjsvd.h"
#include "common.hpp"
#include "internal.hpp"

namespace mpj {

constexpr int TRSM_NB = 64;   // rows per diagonal block

// B(r0 : r0 + kb, c) <- L_kk^{-1} B(r0 : r0 + kb, c) for the kb x kb lower
// triangular diagonal block L_kk (kb <= TB): one lane per right-hand side
// column, the column in registers, the block in LDS (read as broadcasts).
// Column-oriented forward substitution: after z_l is final, every later z_i
// takes z_i - L_il z_l, so each lane has TB - l independent updates in flight;
// z_l itself is scaled by 1 / l_ll, formed once per block.  The block of B
// goes through LDS so that its loads and stores run along the columns (lane =
// row), every load of a lane in flight together.
template <int TB>
__global__ __launch_bounds__(64) void k_trsm_diag(int kb, int nrhs, const double *L, int ldl,
                                                  double *B, int ldb) {
    static_assert(TB == 64, "one lane per row of the block");
    __shared__ double Ls[TB][TB];
    __shared__ double Bs[TB][TB + 1];    // [column][row]
    __shared__ double rinv[TB];
    const int t = threadIdx.x, c0 = blockIdx.x * 64;
    {
        double v[TB];
#pragma unroll
        for (int l = 0; l < TB; ++l) v[l] = (t < kb && l < kb && l <= t) ? L[(size_t)l * ldl + t] : 0.0;
#pragma unroll
        for (int l = 0; l < TB; ++l) Ls[t][l] = v[l];
        rinv[t] = t < kb ? 1.0 / Ls[t][t] : 0.0;   // this lane stored the row
#pragma unroll
        for (int j = 0; j < TB; ++j) v[j] = (t < kb && c0 + j < nrhs) ? B[(size_t)(c0 + j) * ldb + t] : 0.0;
#pragma unroll
        for (int j = 0; j < TB; ++j) Bs[j][t] = v[j];
    }
    __syncthreads();
    double z[TB];
#pragma unroll
    for (int i = 0; i < TB; ++i) z[i] = Bs[t][i];
#pragma unroll
    for (int l = 0; l < TB; ++l) {
        if (l < kb) {
            z[l] *= rinv[l];
#pragma unroll
            for (int i = l + 1; i < TB; ++i) z[i] = fma(-Ls[i][l], z[l], z[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < TB; ++i) Bs[t][i] = z[i];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < TB; ++j)
        if (t < kb && c0 + j < nrhs) B[(size_t)(c0 + j) * ldb + t] = Bs[j][t];
}

// B (n x nrhs, ld ldb) <- L^{-1} B for lower triangular L (n x n, ld ldl):
// blocked right-looking forward substitution, a diagonal-block solve and an
// FP64 matrix-core update of the rows below per block of TRSM_NB rows.
void trsm_lower(hipStream_t s, int n, int nrhs, const double *L, int ldl, double *B, int ldb,
                KernelClock *kc) {
    if (n <= 0 || nrhs <= 0) return;
    for (int r0 = 0; r0 < n; r0 += TRSM_NB) {
        const int kb = n - r0 < TRSM_NB ? n - r0 : TRSM_NB;
        // algorithmic work: the kb x kb block read, kb rows of B read and
        // written, kb^2 flops per right-hand side
        if (kc)
            kc->begin(s, SVD_K_TRSM, ((double)kb * kb + 2.0 * kb * nrhs) * sizeof(double),
                      (double)kb * kb * nrhs);
        hipLaunchKernelGGL((k_trsm_diag<TRSM_NB>), dim3(cdiv(nrhs, 64)), dim3(64), 0, s, kb, nrhs,
                           L + (size_t)r0 * ldl + r0, ldl, B + r0, ldb);
        if (kc) kc->end(s);
        const int r1 = r0 + kb;
        if (r1 < n)
            gemm<double>(s, false, false, n - r1, nrhs, kb, -1.0, L + (size_t)r0 * ldl + r1, ldl,
                         B + r0, ldb, 1.0, B + r1, ldb, nullptr, 0, kc);
    }
}

// U(:, j) = Y(:, j) / ||Y(:, j)|| in FP64 (zero columns stay zero).
__global__ __launch_bounds__(256) void k_norm_cols64(int rows, int cols, const double *Y, int ldy,
                                                     double *U, int ldu) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= cols) return;
    double s = 0.0;
    for (int i = lane; i < rows; i += 64) {
        const double v = Y[(size_t)j * ldy + i];
        s = fma(v, v, s);
    }
    s = wave_sum(s);
    const double d = sqrt(s);
    for (int i = lane; i < rows; i += 64) {
        const double v = Y[(size_t)j * ldy + i];
        U[(size_t)j * ldu + i] = d > 0.0 ? v / d : 0.0;
    }
}

void normalize_cols64(hipStream_t s, int rows, int cols, const double *Y, int ldy, double *U,
                      int ldu) {
    hipLaunchKernelGGL(k_norm_cols64, dim3(cdiv(cols, 4)), dim3(256), 0, s, rows, cols, Y, ldy, U,
                       ldu);
}

} // namespace mpj
