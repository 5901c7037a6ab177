// Memory-bound helpers of the path: ingest with the non-finite scan, layout
// moves (gather by the pivots, transposes for the LQ step, padding), the
// branch tests of Section 3.5 (cond_R, trailing small columns, the scaled FP32
// copy X_t), precision conversions around the FP32 stage, and the final step
// of Algorithm 1 (norms, stable descending sort, normalisation) plus the sign
// rule for the singular vectors.
#include "common.hpp"
#include "internal.hpp"

namespace mpj {

static inline dim3 grid1(size_t n, int bs = 256) { return dim3((unsigned)cdivl((long long)n, bs)); }

__global__ void k_copy_scan(int m, int n, const double *A, int lda, double *D, int ldd, int *nf) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)m * n) return;
    const int i = (int)(e % m), j = (int)(e / m);
    const double v = A[(size_t)j * lda + i];
    // a non-finite entry is flagged and copied as 0 (the outputs of such a
    // call are undefined; the rest of the path then runs on finite data)
    const bool fin = isfinite(v);
    D[(size_t)j * ldd + i] = fin ? v : 0.0;
    if (!fin) *nf = 1;
}
void copy_scan(hipStream_t s, int m, int n, const double *A, int lda, double *D, int ldd, int *nf) {
    if ((size_t)m * n == 0) return;
    hipLaunchKernelGGL(k_copy_scan, grid1((size_t)m * n), dim3(256), 0, s, m, n, A, lda, D, ldd, nf);
}

__global__ void k_copy_upper(int n, const double *R, int ldr, double *D, int ldd) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)n * n) return;
    const int i = (int)(e % n), j = (int)(e / n);
    D[(size_t)j * ldd + i] = (i <= j) ? R[(size_t)j * ldr + i] : 0.0;
}
void copy_upper(hipStream_t s, int n, const double *R, int ldr, double *D, int ldd) {
    hipLaunchKernelGGL(k_copy_upper, grid1((size_t)n * n), dim3(256), 0, s, n, R, ldr, D, ldd);
}

__global__ void k_gather_cols(int rows, int n, const double *A, int lda, const int *piv, double *D,
                              int ldd) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)rows * n) return;
    const int i = (int)(e % rows), k = (int)(e / rows);
    D[(size_t)k * ldd + i] = A[(size_t)piv[k] * lda + i];
}
void gather_cols(hipStream_t s, int rows, int n, const double *A, int lda, const int *piv, double *D,
                 int ldd) {
    hipLaunchKernelGGL(k_gather_cols, grid1((size_t)rows * n), dim3(256), 0, s, rows, n, A, lda, piv,
                       D, ldd);
}

// L (Npad x Npad, ld ldl) = [R^T 0; 0 0] for the n x n upper triangle of R.
__global__ void k_t_upper_lower(int n, const double *R, int ldr, double *L, int ldl, int Np) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)Np * Np) return;
    const int i = (int)(e % Np), j = (int)(e / Np);
    double v = 0.0;
    if (i < n && j < n && i >= j) v = R[(size_t)i * ldr + j];
    L[(size_t)j * ldl + i] = v;
}
void transpose_upper_to_lower(hipStream_t s, int n, const double *R, int ldr, double *L, int ldl,
                              int Npad) {
    hipLaunchKernelGGL(k_t_upper_lower, grid1((size_t)Npad * Npad), dim3(256), 0, s, n, R, ldr, L, ldl,
                       Npad);
}

__global__ void k_identity(int N, double *V, int ldv) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)N * N) return;
    const int i = (int)(e % N), j = (int)(e / N);
    V[(size_t)j * ldv + i] = (i == j) ? 1.0 : 0.0;
}
void set_identity(hipStream_t s, int N, double *V, int ldv) {
    hipLaunchKernelGGL(k_identity, grid1((size_t)N * N), dim3(256), 0, s, N, V, ldv);
}

__global__ void k_zero(int rows, int cols, double *D, int ldd) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)rows * cols) return;
    const int i = (int)(e % rows), j = (int)(e / rows);
    D[(size_t)j * ldd + i] = 0.0;
}
void zero_pad_fill(hipStream_t s, int rows, int cols, double *D, int ldd) {
    if ((size_t)rows * cols == 0) return;
    hipLaunchKernelGGL(k_zero, grid1((size_t)rows * cols), dim3(256), 0, s, rows, cols, D, ldd);
}

// B (cols x rows, ldb) = A^T (A rows x cols, lda), through 32 x 32 LDS tiles
// so that both sides are read and written along their columns.
__global__ __launch_bounds__(256) void k_transpose(int rows, int cols, const double *A, int lda,
                                                   double *B, int ldb) {
    __shared__ double tile[32][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int i = i0 + tx, j = j0 + ty + k;
        if (i < rows && j < cols) tile[ty + k][tx] = A[(size_t)j * lda + i];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int j = j0 + tx, i = i0 + ty + k;   // B(j, i) = A(i, j)
        if (i < rows && j < cols) B[(size_t)i * ldb + j] = tile[tx][ty + k];
    }
}
void transpose64(hipStream_t s, int rows, int cols, const double *A, int lda, double *B, int ldb) {
    if ((size_t)rows * cols == 0) return;
    hipLaunchKernelGGL(k_transpose, dim3(cdiv(rows, 32), cdiv(cols, 32)), dim3(256), 0, s, rows, cols,
                       A, lda, B, ldb);
}

// out[0] = max|r_ii| / min|r_ii|  (cond_R of Algorithm 4, Section 3.5)
__global__ __launch_bounds__(256) void k_diag_cond(int n, const double *R, int ldr, double *out) {
    __shared__ double mx[4], mn[4];
    double a = 0.0, b = INFINITY;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double v = fabs(R[(size_t)i * ldr + i]);
        a = fmax(a, v);
        b = fmin(b, v);
    }
    a = wave_max(a);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b = fmin(b, __shfl_xor(b, o, 64));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { mx[w] = a; mn[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double A = fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3]));
        double B = fmin(fmin(mn[0], mn[1]), fmin(mn[2], mn[3]));
        out[0] = (B > 0.0) ? A / B : INFINITY;
    }
}
void diag_cond(hipStream_t s, int n, const double *R, int ldr, double *out) {
    hipLaunchKernelGGL(k_diag_cond, dim3(1), dim3(256), 0, s, n, R, ldr, out);
}

__global__ __launch_bounds__(256) void k_col_norms(int rows, int n, const double *X, int ldx,
                                                   double *nrm) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    double s = 0.0;
    for (int i = lane; i < rows; i += 64) {
        const double v = X[(size_t)j * ldx + i];
        s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) nrm[j] = sqrt(s);
}
void col_norms(hipStream_t s, int rows, int n, const double *X, int ldx, double *nrm) {
    hipLaunchKernelGGL(k_col_norms, dim3(cdiv(n, 4)), dim3(256), 0, s, rows, n, X, ldx, nrm);
}

// out[0] = length of the run of trailing columns with norm <= rel * max norm.
__global__ __launch_bounds__(256) void k_count_small(int n, const double *nrm, double rel, int *out) {
    __shared__ double mx[4];
    __shared__ int first_big[4];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a = fmax(a, nrm[i]);
    a = wave_max(a);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) mx[w] = a;
    __syncthreads();
    const double thr = rel * fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3]));
    int last = -1;  // largest index with a norm above the threshold
    for (int i = threadIdx.x; i < n; i += 256)
        if (nrm[i] > thr) last = max(last, i);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) last = max(last, __shfl_xor(last, o, 64));
    if ((threadIdx.x & 63) == 0) first_big[w] = last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int L = max(max(first_big[0], first_big[1]), max(first_big[2], first_big[3]));
        out[0] = n - 1 - L;
    }
}
void count_small(hipStream_t s, int n, const double *nrm, double rel, int *out) {
    hipLaunchKernelGGL(k_count_small, dim3(1), dim3(256), 0, s, n, nrm, rel, out);
}

// X_t = low(X) D^-1 with D_jj the 2-norm of column j (Algorithm 4, Section
// 3.5).  The norm is summed in FP64 and the column divided by it before the
// rounding to FP32: squared FP32 norms would underflow for columns below
// about 1e-19 (graded inputs reach 1e-20), and the rounded X_t is the same
// up to one FP32 rounding for every column that an FP32 norm could handle.
__global__ __launch_bounds__(256) void k_make_xt32(int n, const double *X, int ldx, float *Xt,
                                                   int ldt) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double v = X[(size_t)j * ldx + i];
        s = fma(v, v, s);
    }
    s = wave_sum(s);
    const double d = sqrt(s);
    const double inv = d > 0.0 ? 1.0 / d : 0.0;
    for (int i = lane; i < n; i += 64) Xt[(size_t)j * ldt + i] = (float)(X[(size_t)j * ldx + i] * inv);
}
void make_xt32(hipStream_t s, int n, const double *X, int ldx, float *Xt, int ldt) {
    hipLaunchKernelGGL(k_make_xt32, dim3(cdiv(n, 4)), dim3(256), 0, s, n, X, ldx, Xt, ldt);
}

__global__ void k_f64_f32(int rows, int cols, const double *X, int ldx, float *Y, int ldy,
                          const double *scale) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)rows * cols) return;
    const int i = (int)(e % rows), j = (int)(e / rows);
    const double f = scale ? *scale : 1.0;
    Y[(size_t)j * ldy + i] = (float)(X[(size_t)j * ldx + i] * f);
}
void convert_f64_f32(hipStream_t s, int rows, int cols, const double *X, int ldx, float *Y, int ldy,
                     const double *scale) {
    hipLaunchKernelGGL(k_f64_f32, grid1((size_t)rows * cols), dim3(256), 0, s, rows, cols, X, ldx, Y,
                       ldy, scale);
}

// scale[0] = 2^e with e chosen so that the largest of the n column norms
// becomes about 2^56 (e = 56 - ceil(log2(max norm)), clamped to the FP64
// exponent range; 1 for an all-zero matrix).  An FP32 copy of the columns
// times this scale keeps every squared norm and dot product inside the FP32
// range for column norms spanning up to about 2^118: at most 2^112 at the
// top, and above the FP32 normal minimum 2^-126 down to norms 2^-63 times
// the largest.  Scaling by a power of two is exact, and the FP32 stages only
// use scale-invariant quantities (pivot order, rotation angles, normalised
// columns).
__global__ void k_pow2_scale(int n, const double *nrm, double *scale) {
    __shared__ double mx[4];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a = fmax(a, nrm[i]);
    a = wave_max(a);
    if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3]));
        double f = 1.0;
        if (m > 0.0 && isfinite(m)) {
            int e = 56 - ilogb(m) - 1;
            e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
            f = ldexp(1.0, e);
        }
        scale[0] = f;
    }
}
void pow2_scale(hipStream_t s, int n, const double *nrm, double *scale) {
    hipLaunchKernelGGL(k_pow2_scale, dim3(1), dim3(256), 0, s, n, nrm, scale);
}

// BF16 copies for the three-precision variant: Y16 = bf16(X * scale[0])
// (round to nearest even), and the exact widening back to FP32.
__device__ __forceinline__ unsigned short f32_to_bf16(float x) {
    const unsigned r = __float_as_uint(x);
    return (unsigned short)((r + 0x7fffu + ((r >> 16) & 1u)) >> 16);
}
__global__ void k_f64_bf16(int rows, int cols, const double *X, int ldx, unsigned short *Y, int ldy,
                           const double *scale) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)rows * cols) return;
    const int i = (int)(e % rows), j = (int)(e / rows);
    const double f = scale ? *scale : 1.0;
    Y[(size_t)j * ldy + i] = f32_to_bf16((float)(X[(size_t)j * ldx + i] * f));
}
void convert_f64_bf16(hipStream_t s, int rows, int cols, const double *X, int ldx, unsigned short *Y,
                      int ldy, const double *scale) {
    hipLaunchKernelGGL(k_f64_bf16, grid1((size_t)rows * cols), dim3(256), 0, s, rows, cols, X, ldx, Y,
                       ldy, scale);
}
__global__ void k_bf16_f32(int rows, int cols, const unsigned short *Y16, int ld16, float *Y, int ldy) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)rows * cols) return;
    const int i = (int)(e % rows), j = (int)(e / rows);
    Y[(size_t)j * ldy + i] = __uint_as_float((unsigned)Y16[(size_t)j * ld16 + i] << 16);
}
void widen_bf16_f32(hipStream_t s, int rows, int cols, const unsigned short *Y16, int ld16, float *Y,
                    int ldy) {
    hipLaunchKernelGGL(k_bf16_f32, grid1((size_t)rows * cols), dim3(256), 0, s, rows, cols, Y16, ld16,
                       Y, ldy);
}

__global__ void k_f32_f64(int rows, int cols, const float *X, int ldx, double *Y, int ldy) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)rows * cols) return;
    const int i = (int)(e % rows), j = (int)(e / rows);
    Y[(size_t)j * ldy + i] = (double)X[(size_t)j * ldx + i];
}
void convert_f32_f64(hipStream_t s, int rows, int cols, const float *X, int ldx, double *Y, int ldy) {
    hipLaunchKernelGGL(k_f32_f64, grid1((size_t)rows * cols), dim3(256), 0, s, rows, cols, X, ldx, Y,
                       ldy);
}

// U(:, j) = double(Y(:, j) / ||Y(:, j)||), the FP32 left vectors U_low lifted to FP64.
__global__ __launch_bounds__(256) void k_norm_f32_f64(int rows, int cols, const float *Y, int ldy,
                                                      double *U, int ldu) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= cols) return;
    float s = 0.f;
    for (int i = lane; i < rows; i += 64) {
        const float v = Y[(size_t)j * ldy + i];
        s += v * v;
    }
    s = wave_sum(s);
    const float d = sqrtf(s);
    for (int i = lane; i < rows; i += 64) {
        const float v = Y[(size_t)j * ldy + i];
        U[(size_t)j * ldu + i] = d > 0.f ? (double)(v / d) : 0.0;
    }
}
void normalize_f32_to_f64(hipStream_t s, int rows, int cols, const float *Y, int ldy, double *U,
                          int ldu) {
    hipLaunchKernelGGL(k_norm_f32_f64, dim3(cdiv(cols, 4)), dim3(256), 0, s, rows, cols, Y, ldy, U,
                       ldu);
}

// rank_j = #{i : s_i > s_j} + #{i < j : s_i == s_j}: a stable descending order.
// The values are read through LDS, 2048 at a time, by every workgroup (the
// reads are broadcasts: every thread of a wavefront reads the same value).
__global__ __launch_bounds__(256) void k_rank(int n, const double *sig, int *rank) {
    __shared__ double sh[2048];
    const int j = blockIdx.x * 256 + threadIdx.x;
    const double sj = j < n ? sig[j] : 0.0;
    int r = 0;
    for (int i0 = 0; i0 < n; i0 += 2048) {
        const int m = min(2048, n - i0);
        __syncthreads();
        for (int e = threadIdx.x; e < m; e += 256) sh[e] = sig[i0 + e];
        __syncthreads();
        int e = 0;
        for (; e + 8 <= m; e += 8) {   // eight reads in flight
            double si[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) si[u] = sh[e + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) r += (si[u] > sj) || (si[u] == sj && i0 + e + u < j);
        }
        for (; e < m; ++e) {
            const double si = sh[e];
            r += (si > sj) || (si == sj && i0 + e < j);
        }
    }
    if (j < n) rank[j] = r;
}

// Column j of Y / V goes to column rank_j of U_X / V_X (n x n, ld n).
__global__ __launch_bounds__(256) void k_scatter(int n, int N, const double *Y, const double *V,
                                                 const double *sig, const int *rank, double *UX,
                                                 double *VX, double *S, int *nzero, int *nonfinite) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    const int d = rank[j];
    const double sj = sig[j];
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    for (int i = lane; i < n; i += 64) {
        UX[(size_t)d * n + i] = sj > 0.0 ? Y[(size_t)j * N + i] * inv : 0.0;
        if (V) VX[(size_t)d * n + i] = V[(size_t)j * N + i];
    }
    if (lane == 0) {
        S[d] = sj;
        if (sj == 0.0) atomicAdd(nzero, 1);
        if (!isfinite(sj)) *nonfinite = 1;
    }
}

void finalize_sort(hipStream_t s, int n, int N, const double *Y, const double *V, double *sig,
                   int *rank, double *UX, double *VX, double *S, int *nzero, int *nonfinite,
                   bool want_v) {
    col_norms(s, N, n, Y, N, sig);
    hipLaunchKernelGGL(k_rank, dim3(cdiv(n, 256)), dim3(256), 0, s, n, sig, rank);
    hipLaunchKernelGGL(k_scatter, dim3(cdiv(n, 4)), dim3(256), 0, s, n, N, Y, want_v ? V : nullptr,
                       sig, rank, UX, VX, S, nzero, nonfinite);
}

__global__ void k_place_u(int m, int n, const double *W, int ldw, double *U, int ldu) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)m * n) return;
    const int i = (int)(e % m), j = (int)(e / m);
    U[(size_t)j * ldu + i] = (i < n) ? W[(size_t)j * ldw + i] : 0.0;
}
void place_u(hipStream_t s, int m, int n, const double *W, int ldw, double *U, int ldu) {
    hipLaunchKernelGGL(k_place_u, grid1((size_t)m * n), dim3(256), 0, s, m, n, W, ldw, U, ldu);
}

// V(piv[k], :) = T(k, :)   (V = P T)
__global__ void k_perm_rows(int n, const double *T, int ldt, const int *piv, double *V, int ldv) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)n * n) return;
    const int k = (int)(e % n), j = (int)(e / n);
    V[(size_t)j * ldv + piv[k]] = T[(size_t)j * ldt + k];
}
void permute_rows_v(hipStream_t s, int n, const double *T, int ldt, const int *piv, double *V,
                    int ldv) {
    hipLaunchKernelGGL(k_perm_rows, grid1((size_t)n * n), dim3(256), 0, s, n, T, ldt, piv, V, ldv);
}

// For column i: k = first index of max |V(k, i)|; if V(k, i) < 0 negate V(:, i), U(:, i).
__global__ __launch_bounds__(256) void k_sign(int m, int n, double *U, int ldu, int have_u, double *V,
                                              int ldv) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    double best = -1.0;
    int bk = 0;   // a valid row even when no |V(k, i)| compares greater (NaN)
    for (int k = lane; k < n; k += 64) {
        const double a = fabs(V[(size_t)i * ldv + k]);
        if (a > best) { best = a; bk = k; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int okk = __shfl_xor(bk, o, 64);
        if (ob > best || (ob == best && okk < bk)) { best = ob; bk = okk; }
    }
    if (V[(size_t)i * ldv + bk] < 0.0) {
        for (int k = lane; k < n; k += 64) V[(size_t)i * ldv + k] = -V[(size_t)i * ldv + k];
        if (have_u)
            for (int k = lane; k < m; k += 64) U[(size_t)i * ldu + k] = -U[(size_t)i * ldu + k];
    }
}
void sign_normalize(hipStream_t s, int m, int n, double *U, int ldu, bool have_u, double *V, int ldv) {
    hipLaunchKernelGGL(k_sign, dim3(cdiv(n, 4)), dim3(256), 0, s, m, n, U, ldu, (int)have_u, V, ldv);
}

} // namespace mpj

namespace mpj {

// A(:, idx[k]) = D(:, k) for k < n   (the inverse of gather_cols)
__global__ void k_scatter_cols(int rows, int n, const double *D, int ldd, const int *idx, double *A,
                               int lda) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)rows * n) return;
    const int i = (int)(e % rows), k = (int)(e / rows);
    A[(size_t)idx[k] * lda + i] = D[(size_t)k * ldd + i];
}
void scatter_cols(hipStream_t s, int rows, int n, const double *D, int ldd, const int *idx, double *A,
                  int lda) {
    if ((size_t)rows * n == 0) return;
    hipLaunchKernelGGL(k_scatter_cols, grid1((size_t)rows * n), dim3(256), 0, s, rows, n, D, ldd, idx,
                       A, lda);
}

} // namespace mpj
