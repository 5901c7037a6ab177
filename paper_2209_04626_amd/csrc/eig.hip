// Mixed-precision symmetric eigensolver (Section 8, Algorithm 6).
//
// For a symmetric n x n A, Algorithm 6 computes a low-precision spectral
// decomposition, orthogonalises its vectors in working precision (Q) and
// refines with the one-sided Jacobi SVD of A Q, V not formed: for symmetric A
// the left singular vectors are eigenvectors.  Those three steps are the
// mixed-precision Jacobi SVD of A itself (Algorithm 4: FP32 one-sided Jacobi
// as the low-precision decomposition, the switch to Q, FP64 sweeps on X Q with
// the QR preconditioning that the paper's xGEJSV-based implementation also
// applies), so svd_mixed with want_v = 0 performs them here, giving
// A = U Sigma V^T with U and Sigma.  Then:
//   4. the blocks of U^T A U: consecutive sigma whose relative gap is at most
//      tol_cluster form one block (sigma and -sigma can both be eigenvalues);
//   5. each block of two or more is diagonalised by two-sided Jacobi in FP64
//      and its rotation applied to U's columns; a block of one takes the sign
//      of u_i^T A u_i;
//   6. eigenvalues sorted ascending, eigenvectors with them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/mpjsvd.h"
#include "common.hpp"
#include "internal.hpp"

namespace mpj {
namespace {

constexpr int EIG_BMAX = 64;   // largest block diagonalised (held in LDS)
constexpr int EIG_NT = 256;

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct EigLayout {
    int n;
    size_t off_ux, off_t1, off_s, off_d, off_mu, off_blk, off_perm, off_svd, svd_bytes, total;
};

svd_opts eig_svd_opts(const svd_opts &o) {
    svd_opts s = o;
    s.want_u = 1;
    s.want_v = 0;
    s.sign_normalize = 0;
    s.kernel_timing = 0;
    return s;
}

EigLayout eig_layout(int n, const svd_opts &o) {
    EigLayout L;
    L.n = n;
    const size_t d = sizeof(double);
    const size_t nn = (size_t)n * n;
    size_t p = 0;
    auto take = [&](size_t bytes) { size_t o_ = p; p += al256(bytes); return o_; };
    L.off_ux = take(nn * d);
    L.off_t1 = take(nn * d);
    L.off_s = take((size_t)n * d);
    L.off_d = take((size_t)n * d);
    L.off_mu = take((size_t)n * d);
    L.off_blk = take((size_t)n * sizeof(int) + 8);
    L.off_perm = take((size_t)n * sizeof(int));
    const svd_opts so = eig_svd_opts(o);
    L.svd_bytes = svd_workspace_size(n, n, &so);
    L.off_svd = take(L.svd_bytes);
    L.total = p;
    return L;
}

// d[i] = U(:, i) . T(:, i)   (one wavefront per column)
__global__ __launch_bounds__(256) void k_coldot(int n, const double *U, int ldu, const double *T,
                                                int ldt, double *d) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s = fma(U[(size_t)j * ldu + i], T[(size_t)j * ldt + i], s);
    s = wave_sum(s);
    if (lane == 0) d[j] = s;
}

// One workgroup per block (blk[2c] = first column, blk[2c + 1] = size k,
// 2 <= k <= EIG_BMAX):
//   B = U_b^T T_b (T = A U), symmetrised; cyclic two-sided Jacobi on B in
//   FP64 with the rotations accumulated in W (the symmetric Schur rotation:
//   t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (b_qq - b_pp) /
//   (2 b_pq)), until a sweep without rotation or 40 sweeps; mu = diag(B);
//   U_b <- U_b W.
__global__ __launch_bounds__(EIG_NT) void k_eig_block(int n, const int *blk, double *U, int ldu,
                                                     const double *T, int ldt, double *mu,
                                                     double eps) {
    __shared__ double B[EIG_BMAX][EIG_BMAX + 1];
    __shared__ double W[EIG_BMAX][EIG_BMAX + 1];
    __shared__ double rot[3];
    __shared__ int any;
    const int c0 = blk[2 * blockIdx.x], k = blk[2 * blockIdx.x + 1];
    const int t = threadIdx.x;
    double *Ub = U + (size_t)c0 * ldu;
    const double *Tb = T + (size_t)c0 * ldt;
    // 1. B = U_b^T T_b (upper triangle computed, then mirrored as the mean)
    for (int e = t; e < k * k; e += EIG_NT) {
        const int i = e % k, j = e / k;
        double s = 0.0;
        for (int r = 0; r < n; ++r) s = fma(Ub[(size_t)i * ldu + r], Tb[(size_t)j * ldt + r], s);
        B[i][j] = s;
        W[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int e = t; e < k * k; e += EIG_NT) {
        const int i = e % k, j = e / k;
        if (i < j) {
            const double m = 0.5 * (B[i][j] + B[j][i]);
            B[i][j] = m;
            B[j][i] = m;
        }
    }
    __syncthreads();
    // 2. cyclic Jacobi
    for (int sw = 0; sw < 40; ++sw) {
        if (t == 0) any = 0;
        __syncthreads();
        for (int p = 0; p < k - 1; ++p) {
            for (int q = p + 1; q < k; ++q) {
                if (t == 0) {
                    const double bpp = B[p][p], bqq = B[q][q], bpq = B[p][q];
                    double c = 1.0, s = 0.0, tt = 0.0;
                    if (bpq != 0.0 && fabs(bpq) > eps * sqrt(fabs(bpp) * fabs(bqq))) {
                        const double zeta = (bqq - bpp) / (2.0 * bpq);
                        tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                        any = 1;
                    }
                    rot[0] = c; rot[1] = s; rot[2] = tt;
                }
                __syncthreads();
                const double c = rot[0], s = rot[1], tt = rot[2];
                if (s != 0.0) {
                    const double bpq = B[p][q];
                    if (t < k && t != p && t != q) {
                        const double brp = B[t][p], brq = B[t][q];
                        const double np_ = c * brp - s * brq, nq_ = s * brp + c * brq;
                        B[t][p] = np_; B[t][q] = nq_;
                        B[p][t] = np_; B[q][t] = nq_;
                    }
                    if (t < k) {
                        const double wp = W[t][p], wq = W[t][q];
                        W[t][p] = c * wp - s * wq;
                        W[t][q] = s * wp + c * wq;
                    }
                    __syncthreads();
                    if (t == 0) {
                        B[p][p] = B[p][p] - tt * bpq;
                        B[q][q] = B[q][q] + tt * bpq;
                        B[p][q] = 0.0;
                        B[q][p] = 0.0;
                    }
                }
                __syncthreads();
            }
        }
        if (!any) break;
        __syncthreads();
    }
    if (t < k) mu[c0 + t] = B[t][t];
    // 3. U_b <- U_b W, one row per thread
    for (int r = t; r < n; r += EIG_NT) {
        double u[EIG_BMAX];
#pragma unroll
        for (int j = 0; j < EIG_BMAX; ++j) u[j] = j < k ? Ub[(size_t)j * ldu + r] : 0.0;
        for (int j = 0; j < k; ++j) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < EIG_BMAX; ++i)
                if (i < k) s = fma(u[i], W[i][j], s);
            Ub[(size_t)j * ldu + r] = s;
        }
    }
}

// X(:, j) = U(:, perm[j])
__global__ void k_perm_cols(int n, const double *U, int ldu, const int *perm, double *X, int ldx) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)n * n) return;
    const int i = (int)(e % n), j = (int)(e / n);
    X[(size_t)j * ldx + i] = U[(size_t)perm[j] * ldu + i];
}

int eig_read_back(hipStream_t s, void *host, const void *dev, size_t bytes) {
    hipError_t e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        note_hip_error(e, "eig read back");
        return -1;
    }
    return 0;
}

bool eig_opts_ok(const svd_opts &o) {
    return (o.inner_pairs == 0 || o.inner_pairs == 1) && o.v_method >= 0 && o.v_method <= 1 &&
           o.switch_method >= 1 && o.switch_method <= 3 &&
           (o.pivot_precision == 32 || o.pivot_precision == 64);
}

} // namespace
} // namespace mpj

using namespace mpj;

extern "C" size_t eig_workspace_size(int n, const svd_opts *op) {
    if (n < 0 || n > 8192) return 0;
    svd_opts o;
    if (op) o = *op; else svd_default_opts(&o, 1);
    return eig_layout(n, o).total;
}

extern "C" int eig_mixed(int n, const double *A, int lda, double *W, double *X, int ldx, void *work,
                         size_t work_bytes, const svd_opts *op, eig_info *info, void *stream) {
    svd_opts o;
    if (op) o = *op; else svd_default_opts(&o, 1);
    if (n < 0 || n > 8192) return -1;
    if (n > 0 && !A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n > 0 && !W) return -4;
    if (n > 0 && !X) return -5;
    if (ldx < (n > 1 ? n : 1)) return -6;
    if (!eig_opts_ok(o)) return -9;
    if (info) memset(info, 0, sizeof(*info));
    if (n == 0) return 0;
    (void)hipGetLastError();
    const EigLayout L = eig_layout(n, o);
    if (L.svd_bytes == 0) return -1;
    if (!work) return -7;
    if (work_bytes < L.total) return -8;

    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)work;
    auto D = [&](size_t off) { return (double *)(w + off); };
    double *UX = D(L.off_ux), *T1 = D(L.off_t1), *S = D(L.off_s), *dd = D(L.off_d), *mu = D(L.off_mu);
    int *blk = (int *)(w + L.off_blk), *perm = (int *)(w + L.off_perm);

    hipEvent_t ev[5] = {};
    bool evok = true;
    for (int i = 0; i < 5; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) { ev[i] = nullptr; evok = false; }
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 5; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};
    if (evok && hipEventRecord(ev[0], s) != hipSuccess) evok = false;

    // 1-3. A = U Sigma V^T by the mixed-precision Jacobi SVD, V not formed
    const svd_opts so = eig_svd_opts(o);
    svd_info si;
    const int rc = svd_mixed(n, n, A, lda, S, UX, n, nullptr, n, w + L.off_svd, L.svd_bytes, &so, &si,
                             stream);
    if (rc != 0) return rc == SVD_ERR_HIP ? SVD_ERR_HIP : -9;
    if (si.status == SVD_ERR_NONFINITE) {
        if (info) info->status = SVD_ERR_NONFINITE;
        return 0;
    }
    if (evok && hipEventRecord(ev[1], s) != hipSuccess) evok = false;

    // 4. T1 = A U; d_i = u_i^T A u_i
    gemm<double>(s, false, false, n, n, n, 1.0, A, lda, UX, n, 0.0, T1, n, nullptr, 0);
    hipLaunchKernelGGL(k_coldot, dim3(cdiv(n, 4)), dim3(256), 0, s, n, UX, n, T1, n, dd);
    MPJ_CHECK(hipGetLastError());
    std::vector<double> hS(n), hd(n), hmu(n);
    if (eig_read_back(s, hS.data(), S, (size_t)n * sizeof(double))) return SVD_ERR_HIP;
    if (eig_read_back(s, hd.data(), dd, (size_t)n * sizeof(double))) return SVD_ERR_HIP;
    if (evok && hipEventRecord(ev[2], s) != hipSuccess) evok = false;
    const double eps_work = o.eps_work > 0 ? o.eps_work : sqrt((double)n) * ldexp(1.0, -53);

    // 5. blocks of (nearly) equal sigma
    const double tol = o.tol_cluster > 0 ? o.tol_cluster : 1e-8;
    std::vector<int> hblk;
    int ncl = 0, kmax = 1;
    for (int i = 0; i < n;) {
        int j = i + 1;
        while (j < n && hS[j - 1] - hS[j] <= tol * hS[j - 1]) ++j;
        const int k = j - i;
        if (k >= 2) {
            hblk.push_back(i);
            hblk.push_back(k);
            ++ncl;
            kmax = std::max(kmax, k);
        }
        i = j;
    }
    if (kmax > EIG_BMAX) {
        if (info) {
            info->status = EIG_ERR_CLUSTER;
            info->n_clusters = ncl;
            info->max_cluster = kmax;
        }
        return 0;
    }
    if (ncl > 0) {
        MPJ_CHECK(hipMemcpyAsync(blk, hblk.data(), hblk.size() * sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_eig_block, dim3(ncl), dim3(EIG_NT), 0, s, n, (const int *)blk, UX, n,
                           (const double *)T1, n, mu, eps_work);
        MPJ_CHECK(hipGetLastError());
        if (eig_read_back(s, hmu.data(), mu, (size_t)n * sizeof(double))) return SVD_ERR_HIP;
    }
    if (evok && hipEventRecord(ev[3], s) != hipSuccess) evok = false;

    // 6. eigenvalues: sign(u_i^T A u_i) sigma_i for a block of one; in a
    // block, the eigenvalues mu of the diagonalised block give the signs,
    // matched to the block's sigma by decreasing magnitude
    std::vector<double> lam(n);
    for (int i = 0; i < n; ++i) lam[i] = hd[i] < 0.0 ? -hS[i] : hS[i];
    for (int c = 0; c < ncl; ++c) {
        const int c0 = hblk[2 * c], k = hblk[2 * c + 1];
        std::vector<int> ord(k);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int b) { return fabs(hmu[c0 + a]) > fabs(hmu[c0 + b]); });
        for (int r = 0; r < k; ++r) {
            const int jj = ord[r];
            lam[c0 + jj] = hmu[c0 + jj] < 0.0 ? -hS[c0 + r] : hS[c0 + r];
        }
    }
    std::vector<int> hperm(n);
    std::iota(hperm.begin(), hperm.end(), 0);
    std::stable_sort(hperm.begin(), hperm.end(), [&](int a, int b) { return lam[a] < lam[b]; });
    std::vector<double> hW(n);
    for (int j = 0; j < n; ++j) hW[j] = lam[hperm[j]];
    MPJ_CHECK(hipMemcpyAsync(perm, hperm.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, s));
    MPJ_CHECK(hipMemcpyAsync(W, hW.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_perm_cols, dim3((unsigned)cdivl((long long)n * n, 256)), dim3(256), 0, s, n,
                       (const double *)UX, n, (const int *)perm, X, ldx);
    if (o.sign_normalize) sign_normalize(s, n, n, nullptr, 0, false, X, ldx);
    MPJ_CHECK(hipGetLastError());
    if (evok && hipEventRecord(ev[4], s) != hipSuccess) evok = false;
    MPJ_CHECK(hipStreamSynchronize(s));   // the host vectors above are the copies' sources

    if (info) {
        info->status = si.status;
        info->sweeps_low = si.sweeps_low;
        info->sweeps_work = si.sweeps_work;
        info->n_clusters = ncl;
        info->max_cluster = kmax;
        if (evok)
            for (int i = 0; i < 4; ++i) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) ms = 0.f;
                info->stage_ms[i] = ms;
            }
    }
    return 0;
}
