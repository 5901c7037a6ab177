// One-sided Jacobi sweeps (Algorithm 1) as block-Jacobi rounds on gfx950.
//
// The n columns are split into blocks of b columns; each sweep runs the
// nb - 1 rounds of a round-robin tournament over the nb blocks, so every
// column pair (p, q) of the matrix meets in exactly one block pair per sweep
// (pairs inside a block meet in every round).  For each block pair (I, J) of
// a round:
//   1. gram:   G = [Y_I Y_J]^T [Y_I Y_J] (2b x 2b) from MFMA over row chunks;
//              FP32 data accumulates in FP32, FP64 in FP64.
//   2. inner:  in FP64, test every column pair of the block with the rule of
//              Algorithm 1 (|g_pq| > eps sqrt(g_pp g_qq)); if none needs it the
//              pair is skipped.  Otherwise run cyclic Jacobi rounds on G
//              (the rotations of Section 2.1 computed from g_pp, g_qq, g_pq
//              exactly as from the column dot products) and accumulate the
//              2b x 2b orthogonal product W of the rotations.
//   3. update: [Y_I Y_J] <- [Y_I Y_J] W and [V_I V_J] <- [V_I V_J] W (MFMA).
// Applying any orthogonal W keeps the computation rowwise backward stable
// (the argument of Section 4), and convergence is declared only after a sweep
// in which no block pair needed a rotation on a freshly computed Gram block.
#include <string.h>

#include "common.hpp"
#include "internal.hpp"

namespace mpj {

constexpr int JR_NT = 256;   // threads per workgroup
constexpr int JR_RG = 256;   // rows per workgroup in update
constexpr int JR_RGG = 256;  // rows per workgroup in gram
constexpr int JR_SLAB = 32;  // rows staged in LDS at a time

__device__ __forceinline__ int blk_col(int c, int b, int I, int J) {
    return c < b ? I * b + c : J * b + (c - b);
}

// Partial Gram block of one row chunk.  Only the 16 x 16 tiles on or above
// the block diagonal are formed (G is symmetric; the inner solve reads the
// upper triangle).  The next 32-row slab is loaded into registers while the
// matrix cores work on the current one.
template <typename T, int B2>
__global__ __launch_bounds__(JR_NT) void jac_gram(int N, int nblk, int r, const T *__restrict__ Y,
                                                  int ldy, T *__restrict__ Gp, int nchunk) {
    constexpr int b = B2 / 2;
    constexpr int NTT = B2 / 16;                       // tiles per dimension
    constexpr int NUT = NTT * (NTT + 1) / 2;           // upper-triangle tiles
    constexpr int TPW = (NUT + 3) / 4;
    constexpr int PER = B2 * JR_SLAB / JR_NT;          // slab elements per thread
    __shared__ T Ps[B2][JR_SLAB + 1];
    const int pair = blockIdx.x, chunk = blockIdx.y;
    int I, J;
    rr_slot(nblk, r, pair, &I, &J);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // this wavefront's tiles (ti <= tj), enumerated row by row
    int tI[TPW], tJ[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        int u = w + 4 * q, ti = 0;
        while (u >= NTT - ti && ti < NTT) { u -= NTT - ti; ++ti; }
        tI[q] = ti; tJ[q] = ti + u;
    }
    typedef typename acc4<T>::type V4;
    V4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = V4{0, 0, 0, 0};
    const int rbeg = chunk * JR_RGG, rend = min(N, rbeg + JR_RGG);
    T pf[PER];
    auto fetch = [&](int r0) {
#pragma unroll
        for (int e0 = 0; e0 < PER; ++e0) {
            const int e = tid + e0 * JR_NT;
            const int c = e / JR_SLAB, rr = e % JR_SLAB;
            const int gi = r0 + rr;
            pf[e0] = gi < rend ? Y[(size_t)blk_col(c, b, I, J) * ldy + gi] : T(0);
        }
    };
    fetch(rbeg);
    for (int r0 = rbeg; r0 < rend; r0 += JR_SLAB) {
        __syncthreads();
#pragma unroll
        for (int e0 = 0; e0 < PER; ++e0) {
            const int e = tid + e0 * JR_NT;
            Ps[e / JR_SLAB][e % JR_SLAB] = pf[e0];
        }
        __syncthreads();
        if (r0 + JR_SLAB < rend) fetch(r0 + JR_SLAB);
#pragma unroll
        for (int kk = 0; kk < JR_SLAB; kk += 4) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (w + 4 * q < NUT) {
                    const T a = Ps[16 * tI[q] + lane % 16][kk + lane / 16];
                    const T bb = Ps[16 * tJ[q] + lane % 16][kk + lane / 16];
                    acc[q] = mfma16(a, bb, acc[q]);
                }
            }
        }
    }
    T *out = Gp + ((size_t)pair * nchunk + chunk) * B2 * B2;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (w + 4 * q < NUT) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * tI[q] + mfma_row<T>(lane, e), j = 16 * tJ[q] + lane % 16;
                out[i + j * B2] = acc[q][e];
            }
        }
    }
}

// The Jacobi rotation of Section 2.1 for (alpha, beta, gamma): the root
// closest to the identity, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// zeta = (beta - alpha) / (2 gamma), sign(0) = +1.
__device__ __forceinline__ void jac_rot(double al, double be, double ga, double *c, double *s,
                                        double *t) {
    const double zeta = (be - al) / (2.0 * ga);
    const double sg = zeta >= 0.0 ? 1.0 : -1.0;
    const double az = fabs(zeta);
    // sqrt(1 + zeta^2) without overflow: for |zeta| > 1e150 it is |zeta|
    const double root = az > 1e150 ? az : sqrt(1.0 + az * az);
    const double tt = sg / (az + root);
    const double cc = 1.0 / sqrt(1.0 + tt * tt);
    *c = cc; *s = tt * cc; *t = tt;
}

// Inner solve of one block pair.  G and the accumulated W are held in the
// stage's precision T (FP32 in the FP32 stage, FP64 in the FP64 stage); every
// rotation angle and threshold test is evaluated in FP64.  The rotation test
// |g_pq| > eps sqrt(g_pp g_qq) is evaluated squared (no square roots).  Each
// round loads all of a thread's 2x2 groups of G and W entries first, then
// updates and stores them, so the LDS latency is paid once per round.
template <typename T, int B2, int NT>
__global__ __launch_bounds__(NT) void jac_inner(int nchunk, const T *__restrict__ Gp,
                                                T *__restrict__ Wm, int *skip, int *flag,
                                                double eps, int max_inner) {
    constexpr int LD = B2 + 1;
    constexpr int H = B2 / 2;
    constexpr int TG = (H * H) / NT;      // 2x2 groups of G per thread
    constexpr int TW = (B2 * H) / NT;     // W column-pair entries per thread
    constexpr int TE = (B2 * B2) / NT;    // Gram entries per thread
    static_assert(TG * NT == H * H && TW * NT == B2 * H && TE * NT == B2 * B2, "tiling");
    __shared__ T G[B2 * LD];
    __shared__ T W[B2 * LD];
    __shared__ T ca[B2], cb[B2];
    __shared__ T tt[H];
    __shared__ int ired[NT / 64 > 0 ? NT / 64 : 1];
    __shared__ int any_rot;
    const int pair = blockIdx.x, tid = threadIdx.x;
    const double eps2 = eps * eps;

    // 1. reduce the partial Gram blocks (fixed chunk order, FP64 sums)
    {
        const T *gp = Gp + (size_t)pair * nchunk * B2 * B2;
        double acc[TE];
#pragma unroll
        for (int k = 0; k < TE; ++k) acc[k] = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            T v[TE];
#pragma unroll
            for (int k = 0; k < TE; ++k) v[k] = gp[(size_t)c * B2 * B2 + tid + k * NT];
#pragma unroll
            for (int k = 0; k < TE; ++k) acc[k] += (double)v[k];
        }
#pragma unroll
        for (int k = 0; k < TE; ++k) {
            const int e = tid + k * NT, i = e % B2, j = e / B2;
            if (i <= j) { G[i * LD + j] = (T)acc[k]; G[j * LD + i] = (T)acc[k]; }
            W[i * LD + j] = (i == j) ? T(1) : T(0);
        }
    }
    __syncthreads();

    // 2. does any pair of the block need a rotation?  Also the largest
    // |g_pq| / sqrt(g_pp g_qq) of the block, kept per sweep as a diagnostic.
    int need = 0;
    float offmax = 0.f;
#pragma unroll
    for (int k = 0; k < TE; ++k) {
        const int e = tid + k * NT, p = e % B2, q = e / B2;
        if (p < q) {
            const double g = (double)G[p * LD + q];
            const double pq = (double)G[p * LD + p] * (double)G[q * LD + q];
            if (g * g > eps2 * pq) need = 1;
            if (pq > 0.0) offmax = fmaxf(offmax, (float)(fabs(g) / sqrt(pq)));
        }
    }
    offmax = wave_max(offmax);
    if ((tid & 63) == 0 && offmax > 0.f) atomicMax((unsigned int *)(flag + 1), __float_as_uint(offmax));
    need = block_or<NT>(need, ired);
    if (!need) {
        if (tid == 0) skip[pair] = 1;
        return;
    }
    if (tid == 0) { skip[pair] = 0; *flag = 1; }

    // 3. cyclic rounds of disjoint rotations on G, accumulating W = prod J
    float smax = 0.f;   // largest |sin| of the rotations this thread computed
    for (int sw = 0; sw < max_inner; ++sw) {
        __syncthreads();
        if (tid == 0) any_rot = 0;
        __syncthreads();
        for (int rd = 0; rd < B2 - 1; ++rd) {
            if (tid < H) {
                int p, q;
                rr_slot(B2, rd, tid, &p, &q);
                const double al = (double)G[p * LD + p], be = (double)G[q * LD + q];
                const double ga = (double)G[p * LD + q];
                double c = 1.0, s = 0.0, t = 0.0;
                if (ga * ga > eps2 * al * be) {
                    jac_rot(al, be, ga, &c, &s, &t);
                    any_rot = 1;
                    smax = fmaxf(smax, (float)fabs(s));
                }
                ca[p] = (T)c; cb[p] = (T)(-s);
                ca[q] = (T)c; cb[q] = (T)s;
                tt[tid] = (T)t;
            }
            __syncthreads();
            // G <- J^T G J on the 2x2 groups {p_a, q_a} x {p_b, q_b}, a <= b
            int gi[TG][2], gj[TG][2];
            T g[TG][2][2], ci[TG][2], si[TG][2], cj[TG][2], sj[TG][2];
            bool act[TG], diag[TG];
#pragma unroll
            for (int k = 0; k < TG; ++k) {
                const int e = tid + k * NT, a = e % H, bq = e / H;
                act[k] = a <= bq;
                diag[k] = a == bq;
                rr_slot(B2, rd, a, &gi[k][0], &gi[k][1]);
                rr_slot(B2, rd, bq, &gj[k][0], &gj[k][1]);
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    ci[k][x] = ca[gi[k][x]]; si[k][x] = cb[gi[k][x]];
                    cj[k][x] = ca[gj[k][x]]; sj[k][x] = cb[gj[k][x]];
#pragma unroll
                    for (int y = 0; y < 2; ++y) g[k][x][y] = G[gi[k][x] * LD + gj[k][y]];
                }
            }
            // W column pairs
            int wr[TW], wp[TW], wq[TW];
            T w0[TW], w1[TW], cp[TW], sp[TW], cq[TW], sq[TW];
#pragma unroll
            for (int k = 0; k < TW; ++k) {
                const int e = tid + k * NT;
                wr[k] = e % B2;
                rr_slot(B2, rd, e / B2, &wp[k], &wq[k]);
                w0[k] = W[wr[k] * LD + wp[k]]; w1[k] = W[wr[k] * LD + wq[k]];
                cp[k] = ca[wp[k]]; sp[k] = cb[wp[k]]; cq[k] = ca[wq[k]]; sq[k] = cb[wq[k]];
            }
            T tdiag[TG];
#pragma unroll
            for (int k = 0; k < TG; ++k) tdiag[k] = diag[k] ? tt[(tid + k * NT) % H] : T(0);
            // each G / W entry is read and written by the same thread within a
            // round, so no barrier is needed between the loads and the stores
#pragma unroll
            for (int k = 0; k < TG; ++k) {
                if (!act[k]) continue;
                if (diag[k]) {
                    const T t = tdiag[k], gpq = g[k][0][1];
                    if (t != T(0)) {
                        G[gi[k][0] * LD + gi[k][0]] = g[k][0][0] - t * gpq;
                        G[gi[k][1] * LD + gi[k][1]] = g[k][1][1] + t * gpq;
                        G[gi[k][0] * LD + gi[k][1]] = T(0);
                        G[gi[k][1] * LD + gi[k][0]] = T(0);
                    }
                    continue;
                }
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        const T o = ci[k][x] * cj[k][y] * g[k][x][y] + ci[k][x] * sj[k][y] * g[k][x][1 - y] +
                                    si[k][x] * cj[k][y] * g[k][1 - x][y] + si[k][x] * sj[k][y] * g[k][1 - x][1 - y];
                        G[gi[k][x] * LD + gj[k][y]] = o;
                        G[gj[k][y] * LD + gi[k][x]] = o;
                    }
            }
#pragma unroll
            for (int k = 0; k < TW; ++k) {
                W[wr[k] * LD + wp[k]] = cp[k] * w0[k] + sp[k] * w1[k];
                W[wr[k] * LD + wq[k]] = sq[k] * w0[k] + cq[k] * w1[k];
            }
            __syncthreads();
        }
        const int ar = any_rot;
        if (!ar) break;
    }

    smax = wave_max(smax);
    if ((tid & 63) == 0 && smax > 0.f) atomicMax((unsigned int *)(flag + 2), __float_as_uint(smax));

    // 4. write W (column-major)
    T *wo = Wm + (size_t)pair * B2 * B2;
#pragma unroll
    for (int k = 0; k < TE; ++k) {
        const int e = tid + k * NT, i = e % B2, j = e / B2;
        wo[e] = W[i * LD + j];
    }
}

// [Y_I Y_J] <- [Y_I Y_J] W (and V) on one row chunk: 32-row slabs through
// LDS, the next slab loaded into registers during the MFMA of the current one.
template <typename T, int B2>
__global__ __launch_bounds__(JR_NT) void jac_update(int N, int nblk, int r, T *__restrict__ Y,
                                                    int ldy, T *__restrict__ V, int ldv,
                                                    int nchY, const T *__restrict__ Wm,
                                                    const int *__restrict__ skip) {
    constexpr int b = B2 / 2;
    constexpr int NTJ = B2 / 16;                 // column tiles
    constexpr int NT = 2 * NTJ;                  // 2 row tiles (32 rows) x NTJ
    constexpr int TPW = NT / 4;
    constexpr int PER = B2 * JR_SLAB / JR_NT;
    __shared__ T Ws[B2][B2 + 1];
    __shared__ T Ps[B2][JR_SLAB + 1];
    const int pair = blockIdx.x;
    if (skip[pair]) return;
    int I, J;
    rr_slot(nblk, r, pair, &I, &J);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const T *wsrc = Wm + (size_t)pair * B2 * B2;
    for (int e = tid; e < B2 * B2; e += JR_NT) Ws[e % B2][e / B2] = wsrc[e];
    T *M;
    int ld, chunk;
    if ((int)blockIdx.y < nchY) { M = Y; ld = ldy; chunk = blockIdx.y; }
    else { M = V; ld = ldv; chunk = blockIdx.y - nchY; }
    const int rbeg = chunk * JR_RG, rend = min(N, rbeg + JR_RG);
    typedef typename acc4<T>::type V4;
    T pf[PER];
    auto fetch = [&](int r0) {
#pragma unroll
        for (int e0 = 0; e0 < PER; ++e0) {
            const int e = tid + e0 * JR_NT;
            const int c = e / JR_SLAB, rr = e % JR_SLAB;
            const int gi = r0 + rr;
            pf[e0] = gi < rend ? M[(size_t)blk_col(c, b, I, J) * ld + gi] : T(0);
        }
    };
    fetch(rbeg);
    for (int r0 = rbeg; r0 < rend; r0 += JR_SLAB) {
        __syncthreads();
#pragma unroll
        for (int e0 = 0; e0 < PER; ++e0) {
            const int e = tid + e0 * JR_NT;
            Ps[e / JR_SLAB][e % JR_SLAB] = pf[e0];
        }
        __syncthreads();
        if (r0 + JR_SLAB < rend) fetch(r0 + JR_SLAB);
        V4 acc[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) acc[q] = V4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < B2; kk += 4) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                const int tile = w + 4 * q;
                const int ti = tile % 2, tj = tile / 2;
                const T a = Ps[kk + lane / 16][16 * ti + lane % 16];
                const T bb = Ws[kk + lane / 16][16 * tj + lane % 16];
                acc[q] = mfma16(a, bb, acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = w + 4 * q;
            const int ti = tile % 2, tj = tile / 2;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * ti + mfma_row<T>(lane, e);
                const int j = 16 * tj + lane % 16;
                const int gi = r0 + i;
                if (gi < rend) M[(size_t)blk_col(j, b, I, J) * ld + gi] = acc[q][e];
            }
        }
    }
}

size_t jacobi_scratch_bytes(int N, int b, int elem) {
    const int B2 = 2 * b;
    const int npairs = N / B2;
    const int nch = cdiv(N, JR_RGG);
    size_t bytes = (size_t)npairs * nch * B2 * B2 * elem;   // gram partials
    bytes += (size_t)npairs * B2 * B2 * elem;                // W blocks
    bytes += (size_t)npairs * sizeof(int) + 256;             // skip flags
    bytes += 256;                                             // flag
    return bytes + 1024;
}

void jacobi_carve(JacobiWork &jw, char *base, int N, int b, int elem) {
    const int B2 = 2 * b;
    const int npairs = N / B2;
    const int nch = cdiv(N, JR_RGG);
    char *p = base;
    jw.gram = p; p += (size_t)npairs * nch * B2 * B2 * elem;
    jw.wmat = p; p += (size_t)npairs * B2 * B2 * elem;
    jw.skip = (int *)p; p += (size_t)npairs * sizeof(int) + 256;
    jw.flag = (int *)p;
}

template <typename T, int B2, int INNER_NT>
static int sweeps_impl(hipStream_t s, int N, T *Y, T *V, double eps, int maxsweep, int max_inner,
                       JacobiWork &jw, int *conv) {
    constexpr int b = B2 / 2;
    const int nblk = N / b;
    const int npairs = nblk / 2;
    const int nch = cdiv(N, JR_RG);
    const int nchG = cdiv(N, JR_RGG);
    const int nchV = V ? nch : 0;
    *conv = 0;
    int sw = 0;
    for (; sw < maxsweep; ++sw) {
        hipError_t e = hipMemsetAsync(jw.flag, 0, 3 * sizeof(int), s);
        if (e != hipSuccess) { note_hip_error(e, "jacobi flag reset"); return -1; }
        // kernel-class ids for the optional per-launch clock
        const int kbase = sizeof(T) == 4 ? 0 : 3;
        const double E = sizeof(T);
        const double gram_bytes = (double)N * N * E;                      // Y read once
        const double upd_bytes = 2.0 * (double)N * N * E * (V ? 2 : 1);   // Y (and V) read + written
        for (int r = 0; r < nblk - 1; ++r) {
            if (jw.kc) jw.kc->begin(s, kbase + 0, gram_bytes);
            hipLaunchKernelGGL((jac_gram<T, B2>), dim3(npairs, nchG), dim3(JR_NT), 0, s, N, nblk, r, Y,
                               N, (T *)jw.gram, nchG);
            if (jw.kc) { jw.kc->end(s); jw.kc->begin(s, kbase + 1, 0.0); }
            hipLaunchKernelGGL((jac_inner<T, B2, INNER_NT>), dim3(npairs), dim3(INNER_NT), 0, s, nchG,
                               (const T *)jw.gram, (T *)jw.wmat, jw.skip, jw.flag, eps, max_inner);
            if (jw.kc) { jw.kc->end(s); jw.kc->begin(s, kbase + 2, upd_bytes); }
            hipLaunchKernelGGL((jac_update<T, B2>), dim3(npairs, nch + nchV), dim3(JR_NT), 0, s, N,
                               nblk, r, Y, N, V, N, nch, (const T *)jw.wmat, jw.skip);
            if (jw.kc) jw.kc->end(s);
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(jw.hflag, jw.flag, 3 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { note_hip_error(e, "jacobi sweep"); return -1; }
        if (jw.kc) jw.kc->collect();
        float off, smx;
        memcpy(&off, jw.hflag + 1, sizeof(float));
        memcpy(&smx, jw.hflag + 2, sizeof(float));
        if (jw.off_hist && sw < 32) jw.off_hist[sw] = off;
        // Algorithm 1's rule: a sweep without rotations
        if (*jw.hflag == 0) { *conv = 1; ++sw; break; }
        // xGESVJ's rule: the remaining off-diagonal is within sqrt(n) of the
        // tolerance and the rotations of the sweep were too small to matter
        const double nn = jw.n_real;
        if ((double)off < sqrt(nn) * eps && nn * (double)off * (double)smx < eps) {
            *conv = 1; ++sw; break;
        }
        if (jw.stop_off > 0.0 && off <= jw.stop_off) { *conv = 1; ++sw; break; }
    }
    return sw;
}

template <typename T>
int jacobi_sweeps(hipStream_t s, int N, int b, T *Y, T *V, double eps, int maxsweep, int max_inner,
                  JacobiWork &jw, int *conv) {
    if (b == 16) return sweeps_impl<T, 32, 256>(s, N, Y, V, eps, maxsweep, max_inner, jw, conv);
    return sweeps_impl<T, 64, 1024>(s, N, Y, V, eps, maxsweep, max_inner, jw, conv);
}

template int jacobi_sweeps<float>(hipStream_t, int, int, float *, float *, double, int, int,
                                  JacobiWork &, int *);
template int jacobi_sweeps<double>(hipStream_t, int, int, double *, double *, double, int, int,
                                   JacobiWork &, int *);

} // namespace mpj
