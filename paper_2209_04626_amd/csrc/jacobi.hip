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
#include <hip/hip_ext.h>

#include <atomic>

#include <utility>
#include <vector>

#include "../../include/mpjsvd.h"
#include "common.hpp"
#include "internal.hpp"

namespace mpj {

constexpr int JR_NT = 256;   // threads per workgroup

constexpr int JU_RG = 256;   // rows per workgroup of the update

constexpr int JF_MAX_WG = 512;      // workgroups of a fused FP32 round
constexpr int JF_MAX_G = 16;        // workgroups per pair slot
constexpr int JF_MAX_TILES = 10;    // upper 16 x 16 tiles of a 64-wide block
constexpr int JF_SPIN = 1 << 22;    // default polls of the fused round's wait

// Rows per workgroup of the Gram kernels: a quarter of N in whole 64-row
// stripes, between 256 and 1024.  Each workgroup writes one partial Gram
// block that the inner solve reduces, so long chunks save the reduction and
// the per-workgroup set-up (at n = 4096: 4 partials per pair instead of 16);
// the lower bound keeps enough workgroups in flight for small N.
inline int gram_rows(int N) {
    const int rg = (N / 4) / 64 * 64;
    return rg < 256 ? 256 : (rg > 1024 ? 1024 : rg);
}
inline int gram_chunks(int N) { return cdiv(N, gram_rows(N)); }

__device__ __forceinline__ int blk_col(int c, int b, int I, int J) {
    return c < b ? I * b + c : J * b + (c - b);
}

// Partial Gram blocks.  Only the 16 x 16 tiles on or above the block
// diagonal are formed (G is symmetric; the inner solve reads the upper
// triangle), one partial block per row chunk.
//
// FP32 partial Gram block without staging the columns in LDS.  Each
// wavefront owns 64-row stripes of the chunk.  Lane (g, i) of the wavefront
// (g = lane / 16, i = lane % 16) reads, for every 16-column tile h of the pair
// and u = 0..3, rows 16 u + 4 g .. + 3 of column 16 h + i as one 16-byte
// vector; element t of it is row k = (u, t) of the MFMA step for both
// operands, so the A and B operands of every tile come straight from these
// registers (the MFMA sums over k in any order).  All four wavefronts form
// every tile on or above the block diagonal over their own rows; the four
// partial tiles are then summed in a fixed order through LDS.
template <int B2>
__global__ __launch_bounds__(JR_NT) void jac_gram_f32(int N, int nblk, int r, const float *__restrict__ Y,
                                                      int ldy, float *__restrict__ Gp, int nchunk, int RG,
                                                      const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr int b = B2 / 2;
    constexpr int NTT = B2 / 16;                       // tiles per dimension
    constexpr int NUT = NTT * (NTT + 1) / 2;           // upper-triangle tiles
    __shared__ float red[4][NUT][256];
    const int pair = blockIdx.x, chunk = blockIdx.y;
    int I, J;
    rr_slot(nblk, r, pair, &I, &J);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, li = lane & 15;
    const float *col[NTT];
#pragma unroll
    for (int h = 0; h < NTT; ++h) col[h] = Y + (size_t)blk_col(16 * h + li, b, I, J) * ldy + 4 * g;
    flt4 acc[NUT];
#pragma unroll
    for (int q = 0; q < NUT; ++q) acc[q] = flt4{0, 0, 0, 0};
    const int rbeg = chunk * RG, rend = min(N, rbeg + RG);
    for (int r0 = rbeg + 64 * w; r0 + 64 <= rend; r0 += 64 * (JR_NT / 64)) {
        flt4 v[NTT][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int h = 0; h < NTT; ++h) v[h][u] = *(const flt4 *)(col[h] + r0 + 16 * u);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                int q = 0;
#pragma unroll
                for (int ta = 0; ta < NTT; ++ta)
#pragma unroll
                    for (int tc = ta; tc < NTT; ++tc, ++q) acc[q] = mfma16(v[ta][u][t], v[tc][u][t], acc[q]);
            }
    }
    // lane l, element e of tile q holds G entry (4 (l / 16) + e, l % 16) of q
#pragma unroll
    for (int q = 0; q < NUT; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[w][q][lane * 4 + e] = acc[q][e];
    __syncthreads();
    float *out = Gp + ((size_t)pair * nchunk + chunk) * B2 * B2;
    for (int idx = tid; idx < NUT * 256; idx += JR_NT) {
        const int q = idx >> 8, jl = (idx >> 4) & 15, il = idx & 15;
        int ta = 0, qq = q;
        while (qq >= NTT - ta) { qq -= NTT - ta; ++ta; }
        const int tc = ta + qq;
        const int src = ((il >> 2) * 16 + jl) * 4 + (il & 3);
        const float s = ((red[0][q][src] + red[1][q][src]) + red[2][q][src]) + red[3][q][src];
        out[(16 * ta + il) + (16 * tc + jl) * B2] = s;
    }
}

// FP64 partial Gram block in the same register-direct form: a stripe is 32
// rows, lane (g, i) reads rows 8 u + 2 g, + 1 of column 16 h + i as one
// 16-byte vector (u = 0..3), and element t is row k = (u, t) of the MFMA step
// for both operands.  Every wavefront forms all upper tiles over its own
// rows (an even split of the MFMA work); the four partial tiles are added in
// wavefront order through one LDS buffer.
template <int B2>
__global__ __launch_bounds__(JR_NT) void jac_gram_f64(int N, int nblk, int r, const double *__restrict__ Y,
                                                      int ldy, double *__restrict__ Gp, int nchunk, int RG,
                                                      const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr int b = B2 / 2;
    constexpr int NTT = B2 / 16;                       // tiles per dimension
    constexpr int NUT = NTT * (NTT + 1) / 2;           // upper-triangle tiles
    typedef double d2 __attribute__((ext_vector_type(2)));
    __shared__ double red[NUT][256];
    const int pair = blockIdx.x, chunk = blockIdx.y;
    int I, J;
    rr_slot(nblk, r, pair, &I, &J);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, li = lane & 15;
    const double *col[NTT];
#pragma unroll
    for (int h = 0; h < NTT; ++h) col[h] = Y + (size_t)blk_col(16 * h + li, b, I, J) * ldy + 2 * g;
    dbl4 acc[NUT];
#pragma unroll
    for (int q = 0; q < NUT; ++q) acc[q] = dbl4{0, 0, 0, 0};
    const int rbeg = chunk * RG, rend = min(N, rbeg + RG);
    for (int r0 = rbeg + 32 * w; r0 + 32 <= rend; r0 += 32 * (JR_NT / 64)) {
        d2 v[NTT][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int h = 0; h < NTT; ++h) v[h][u] = *(const d2 *)(col[h] + r0 + 8 * u);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                int q = 0;
#pragma unroll
                for (int ta = 0; ta < NTT; ++ta)
#pragma unroll
                    for (int tc = ta; tc < NTT; ++tc, ++q) acc[q] = mfma16(v[ta][u][t], v[tc][u][t], acc[q]);
            }
    }
    // lane l, element e of tile q holds G entry (l / 16 + 4 e, l % 16) of q;
    // the partials are summed as ((w0 + w1) + w2) + w3
#pragma unroll
    for (int wv = 0; wv < 4; ++wv) {
        if (w == wv) {
#pragma unroll
            for (int q = 0; q < NUT; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    red[q][lane * 4 + e] = wv == 0 ? acc[q][e] : red[q][lane * 4 + e] + acc[q][e];
        }
        __syncthreads();
    }
    double *out = Gp + ((size_t)pair * nchunk + chunk) * B2 * B2;
    for (int idx = tid; idx < NUT * 256; idx += JR_NT) {
        const int q = idx >> 8, jl = (idx >> 4) & 15, il = idx & 15;
        int ta = 0, qq = q;
        while (qq >= NTT - ta) { qq -= NTT - ta; ++ta; }
        const int tc = ta + qq;
        out[(16 * ta + il) + (16 * tc + jl) * B2] = red[q][((il & 3) * 16 + jl) * 4 + (il >> 2)];
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

// 1/sqrt(x) and 1/x for x > 0 in FP64 from the hardware estimates refined by
// NR Newton steps (each squares the relative error): two give FP64 accuracy,
// one is ample when the rotation is rounded to FP32 afterwards.
template <int NR>
__device__ __forceinline__ double rsq64(double x) {
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
#pragma unroll
    for (int i = 0; i < NR; ++i) r = r * fma(-h * r, r, 1.5);
    return r;
}
template <int NR>
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int i = 0; i < NR; ++i) r = r * fma(-x, r, 2.0);
    return r;
}

// The same rotation from d = beta - alpha and g2 = 2 gamma without forming
// zeta: t = sign(zeta) |g2| / (|d| + sqrt(d^2 + g2^2)), c = 1/sqrt(1 + t^2),
// s = t c, with the square roots and the quotient from refined hardware
// estimates.  Returns false, with the identity, when the pair passes the test
// g^2 <= eps^2 g_pp g_qq of Algorithm 1, and when g_pp g_qq is not positive:
// in exact arithmetic a zero column has g_pq = 0, and a product that rounded
// to zero (squares below the format's range) must not rotate for ever.
template <int NR>
__device__ __forceinline__ bool jac_rot_test(double al, double be, double ga, double eps2,
                                             double *c, double *s, double *t) {
    if (!(ga * ga > eps2 * al * be) || !(al * be > 0.0)) {
        *c = 1.0; *s = 0.0; *t = 0.0;
        return false;
    }
    const double d = be - al, g2 = 2.0 * ga;
    double tt;
    if (d == 0.0) {
        tt = 1.0;
    } else if (fabs(d) < 1e150 && fabs(g2) < 1e150) {
        const double h = fma(d, d, g2 * g2);
        const double rh = rsq64<NR>(h);
        double y = h * rh;                            // sqrt(h)
        y = fma(0.5 * rh, fma(-y, y, h), y);
        const double den = fabs(d) + y;
        const double num = copysign(1.0, d) * g2;
        tt = num * rcp64<NR>(den);
    } else {
        double cc, ss;
        jac_rot(al, be, ga, &cc, &ss, &tt);
    }
    const double cc = rsq64<NR>(fma(tt, tt, 1.0));
    *t = tt; *c = cc; *s = tt * cc;
    return true;
}

template <typename T, int B2, int NT, int NTW, bool CROSS>
__device__ __forceinline__ float inner_rounds_t(T (*G)[B2 * (B2 + 1)], T *W, int *ired, double eps2,
                                                int max_inner, unsigned rmask) {
    constexpr int LD = B2 + 1;
    constexpr int H = B2 / 2;
    constexpr int M = B2 - 1;
    constexpr int CG = NTW / H;           // thread groups along c
    constexpr int GPT = H / CG;           // 2x2 groups per thread
    constexpr int RPT = B2 / CG;          // W rows per thread
    constexpr int NRS = sizeof(T) == 4 ? 1 : 2;
    static_assert(CG * H == NTW && GPT * CG == H && RPT * CG == B2, "tiling");
    static_assert(64 % H == 0 && NTW % 64 == 0 && NTW <= NT, "every wavefront holds every pair index");
    static_assert((H & (H - 1)) == 0, "cross rounds index the second block modulo H");
    const int tid = threadIdx.x;
    // threads from NTW on (whole wavefronts) only keep step with the barriers
    const bool work = NTW == NT || tid < NTW;
    const int a = tid % H, cg = tid / H;
    const int c0 = cg * GPT, w0 = cg * RPT;
    const bool own_diag = a / GPT == cg;      // this thread holds group (a, a)
    const int kd = a % GPT;
    // schedule positions of pair a and of the thread's pairs c at round 0
    int ax = a, ay = CROSS ? H + a : (a == 0 ? M : M - a);
    int cx[GPT], cy[GPT];
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
        const int c = c0 + k;
        cx[k] = c;
        cy[k] = CROSS ? H + c : (c == 0 ? M : M - c);
    }
    // Between the two blocks, pair a always rotates column a of the first
    // block: its rows of W's column a, its entries (a, c) of G and g_aa stay
    // in registers for the whole solve (only this thread writes them; every
    // thread of pair a updates g_aa identically).  Those LDS copies go stale.
    T wpr[RPT], greg[GPT];
    double alp_r = 0.0;
    if (CROSS && work) {
#pragma unroll
        for (int j = 0; j < RPT; ++j) wpr[j] = W[(w0 + j) * LD + a];
#pragma unroll
        for (int k = 0; k < GPT; ++k) greg[k] = G[0][a * LD + c0 + k];
        alp_r = (double)G[0][a * LD + a];
    }
    const int nround = CROSS ? H : M;
    float smax = 0.f;   // largest |sin| of the rotations of pair a (owner only)
    int cur = 0;
    for (int sw = 0; sw < max_inner; ++sw) {
        int rotated = 0;
        for (int rd = 0; rd < nround; ++rd) {
          if constexpr (CROSS) {
            // a round none of whose pairs needed a rotation when the block
            // was tested is left out of the first cycle (rmask is the same
            // in every thread, so the barriers still match)
            if (sw == 0 && !((rmask >> rd) & 1u)) continue;
            ay = H + ((a + rd) & (H - 1));
#pragma unroll
            for (int k = 0; k < GPT; ++k) cy[k] = H + ((c0 + k + rd) & (H - 1));
          }
          if (work) {
            const T *g = G[cur];
            T *gn = G[cur ^ 1];
            const int p = min(ax, ay), q = max(ax, ay);
            const double alp = CROSS ? alp_r : (double)g[p * LD + p];
            const double bep = (double)g[q * LD + q];
            const double gap = (double)g[p * LD + q];
            int r[GPT], s[GPT];
            T blk[GPT][4];
#pragma unroll
            for (int k = 0; k < GPT; ++k) {
                r[k] = min(cx[k], cy[k]);
                s[k] = max(cx[k], cy[k]);
                blk[k][0] = CROSS ? greg[k] : g[p * LD + r[k]];
                blk[k][1] = g[p * LD + s[k]];
                blk[k][2] = g[q * LD + r[k]]; blk[k][3] = g[q * LD + s[k]];
            }
            T wp[RPT], wq[RPT];
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                wp[j] = CROSS ? wpr[j] : W[(w0 + j) * LD + p];
                wq[j] = W[(w0 + j) * LD + q];
            }
            double ca, sa, ta;
            const bool ra = jac_rot_test<NRS>(alp, bep, gap, eps2, &ca, &sa, &ta);
            if (own_diag && ra) {
                rotated = 1;
                smax = fmaxf(smax, (float)fabs(sa));
            }
            const T c1 = (T)ca, s1 = (T)sa;
            // the rotations of this thread's pairs c, from their lanes (all
            // in flight while W is updated)
            T cc2[GPT], ss2[GPT];
#pragma unroll
            for (int k = 0; k < GPT; ++k) {
                cc2[k] = __shfl(c1, c0 + k, 64);
                ss2[k] = __shfl(s1, c0 + k, 64);
            }
            // W <- W J on the column pair (p, q): x_p' = c x_p - s x_q, x_q' = s x_p + c x_q
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const T np_ = c1 * wp[j] - s1 * wq[j];
                if constexpr (CROSS) wpr[j] = np_;
                else W[(w0 + j) * LD + p] = np_;
                W[(w0 + j) * LD + q] = s1 * wp[j] + c1 * wq[j];
            }
            // G <- J^T G J on the groups: rows (p, q) by pair a, columns (r, s) by pair c
#pragma unroll
            for (int k = 0; k < GPT; ++k) {
                const T c2 = cc2[k], s2 = ss2[k];
                const T h00 = c1 * blk[k][0] - s1 * blk[k][2], h01 = c1 * blk[k][1] - s1 * blk[k][3];
                const T h10 = s1 * blk[k][0] + c1 * blk[k][2], h11 = s1 * blk[k][1] + c1 * blk[k][3];
                T o00 = c2 * h00 - s2 * h01, o01 = s2 * h00 + c2 * h01;
                T o10 = c2 * h10 - s2 * h11, o11 = s2 * h10 + c2 * h11;
                if (own_diag && k == kd && ra) {
                    // the diagonal group: the rotation zeroes g_pq exactly
                    o00 = (T)(alp - ta * gap);
                    o11 = (T)(bep + ta * gap);
                    o01 = T(0); o10 = T(0);
                }
                if constexpr (CROSS) greg[k] = o00;
                else gn[p * LD + r[k]] = o00;
                gn[p * LD + s[k]] = o01;
                gn[q * LD + r[k]] = o10; gn[q * LD + s[k]] = o11;
            }
            if constexpr (CROSS) {
                if (ra) alp_r = (double)(T)(alp - ta * gap);
            }
          }
            __syncthreads();
            cur ^= 1;
            if constexpr (!CROSS) {
                // next round: every schedule position advances by one (mod
                // 2b-1), except the fixed partner 2b-1 of pair 0
                ax = ax + 1 == M ? 0 : ax + 1;
                if (a != 0) ay = ay + 1 == M ? 0 : ay + 1;
#pragma unroll
                for (int k = 0; k < GPT; ++k) {
                    cx[k] = cx[k] + 1 == M ? 0 : cx[k] + 1;
                    if (c0 + k != 0) cy[k] = cy[k] + 1 == M ? 0 : cy[k] + 1;
                }
            }
        }
        // positions after a full cycle are back where they started
        if (!block_or<NT>(rotated, ired)) break;
    }
    if constexpr (CROSS) {
        if (work) {
#pragma unroll
            for (int j = 0; j < RPT; ++j) W[(w0 + j) * LD + a] = wpr[j];
        }
        __syncthreads();
    }
    return smax;
}

// Cyclic rounds of disjoint rotations on the 2b x 2b block G (LDS, row
// stride B2 + 1, double-buffered: G[0] holds the symmetric block on entry),
// accumulating W = prod J (LDS, the identity on entry), until a full cycle
// rotates nothing or max_inner cycles have run.  Round rd rotates the column
// pairs of the round-robin schedule (pair k joins (rd + k) mod (2b-1) and
// (rd - k) mod (2b-1); pair 0 joins rd and 2b-1); 2b - 1 rounds reach every
// pair of the 2b columns.  With cross set, only the b^2 pairs between the two
// blocks are rotated: round rd joins column k of the first block with column
// (k + rd) mod b of the second, b rounds, and round rd is left out of the
// first cycle when bit rd of rmask is clear (the caller clears the rounds none
// of whose pairs needed a rotation when the block was tested; a pair of such
// a round that rotations of earlier rounds push over the threshold waits for
// the next sweep, which tests it on a fresh Gram block).  Thread (a, g) computes the rotation
// of pair a from the current G and owns the 2x2 groups {p_a, q_a} x {p_c, q_c}
// of G for its GPT pairs c (the groups tile G) and RPT rows of W's column
// pair a.  Pair c's rotation comes from the lane of the same wavefront whose
// pair is c (every wavefront holds every pair index), so a round reads G from
// one LDS buffer, writes the rotated G to the other, and needs a single
// barrier; no thread branches on its role.  Every thread of the workgroup
// calls it; only the first NTW threads work, the rest (whole wavefronts) keep
// step with the barriers.  Returns the largest |sin| of the rotations of this
// thread's pair (0 for threads that do not own a diagonal group).  W is
// complete in LDS on return; G is not (with cross set, part of it was kept in
// registers).
template <typename T, int B2, int NT, int NTW = NT>
__device__ __forceinline__ float inner_rounds(T (*G)[B2 * (B2 + 1)], T *W, int *ired, double eps2,
                                              int max_inner, int cross, unsigned rmask) {
    return cross ? inner_rounds_t<T, B2, NT, NTW, true>(G, W, ired, eps2, max_inner, rmask)
                 : inner_rounds_t<T, B2, NT, NTW, false>(G, W, ired, eps2, max_inner, rmask);
}

// Inner solve of one block pair.  G and the accumulated W are held in the
// stage's precision T (FP32 in the FP32 stage, FP64 in the FP64 stage); every
// rotation angle and threshold test is evaluated in FP64.  The partial Gram
// blocks of the pair are reduced into G, the pairs are tested, and when any
// needs it the rotation rounds of inner_rounds produce W, written out for the
// update.
template <typename T, int B2, int NT>
__global__ __launch_bounds__(NT) void jac_inner(int nchunk, const T *__restrict__ Gp,
                                                T *__restrict__ Wm, int *skip, int *flag,
                                                float *offp, float *smxp, int *rot, double eps,
                                                int max_inner, int cross, const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr int LD = B2 + 1;
    constexpr int H = B2 / 2;
    constexpr int TE = (B2 * B2) / NT;    // Gram entries per thread (set-up)
    static_assert(TE * NT == B2 * B2, "tiling");
    __shared__ T G[2][B2 * LD];
    __shared__ T W[B2 * LD];
    __shared__ int ired[NT / 64];
    const int pair = blockIdx.x, tid = threadIdx.x;
    const double eps2 = eps * eps;

    // 1. reduce the partial Gram blocks (fixed chunk order, FP64 sums).  For
    // the 64-wide block only the upper triangle is read (the Gram kernel
    // writes the tiles on and above the diagonal) with all loads of a thread
    // in flight together; the 32-wide block reads whole blocks, coalesced,
    // four chunks at a time (measured faster there).
    constexpr int NUP = B2 * (B2 + 1) / 2;
    constexpr bool UPPER = B2 >= 64;
    constexpr int UE = UPPER ? (NUP + NT - 1) / NT : TE;
    constexpr int MAXC = 16;
    int ui[UE], uj[UE];
    bool uok[UE];
    {
        const T *gp = Gp + (size_t)pair * nchunk * B2 * B2;
        double acc[UE];
#pragma unroll
        for (int k = 0; k < UE; ++k) {
            if constexpr (UPPER) {
                const int u = min(tid + k * NT, NUP - 1);
                int j = (int)((sqrtf(8.f * u + 1.f) - 1.f) * 0.5f);
                while (j * (j + 1) / 2 > u) --j;
                while ((j + 1) * (j + 2) / 2 <= u) ++j;
                uj[k] = j;
                ui[k] = u - j * (j + 1) / 2;
                uok[k] = tid + k * NT < NUP;
            } else {
                const int e = tid + k * NT;
                ui[k] = e % B2;
                uj[k] = e / B2;
                uok[k] = ui[k] <= uj[k];
            }
            acc[k] = 0.0;
        }
        if (UPPER && nchunk <= MAXC) {
            T v[MAXC][UE];
#pragma unroll
            for (int c = 0; c < MAXC; ++c)
#pragma unroll
                for (int k = 0; k < UE; ++k)
                    v[c][k] = c < nchunk ? gp[(size_t)c * B2 * B2 + ui[k] + uj[k] * B2] : T(0);
#pragma unroll
            for (int c = 0; c < MAXC; ++c)
#pragma unroll
                for (int k = 0; k < UE; ++k) acc[k] += (double)v[c][k];
        } else {
            int c = 0;
            for (; c + 4 <= nchunk; c += 4) {
                T v[4][UE];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int k = 0; k < UE; ++k)
                        v[u][k] = gp[(size_t)(c + u) * B2 * B2 + ui[k] + uj[k] * B2];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int k = 0; k < UE; ++k) acc[k] += (double)v[u][k];
            }
            for (; c < nchunk; ++c)
#pragma unroll
                for (int k = 0; k < UE; ++k)
                    acc[k] += (double)gp[(size_t)c * B2 * B2 + ui[k] + uj[k] * B2];
        }
#pragma unroll
        for (int k = 0; k < UE; ++k) {
            if (uok[k]) {
                G[0][ui[k] * LD + uj[k]] = (T)acc[k];
                G[0][uj[k] * LD + ui[k]] = (T)acc[k];
            }
        }
#pragma unroll
        for (int k = 0; k < TE; ++k) {
            const int e = tid + k * NT, i = e % B2, j = e / B2;
            W[i * LD + j] = (i == j) ? T(1) : T(0);
        }
    }
    __syncthreads();

    // 2. does any pair of the block need a rotation?  Also the largest
    // |g_pq| / sqrt(g_pp g_qq) of the block, kept per sweep as a diagnostic.
    // With cross set, `need` holds the cross rounds (bit (q - p) mod b for
    // the pair p < b <= q) that have a pair to rotate.
    int need = 0;
    float offmax = 0.f;
#pragma unroll
    for (int k = 0; k < UE; ++k) {
        const int p = ui[k], q = uj[k];
        if (uok[k] && p < q) {
            const double g = (double)G[0][p * LD + q];
            const double pq = (double)G[0][p * LD + p] * (double)G[0][q * LD + q];
            if (g * g > eps2 * pq && pq > 0.0) {
                if (!cross) need = 1;
                else if (p < H && q >= H) need |= (int)(1u << ((q - H - p) & (H - 1)));
            }
            if (pq > 0.0) offmax = fmaxf(offmax, (float)(fabs(g) / sqrt(pq)));
        }
    }
    // The per-sweep maxima and the rotated-pair map are kept per pair slot
    // (this workgroup is the slot's only writer in a launch, and rounds are
    // ordered launches), so no two workgroups touch the same word: atomics
    // on one shared word cost several microseconds per launch here.
    __shared__ float wmx[NT / 64], wsm[NT / 64];
    offmax = wave_max(offmax);
    if ((tid & 63) == 0) wmx[tid >> 6] = offmax;
    need = block_or<NT>(need, ired);
    const unsigned rmask = cross ? (unsigned)need : ~0u;
    if (tid == 0) {
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) m = fmaxf(m, wmx[q]);
        if (m > offp[pair]) offp[pair] = m;
        skip[pair] = need ? 0 : 1;
        rot[pair] = need ? 1 : 0;
        if (need) *flag = 1;
    }
    if (!need) return;

    // 3. cyclic rounds of disjoint rotations on G, accumulating W = prod J
    float smax = inner_rounds<T, B2, NT>(G, W, ired, eps2, max_inner, cross, rmask);

    smax = wave_max(smax);
    if ((tid & 63) == 0) wsm[tid >> 6] = smax;
    __syncthreads();
    if (tid == 0) {
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) m = fmaxf(m, wsm[q]);
        if (m > smxp[pair]) smxp[pair] = m;
    }

    // 4. write W (column-major)
    T *wo = Wm + (size_t)pair * B2 * B2;
#pragma unroll
    for (int k = 0; k < TE; ++k) {
        const int e = tid + k * NT, i = e % B2, j = e / B2;
        wo[e] = W[i * LD + j];
    }
}

// FP32 update without LDS.  Each wavefront owns a 64-row stripe of the
// chunk and forms its transpose, [Y_I Y_J]^T <- W^T [Y_I Y_J]^T, on the matrix
// cores: W^T is the A operand (held in registers for the whole launch) and the
// stripe, read as 16-byte vectors, the B operand.  The MFMA sums over k in
// any order, and its column index is free as well: lane j of a 16-lane group
// reads rows 4j..4j+3 of one column, and element t of that vector feeds the
// product of column tile t (stripe rows 4j + t).  With the FP32 accumulator
// layout (lane l holds rows 4 (l / 16) + e of column l % 16) lane l ends up
// with rows 4 (l % 16) .. + 3 of output columns 4 (l / 16) + e, so both the
// reads and the writes cover 256 contiguous bytes of a column per 16 lanes.
// The k index of step s on lane group g is column (B2/4) g + s, which keeps
// each lane's W entries contiguous (two 16-byte reads per 16-column tile).
// Requires N a multiple of 64 (whole stripes) and 16-byte aligned columns.
template <int B2>
__global__ __launch_bounds__(JR_NT) void jac_update_f32(int N, int nblk, int r, float *__restrict__ Y,
                                                        int ldy, float *__restrict__ V, int ldv,
                                                        int nchY, const float *__restrict__ Wm,
                                                        const int *__restrict__ skip,
                                                        const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr int b = B2 / 2, KS = B2 / 4, NTI = B2 / 16;
    static_assert(KS % 4 == 0 && b % KS == 0, "k mapping");
    const int pair = blockIdx.x;
    if (skip[pair]) return;
    int I, J;
    rr_slot(nblk, r, pair, &I, &J);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    float *M;
    int ld, chunk;
    if ((int)blockIdx.y < nchY) { M = Y; ld = ldy; chunk = blockIdx.y; }
    else { M = V; ld = ldv; chunk = blockIdx.y - nchY; }
    const int rbeg = chunk * JU_RG, rend = min(N, rbeg + JU_RG);
    // A operand: wr[ti][s] = W[KS g + s][16 ti + li] (W column-major, B2 x B2)
    const float *wsrc = Wm + (size_t)pair * B2 * B2;
    float wr[NTI][KS];
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
        for (int s4 = 0; s4 < KS / 4; ++s4) {
            const flt4 v = *(const flt4 *)(wsrc + (size_t)(16 * ti + li) * B2 + KS * g + 4 * s4);
#pragma unroll
            for (int q = 0; q < 4; ++q) wr[ti][4 * s4 + q] = v[q];
        }
    // lane group g reads columns KS g .. KS g + KS - 1 of the pair, all in
    // one of the two blocks
    const int c0 = KS * g;
    const float *ag = M + (size_t)(c0 < b ? I * b + c0 : J * b + c0 - b) * ld;
    for (int r0 = rbeg + 64 * w; r0 + 64 <= rend; r0 += 64 * (JR_NT / 64)) {
        flt4 a[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) a[s] = *(const flt4 *)(ag + (size_t)s * ld + r0 + 4 * li);
        flt4 acc[4][NTI];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int ti = 0; ti < NTI; ++ti) acc[t][ti] = flt4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int ti = 0; ti < NTI; ++ti) acc[t][ti] = mfma16(wr[ti][s], a[s][t], acc[t][ti]);
#pragma unroll
        for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = 16 * ti + 4 * g + e;
                *(flt4 *)(M + (size_t)blk_col(c, b, I, J) * ld + r0 + 4 * li) =
                    flt4{acc[0][ti][e], acc[1][ti][e], acc[2][ti][e], acc[3][ti][e]};
            }
    }
}

// FP64 update in the same transposed form: W^T (the A operand) is read from
// LDS, the stripe (the B operand) straight from 16-byte loads.  A stripe is
// 32 rows: lane j of a 16-lane group reads rows 2j, 2j + 1 of one column, and
// element t feeds column tile t of the product.  With the FP64 accumulator
// layout (lane l holds rows l / 16 + 4 e of column l % 16), lane l ends up
// with rows 2 (l % 16), + 1 of output columns l / 16 + 4 e: 256 contiguous
// bytes per column per 16 lanes, read and written.
typedef double dbl2 __attribute__((ext_vector_type(2)));
template <int B2>
__global__ __launch_bounds__(JR_NT, 2) void jac_update_f64(int N, int nblk, int r, double *__restrict__ Y,
                                                        int ldy, double *__restrict__ V, int ldv,
                                                        int nchY, const double *__restrict__ Wm,
                                                        const int *__restrict__ skip,
                                                        const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr int b = B2 / 2, KS = B2 / 4, NTI = B2 / 16, LDW = B2 + 1;
    constexpr int RG = JU_RG;
    constexpr int TP = NTI > 2 ? 2 : NTI;
    static_assert(b % KS == 0, "k mapping");
    __shared__ double Ws[B2 * LDW];   // Ws[j LDW + k] = W[k][j]
    const int pair = blockIdx.x;
    if (skip[pair]) return;
    int I, J;
    rr_slot(nblk, r, pair, &I, &J);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, li = lane & 15;
    const double *wsrc = Wm + (size_t)pair * B2 * B2;   // column-major B2 x B2
    for (int e = tid; e < B2 * B2; e += JR_NT) Ws[(e / B2) * LDW + e % B2] = wsrc[e];
    __syncthreads();
    double *M;
    int ld, chunk;
    if ((int)blockIdx.y < nchY) { M = Y; ld = ldy; chunk = blockIdx.y; }
    else { M = V; ld = ldv; chunk = blockIdx.y - nchY; }
    const int rbeg = chunk * RG, rend = min(N, rbeg + RG);
    // lane group g reads columns KS g .. KS g + KS - 1 of the pair, all in
    // one of the two blocks
    const int c0 = KS * g;
    const double *ag = M + (size_t)(c0 < b ? I * b + c0 : J * b + c0 - b) * ld;
    const double *wl = Ws + li * LDW + c0;
    for (int r0 = rbeg + 32 * w; r0 + 32 <= rend; r0 += 32 * (JR_NT / 64)) {
        dbl2 a[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) a[s] = *(const dbl2 *)(ag + (size_t)s * ld + r0 + 2 * li);
        // output column tiles in passes of TP (register pressure)
#pragma unroll
        for (int t0 = 0; t0 < NTI; t0 += TP) {
            dbl4 acc[2][TP];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int ti = 0; ti < TP; ++ti) acc[t][ti] = dbl4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int ti = 0; ti < TP; ++ti) {
                    const double wv = wl[16 * (t0 + ti) * LDW + s];
#pragma unroll
                    for (int t = 0; t < 2; ++t) acc[t][ti] = mfma16(wv, a[s][t], acc[t][ti]);
                }
#pragma unroll
            for (int ti = 0; ti < TP; ++ti)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = 16 * (t0 + ti) + g + 4 * e;
                    *(dbl2 *)(M + (size_t)blk_col(c, b, I, J) * ld + r0 + 2 * li) =
                        dbl2{acc[0][ti][e], acc[1][ti][e]};
                }
        }
    }
}

// Fused round of the FP32 stage: the Gram block, the inner solve and the
// update of every block pair in one launch.  The G workgroups of pair slot k
// (blockIdx.x = k G + part) share the slot's rows: workgroup `part` holds rows
// [part R, min(N, part R + R)) of the slot's 2b columns in registers from the
// load to the store, so Y is read once and written once per round (the
// separate kernels read it twice).  Each workgroup forms the partial Gram
// block of its rows, publishes it with device-coherent stores and a flag
// (raised to `tag`), waits (bounded) for the other workgroups of its slot,
// and adds the G partials in a fixed order in FP64, so every workgroup of the
// slot holds the same block and computes the same W.  Rows of a slot are
// never touched by another slot within a round, and rounds are separate
// launches, so nothing else is exchanged.
//
// Register layout of a 64-row stripe: lane (g, l) holds rows 4 l .. 4 l + 3
// (one 16-byte vector) of the columns c(g, s) = 16 (s / 4) + 4 g + s % 4,
// s = 0 .. B2/4 - 1, the layout in which the update's MFMA produces its
// result (the update sums over the pair's columns in any order, so its k
// index is mapped to these columns).  The Gram needs the rows on the k index
// instead: each wave writes its stripe to LDS column by column and reads it
// back in the layout of jac_gram_f32.
//
// A wait that runs out sets *err and the workgroup leaves without touching Y;
// the stage is then invalid and the caller starts it again with the separate
// kernels.
// Storage of Y in the fused round: FP32, or BF16 (the upper half of the
// FP32 bit pattern, rounded to nearest even) for the first sweeps of the
// three-precision variant.  Four consecutive rows of one column at a time.
typedef unsigned short bf16_t;
typedef short sh4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ flt4 ld4(const float *p) { return *(const flt4 *)p; }
__device__ __forceinline__ flt4 ld4(const bf16_t *p) {
    const uint2 u = *(const uint2 *)p;
    return flt4{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u)};
}
__device__ __forceinline__ unsigned bf16_rne(float x) {
    const unsigned r = __float_as_uint(x);
    return (r + 0x7fffu + ((r >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ void st4(float *p, flt4 v) { *(flt4 *)p = v; }
__device__ __forceinline__ void st4(bf16_t *p, flt4 v) {
    uint2 u;
    u.x = bf16_rne(v[0]) | (bf16_rne(v[1]) << 16);
    u.y = bf16_rne(v[2]) | (bf16_rne(v[3]) << 16);
    *(uint2 *)p = u;
}
// FP32 values as the operand of a BF16 MFMA, rounded to nearest even (exact
// when they are BF16 numbers already)
__device__ __forceinline__ sh4 as_bf16x4(flt4 v) {
    return sh4{(short)bf16_rne(v[0]), (short)bf16_rne(v[1]), (short)bf16_rne(v[2]),
               (short)bf16_rne(v[3])};
}

// BG: Gram products on the BF16 matrix cores (operands rounded to BF16, FP32
// sums), the three-precision variant's first sweeps; with ST = bf16_t, Y is
// stored in BF16 as well.
template <int B2, int NT, int SPW, typename ST, bool BG>
__global__ __launch_bounds__(NT) void jac_round_f32(int N, int nblk, int r, void *__restrict__ Yv,
                                                    int ldy, int G, int R, float *__restrict__ gpart,
                                                    int *__restrict__ gflag, int tag, int *flag,
                                                    float *offp, float *smxp, int *rot, double eps,
                                                    int max_inner, int cross, int spin,
                                                    int *__restrict__ err, const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr int b = B2 / 2, KS = B2 / 4, NTI = B2 / 16, NW = NT / 64;
    constexpr int NTT = B2 / 16, NUT = NTT * (NTT + 1) / 2;
    constexpr int LD = B2 + 1;
    constexpr int LDT = 64 + 4;            // a transposed stripe: column c at c LDT
    constexpr int H = b;
    static_assert(KS % 4 == 0 && NUT * 256 % 4 == 0, "layout");
    struct Tr { float t[NW][B2 * LDT]; };             // per-wave transposed stripe
    struct Red { float t[NW][NUT * 256]; };           // per-wave partial Gram tiles
    struct In { float G[2][B2 * LD]; float W[B2 * LD]; };
    __shared__ union { Tr tr; Red red; In in; } sm;
    __shared__ int ired[NW];
    __shared__ float wmx[NW], wsm[NW];
    __shared__ int bad;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g4 = lane >> 4, li = lane & 15;
    const int slot = blockIdx.x / G, part = blockIdx.x % G;
    int I, J;
    rr_slot(nblk, r, slot, &I, &J);
    const int r0 = part * R, r1 = min(N, r0 + R);
    const int nstripe = (r1 - r0) / 64;
    if (tid == 0) bad = 0;
    ST *Y = (ST *)Yv;
    // columns s < KS/2 lie in block I, the others in block J
    const ST *srcI = Y + (size_t)(I * b + 4 * g4) * ldy + r0 + 4 * li;
    const ST *srcJ = Y + (size_t)(J * b - b + 4 * g4) * ldy + r0 + 4 * li;

    // 1. load this wave's stripes
    flt4 a[SPW][KS];
#pragma unroll
    for (int i = 0; i < SPW; ++i) {
        const int st = w + i * NW;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int co = 16 * (s / 4) + (s % 4);
            const ST *src = (s < KS / 2 ? srcI : srcJ) + (size_t)co * ldy + 64 * st;
            a[i][s] = st < nstripe ? ld4(src) : flt4{0, 0, 0, 0};
        }
    }

    // 2. partial Gram block over this workgroup's rows (upper tiles)
    flt4 acc[NUT];
#pragma unroll
    for (int q = 0; q < NUT; ++q) acc[q] = flt4{0, 0, 0, 0};
    float *tr = sm.tr.t[w];
#pragma unroll
    for (int i = 0; i < SPW; ++i) {
        const bool live = w + i * NW < nstripe;
        if (live) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int c = 16 * (s / 4) + 4 * g4 + (s % 4);
                *(flt4 *)(tr + c * LDT + 4 * li) = a[i][s];
            }
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                flt4 v[NTT];
#pragma unroll
                for (int h = 0; h < NTT; ++h) v[h] = *(const flt4 *)(tr + (16 * h + li) * LDT + 16 * u + 4 * g4);
                if constexpr (BG) {
                    // one 16x16x16 BF16 product (FP32 sums) per tile and 16
                    // rows; lane (g, i) supplies k = 4 g .. 4 g + 3
                    sh4 vb[NTT];
#pragma unroll
                    for (int h = 0; h < NTT; ++h) vb[h] = as_bf16x4(v[h]);
                    int q = 0;
#pragma unroll
                    for (int ta = 0; ta < NTT; ++ta)
#pragma unroll
                        for (int tc = ta; tc < NTT; ++tc, ++q)
                            acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vb[ta], vb[tc], acc[q], 0, 0, 0);
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        int q = 0;
#pragma unroll
                        for (int ta = 0; ta < NTT; ++ta)
#pragma unroll
                            for (int tc = ta; tc < NTT; ++tc, ++q) acc[q] = mfma16(v[ta][t], v[tc][t], acc[q]);
                    }
                }
            }
        }
        __syncthreads();
    }
    // wave partials summed in wave order; the workgroup's partial published
    {
        float *red = sm.red.t[w];
#pragma unroll
        for (int q = 0; q < NUT; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[q * 256 + lane * 4 + e] = acc[q][e];
    }
    __syncthreads();
    float *gout = gpart + ((size_t)slot * G + part) * NUT * 256;
    for (int idx = tid; idx < NUT * 256; idx += NT) {
        float sacc = sm.red.t[0][idx];
#pragma unroll
        for (int q = 1; q < NW; ++q) sacc += sm.red.t[q][idx];
        coh_store(gout + idx, sacc);
    }
    publish_fence();
    __syncthreads();
    if (tid == 0) coh_store(gflag + (size_t)slot * G + part, tag);

    // 3. wait for the slot's other partials (bounded; spin < 0 gives up at once)
    if (tid < G && tid != part) {
        int it = 0;
        while (spin < 0 || coh_load(gflag + (size_t)slot * G + tid) < tag) {
            if (spin < 0 || ++it > spin) { bad = 1; break; }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) coh_store(err, 1);
        return;
    }

    // 4. G = sum of the partials (FP64, partial order) in LDS, symmetric; W = I.
    // Four entries per 16-byte coherent load, every partial's load in flight
    // together.
    const float *gin = gpart + (size_t)slot * G * NUT * 256;
    for (int v = tid; v < NUT * 64; v += NT) {
        flt4 x[JF_MAX_G];
#pragma unroll
        for (int q = 0; q < JF_MAX_G; ++q)
            if (q < G) x[q] = coh_load4(gin, (q * NUT * 256 + 4 * v) * (int)sizeof(float));
        double sacc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < JF_MAX_G; ++q)
            if (q < G)
#pragma unroll
                for (int e = 0; e < 4; ++e) sacc[e] += (double)x[q][e];
        // tile q, lane l, element e: entry (4 (l / 16) + e, l % 16) of tile (ta, tc)
        const int q = v >> 6, l = v & 63;
        int ta = 0, qq = q;
        while (qq >= NTT - ta) { qq -= NTT - ta; ++ta; }
        const int tc = ta + qq;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 16 * ta + 4 * (l >> 4) + e, j = 16 * tc + (l & 15);
            sm.in.G[0][i * LD + j] = (float)sacc[e];
            sm.in.G[0][j * LD + i] = (float)sacc[e];
        }
    }
    for (int e = tid; e < B2 * B2; e += NT) sm.in.W[(e / B2) * LD + e % B2] = (e / B2 == e % B2) ? 1.f : 0.f;
    __syncthreads();

    // 5. test the pairs (Algorithm 1's rule, FP64), the largest relative
    // off-diagonal; part 0 keeps the slot's bookkeeping
    // (thread t tests column q = t mod B2 against the rows p = t / B2 + k NT / B2:
    // g_qq is read once; the largest g_pq^2 / (g_pp g_qq) is kept and its root
    // taken once)
    const double eps2 = eps * eps;
    static_assert(NT % B2 == 0, "test layout");
    // (with cross set, `need` holds the cross rounds that have a pair to
    // rotate, as in jac_inner)
    int need = 0;
    double offsq = 0.0;
    {
        const int q = tid % B2;
        const double gqq = (double)sm.in.G[0][q * LD + q];
        for (int p = tid / B2; p < q; p += NT / B2) {
            const double g = (double)sm.in.G[0][p * LD + q];
            const double pq = (double)sm.in.G[0][p * LD + p] * gqq;
            if (g * g > eps2 * pq && pq > 0.0) {
                if (!cross) need = 1;
                else if (p < H && q >= H) need |= (int)(1u << ((q - H - p) & (H - 1)));
            }
            if (pq > 0.0) offsq = fmax(offsq, g * g * __builtin_amdgcn_rcp(pq));
        }
    }
    float offmax = (float)sqrt(offsq);
    offmax = wave_max(offmax);
    if (lane == 0) wmx[w] = offmax;
    need = block_or<NT>(need, ired);
    const unsigned rmask = cross ? (unsigned)need : ~0u;
    if (part == 0 && tid == 0) {
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < NW; ++q) m = fmaxf(m, wmx[q]);
        if (m > offp[slot]) offp[slot] = m;
        rot[slot] = need ? 1 : 0;
        if (need) *flag = 1;
    }
    if (!need) return;   // nothing rotates: Y keeps this slot's columns

    // 6. rotations
    float smax = inner_rounds<float, B2, NT>(sm.in.G, sm.in.W, ired, eps2, max_inner, cross, rmask);
    smax = wave_max(smax);
    if (lane == 0) wsm[w] = smax;
    __syncthreads();
    if (part == 0 && tid == 0) {
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < NW; ++q) m = fmaxf(m, wsm[q]);
        if (m > smxp[slot]) smxp[slot] = m;
    }

    // 7. update from registers: [Y_I Y_J]^T <- W^T [Y_I Y_J]^T per stripe; the
    // output tile ti holds columns 16 ti + 4 g + e, rows 4 l + t
    ST *dstI = Y + (size_t)(I * b + 4 * g4) * ldy + r0 + 4 * li;
    ST *dstJ = Y + (size_t)(J * b - b + 4 * g4) * ldy + r0 + 4 * li;
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti) {
        float wr[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) wr[s] = sm.in.W[(16 * (s / 4) + 4 * g4 + (s % 4)) * LD + 16 * ti + li];
#pragma unroll
        for (int i = 0; i < SPW; ++i) {
            const int st = w + i * NW;
            if (st >= nstripe) continue;
            flt4 o[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) o[t] = flt4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t) o[t] = mfma16(wr[s], a[i][s][t], o[t]);
            ST *dst = (ti < NTI / 2 ? dstI : dstJ) + (size_t)(16 * ti) * ldy + 64 * st;
#pragma unroll
            for (int e = 0; e < 4; ++e) st4(dst + (size_t)e * ldy, flt4{o[0][e], o[1][e], o[2][e], o[3][e]});
        }
    }
}

size_t jacobi_scratch_bytes(int N, int b, int elem) {
    const int B2 = 2 * b;
    const int npairs = N / B2;
    const int nch = gram_chunks(N);
    size_t bytes = (size_t)npairs * nch * B2 * B2 * elem;   // gram partials
    bytes += (size_t)npairs * B2 * B2 * elem;                // W blocks
    bytes += (size_t)npairs * sizeof(int) + 256;             // skip flags
    bytes += 256;                                             // flag
    bytes += 2 * ((size_t)npairs * sizeof(float) + 256);     // per-slot maxima
    bytes += (size_t)(N / b) * npairs * sizeof(int) + 256;   // rotated map per round
    if (elem == 4) {                                          // fused FP32 rounds
        bytes += 256;                                                            // alignment
        bytes += (size_t)JF_MAX_WG * JF_MAX_TILES * 256 * sizeof(float) + 256;   // partial Grams
        bytes += (size_t)JF_MAX_WG * sizeof(int) + 256;                          // their flags
    }
    return bytes + 1024;
}

void jacobi_carve(JacobiWork &jw, char *base, int N, int b, int elem) {
    const int B2 = 2 * b;
    const int npairs = N / B2;
    const int nch = gram_chunks(N);
    char *p = base;
    jw.gram = p; p += (size_t)npairs * nch * B2 * B2 * elem;
    jw.wmat = p; p += (size_t)npairs * B2 * B2 * elem;
    jw.skip = (int *)p; p += (size_t)npairs * sizeof(int) + 256;
    jw.flag = (int *)p; p += 256;
    jw.offp = (float *)p; p += (size_t)npairs * sizeof(float) + 256;
    jw.smxp = (float *)p; p += (size_t)npairs * sizeof(float) + 256;
    jw.rotmap = (int *)p; p += (size_t)(N / b) * npairs * sizeof(int) + 256;
    if (elem == 4) {
        p = base + ((p - base + 255) & ~(size_t)255);   // 16-byte loads of the partials
        jw.gpart = (float *)p; p += (size_t)JF_MAX_WG * JF_MAX_TILES * 256 * sizeof(float) + 256;
        jw.gflag = (int *)p;
    } else {
        jw.gpart = nullptr;
        jw.gflag = nullptr;
    }
}

// ---------------------------------------------------------------- sweep control
// Start of a sweep: the any-rotation and time-out flags and the per-slot
// maxima cleared (a kernel, not a memset, so the call can be captured in a
// graph).  With ctl: nothing once the stage has stopped.
__global__ __launch_bounds__(256) void jac_sweep_begin(const SweepCtl *ctl, int *flag, float *offp,
                                                       float *smxp, int npairs) {
    if (ctl && ctl->stop) return;
    for (int i = threadIdx.x; i < npairs; i += 256) {
        offp[i] = 0.f;
        smxp[i] = 0.f;
    }
    if (threadIdx.x < 3) flag[threadIdx.x] = 0;
}

// End of a sweep in the stream-ordered mode: the stopping rules that the
// host applies otherwise (a sweep without rotations, Algorithm 1; the
// remaining off-diagonal and rotation sizes, as xGESVJ; the FP32 stage's
// off-diagonal target), evaluated on the device.  The sweeps still enqueued
// after `stop` is set exit at their first instruction.
__global__ __launch_bounds__(256) void jac_sweep_end(SweepCtl *ctl, const int *flag, const float *offp,
                                                     const float *smxp, int npairs, double n_real,
                                                     double eps, double stop_off) {
    __shared__ float ro[4], rs[4];
    if (ctl->stop) return;
    float o = 0.f, m = 0.f;
    for (int i = threadIdx.x; i < npairs; i += 256) {
        o = fmaxf(o, offp[i]);
        m = fmaxf(m, smxp[i]);
    }
    o = wave_max(o);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) { ro[threadIdx.x >> 6] = o; rs[threadIdx.x >> 6] = m; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const float off = fmaxf(fmaxf(ro[0], ro[1]), fmaxf(ro[2], ro[3]));
    const float smx = fmaxf(fmaxf(rs[0], rs[1]), fmaxf(rs[2], rs[3]));
    const int k = ctl->sweeps;
    if (k < 32) ctl->off[k] = off;
    ctl->sweeps = k + 1;
    if (flag[1]) { ctl->timeout = 1; ctl->stop = 1; return; }
    bool done = flag[0] == 0;
    if (!done && (double)off < sqrt(n_real) * eps && n_real * (double)off * (double)smx < eps)
        done = true;
    if (!done && stop_off > 0.0 && off <= stop_off) done = true;
    if (done) { ctl->conv = 1; ctl->stop = 1; }
}

__global__ void jac_fill_zero(int *p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- fused FP32 rounds
typedef void (*RoundFn)(int, int, int, void *, int, int, int, float *, int *, int, int *, float *,
                        float *, int *, double, int, int, int, int *, const int *);

struct FusedCfg {
    int G = 0, R = 0, nt = 0;   // workgroups per pair slot, rows per workgroup, threads
    RoundFn fn = nullptr;
};

// Workgroups of `fn` the current device holds at once (compute units times
// the kernel's occupancy per unit), cached per device and variant.
static int round_capacity(int variant, RoundFn fn, int nt) {
    static std::atomic<int> cap[64][9];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 0;
    }
    int c = cap[dev][variant].load(std::memory_order_relaxed);
    if (c > 0) return c;
    int ncu = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, nt, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    c = ncu * per_cu;
    cap[dev][variant].store(c, std::memory_order_relaxed);
    return c;
}

// The fused round needs every workgroup of a pair slot resident at once (they
// wait for each other's partial Gram blocks): the whole grid must fit on the
// device, one pair slot's rows split over G workgroups of at most 16 stripes.
// half: 0 FP32, 1 BF16 Gram products, 2 BF16 Gram products and BF16 storage
static bool fused_config(int N, int B2, FusedCfg *fc, int half = 0) {
    if (B2 != 64 || N % 64 != 0) return false;
    const int npairs = N / B2;
    int ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    int G = ncu / npairs;
    G = G < 1 ? 1 : (G > JF_MAX_G ? JF_MAX_G : G);
    const int R = cdiv(cdiv(N, G), 64) * 64;
    G = cdiv(N, R);
    const int stripes = R / 64;
    int variant, nt;
    RoundFn fn;
    if (stripes <= 4) { variant = 0; nt = 256; fn = jac_round_f32<64, 256, 1, float, false>; }
    else if (stripes <= 8) { variant = 1; nt = 256; fn = jac_round_f32<64, 256, 2, float, false>; }
    else if (stripes <= 16) { variant = 2; nt = 512; fn = jac_round_f32<64, 512, 2, float, false>; }
    else return false;
    if (half == 1) {
        const RoundFn hf[3] = {jac_round_f32<64, 256, 1, float, true>,
                               jac_round_f32<64, 256, 2, float, true>,
                               jac_round_f32<64, 512, 2, float, true>};
        fn = hf[variant];
        variant += 3;
    } else if (half == 2) {
        const RoundFn hf[3] = {jac_round_f32<64, 256, 1, bf16_t, true>,
                               jac_round_f32<64, 256, 2, bf16_t, true>,
                               jac_round_f32<64, 512, 2, bf16_t, true>};
        fn = hf[variant];
        variant += 6;
    }
    if (npairs * G > JF_MAX_WG || npairs * G > round_capacity(variant, fn, nt)) return false;
    fc->G = G; fc->R = R; fc->nt = nt; fc->fn = fn;
    return true;
}

// Sweeps over the ncols columns of Y (N rows, ld N; ncols a multiple of 2b,
// at most N) and of V (N rows).
//
// fc (FP32 stage, 64-wide blocks, no V): each round is one launch of the
// fused kernel instead of the Gram, inner and update launches.  Returns -2 if
// a wait of the fused kernel ran out (Y is then invalid).
//
// jw.ctl set (stream-ordered mode): all maxsweep sweeps are enqueued with no
// host synchronisation, each ended by jac_sweep_end, which applies the
// stopping rules on the device; the kernels of a sweep after the stop exit at
// once.  Returns maxsweep; the sweeps run, convergence and a fused round's
// time-out are in *jw.ctl.
template <typename T, int B2, int INNER_NT>
static int sweeps_impl(hipStream_t s, int N, int ncols, T *Y, T *V, double eps, int maxsweep,
                       int max_inner, JacobiWork &jw, int *conv, const FusedCfg *fc = nullptr) {
    constexpr int b = B2 / 2;
    const int nblk = ncols / b;
    const int npairs = nblk / 2;
    const int nch = cdiv(N, JU_RG);
    const int rgG = gram_rows(N), nchG = gram_chunks(N);
    const int nchV = V ? nch : 0;
    *conv = 0;
    int sw = 0;
    std::vector<std::pair<size_t, int>> upd_slots;   // clocked update launches (slot, round)
    std::vector<int> hrot((size_t)nblk * npairs);
    std::vector<float> hoff(npairs), hsmx(npairs);
    // one rotated pair in the update: its 2b columns of Y (and V) read and
    // written once, 2 N (2b)^2 flops per matrix
    // (element size: FP32, FP64, or BF16 for the fused round's BF16 sweeps)
    const bool half = fc && jw.half;
    const double Es = (fc && jw.half == 2) ? 2.0 : (double)sizeof(T);
    const double pair_upd_bytes = 2.0 * N * B2 * Es * (V ? 2 : 1);
    const double pair_upd_flops = 2.0 * N * B2 * B2 * (V ? 2 : 1);
    std::vector<std::pair<size_t, int>> round_slots;   // clocked fused launches (slot, round)
    // stream-ordered mode: every sweep is enqueued and stops on the device
    SweepCtl *ctl = jw.ctl;
    const int *stop = ctl ? &ctl->stop : nullptr;
    if (fc) {
        const int nf = npairs * fc->G;
        hipLaunchKernelGGL(jac_fill_zero, dim3(cdiv(nf, 256)), dim3(256), 0, s, jw.gflag, nf);
    }
    for (; sw < maxsweep; ++sw) {
        round_slots.clear();
        upd_slots.clear();
        hipLaunchKernelGGL(jac_sweep_begin, dim3(1), dim3(256), 0, s, (const SweepCtl *)ctl, jw.flag,
                           jw.offp, jw.smxp, npairs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { note_hip_error(e, "jacobi flag reset"); return -1; }
        // kernel-class ids for the optional per-launch clock
        const int kbase = sizeof(T) == 4 ? 0 : 3;
        const double E = Es;
        // algorithmic work per round: the Gram blocks read Y once and cost
        // N (2b)^2 flops per pair for the symmetric product; the update reads
        // and writes Y (and V) once and costs 2 N (2b)^2 flops per pair and
        // matrix; the inner solve is (2b - 1) rounds of b rotations applied
        // two-sided to the 2b x 2b block and one-sided to W (12 (2b)^2 b flops)
        const double gram_bytes = (double)N * ncols * E;
        const double gram_flops = (double)npairs * N * B2 * B2;
        const double upd_bytes = 2.0 * (double)N * ncols * E * (V ? 2 : 1);
        const double upd_flops = 2.0 * (double)npairs * N * B2 * B2 * (V ? 2 : 1);
        const double inner_flops = 12.0 * (double)npairs * B2 * B2 * b;
        for (int r = 0; r < nblk - 1; ++r) {
            // optional per-launch clock: events recorded by the dispatch itself
            hipEvent_t e0, e1;
            const int cross = (jw.cross_pairs && r > 0) ? 1 : 0;
            if constexpr (sizeof(T) == 4 && B2 == 64) {
                if (fc) {
                    // algorithmic work: Y read once, the Gram blocks, the inner
                    // solves; the rotated pairs' writes and updates are added
                    // after the sweep
                    const int tag = 1 + sw * (nblk - 1) + r;
                    const int spin = jw.spin == 0 ? JF_SPIN : jw.spin;
                    const dim3 grid(npairs * fc->G), blk(fc->nt);
                    const bool clk = jw.kc && jw.kc->slot(half ? SVD_K_ROUND16 : SVD_K_ROUND32, gram_bytes,
                                                          gram_flops + inner_flops, &e0, &e1);
                    if (clk) {
                        round_slots.push_back({jw.kc->used / 2 - 1, r});
                        hipExtLaunchKernelGGL(fc->fn, grid, blk, 0, s, e0, e1, 0, N, nblk, r, (void *)Y,
                                              N, fc->G, fc->R, jw.gpart, jw.gflag, tag, jw.flag, jw.offp,
                                              jw.smxp, jw.rotmap + (size_t)r * npairs, eps, max_inner,
                                              cross, spin, jw.flag + 1, stop);
                    } else {
                        hipLaunchKernelGGL(fc->fn, grid, blk, 0, s, N, nblk, r, (void *)Y, N, fc->G,
                                           fc->R, jw.gpart, jw.gflag, tag, jw.flag, jw.offp, jw.smxp,
                                           jw.rotmap + (size_t)r * npairs, eps, max_inner, cross, spin,
                                           jw.flag + 1, stop);
                    }
                    continue;
                }
            }
            const bool gclk = jw.kc && jw.kc->slot(kbase + 0, gram_bytes, gram_flops, &e0, &e1);
            if constexpr (sizeof(T) == 4) {
                if (gclk)
                    hipExtLaunchKernelGGL((jac_gram_f32<B2>), dim3(npairs, nchG), dim3(JR_NT), 0, s, e0,
                                          e1, 0, N, nblk, r, (const T *)Y, N, (T *)jw.gram, nchG, rgG, stop);
                else
                    hipLaunchKernelGGL((jac_gram_f32<B2>), dim3(npairs, nchG), dim3(JR_NT), 0, s, N, nblk,
                                       r, (const T *)Y, N, (T *)jw.gram, nchG, rgG, stop);
            } else {
                if (gclk)
                    hipExtLaunchKernelGGL((jac_gram_f64<B2>), dim3(npairs, nchG), dim3(JR_NT), 0, s, e0,
                                          e1, 0, N, nblk, r, (const T *)Y, N, (T *)jw.gram, nchG, rgG, stop);
                else
                    hipLaunchKernelGGL((jac_gram_f64<B2>), dim3(npairs, nchG), dim3(JR_NT), 0, s, N, nblk,
                                       r, (const T *)Y, N, (T *)jw.gram, nchG, rgG, stop);
            }
            if (jw.kc && jw.kc->slot(kbase + 1, 0.0, inner_flops, &e0, &e1))
                hipExtLaunchKernelGGL((jac_inner<T, B2, INNER_NT>), dim3(npairs), dim3(INNER_NT), 0, s,
                                      e0, e1, 0, nchG, (const T *)jw.gram, (T *)jw.wmat, jw.skip,
                                      jw.flag, jw.offp, jw.smxp, jw.rotmap + (size_t)r * npairs, eps,
                                      max_inner, cross, stop);
            else
                hipLaunchKernelGGL((jac_inner<T, B2, INNER_NT>), dim3(npairs), dim3(INNER_NT), 0, s,
                                   nchG, (const T *)jw.gram, (T *)jw.wmat, jw.skip, jw.flag, jw.offp,
                                   jw.smxp, jw.rotmap + (size_t)r * npairs, eps, max_inner, cross,
                                   stop);
            const bool clk = jw.kc && jw.kc->slot(kbase + 2, upd_bytes, upd_flops, &e0, &e1);
            if (clk) upd_slots.push_back({jw.kc->used / 2 - 1, r});
            if constexpr (sizeof(T) == 4) {
                const dim3 ugrid(npairs, nch + nchV);
                if (clk)
                    hipExtLaunchKernelGGL((jac_update_f32<B2>), ugrid, dim3(JR_NT), 0, s, e0, e1, 0, N,
                                          nblk, r, Y, N, V, N, nch, (const T *)jw.wmat,
                                          (const int *)jw.skip, stop);
                else
                    hipLaunchKernelGGL((jac_update_f32<B2>), ugrid, dim3(JR_NT), 0, s, N, nblk, r, Y, N,
                                       V, N, nch, (const T *)jw.wmat, (const int *)jw.skip, stop);
            } else {
                const dim3 ugrid(npairs, nch + nchV);
                if (clk)
                    hipExtLaunchKernelGGL((jac_update_f64<B2>), ugrid, dim3(JR_NT), 0, s, e0, e1, 0, N,
                                          nblk, r, Y, N, V, N, nch, (const T *)jw.wmat,
                                          (const int *)jw.skip, stop);
                else
                    hipLaunchKernelGGL((jac_update_f64<B2>), ugrid, dim3(JR_NT), 0, s, N, nblk, r, Y, N,
                                       V, N, nch, (const T *)jw.wmat, (const int *)jw.skip, stop);
            }
        }
        if (ctl) {
            hipLaunchKernelGGL(jac_sweep_end, dim3(1), dim3(256), 0, s, ctl, (const int *)jw.flag,
                               (const float *)jw.offp, (const float *)jw.smxp, npairs,
                               (double)jw.n_real, eps, jw.stop_off);
            e = hipGetLastError();
            if (e != hipSuccess) { note_hip_error(e, "jacobi sweep"); return -1; }
            continue;
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(jw.hflag, jw.flag, 3 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hoff.data(), jw.offp, (size_t)npairs * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hsmx.data(), jw.smxp, (size_t)npairs * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && (!upd_slots.empty() || !round_slots.empty()))
            e = hipMemcpyAsync(hrot.data(), jw.rotmap, (size_t)(nblk - 1) * npairs * sizeof(int),
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { note_hip_error(e, "jacobi sweep"); return -1; }
        // a clocked update launch moves the columns of the pairs its round
        // rotated (the others are skipped): its algorithmic bytes and flops
        for (auto &us : upd_slots) {
            double k = 0.0;
            for (int q = 0; q < npairs; ++q) k += hrot[(size_t)us.second * npairs + q];
            jw.kc->bytes[us.first] = k * pair_upd_bytes;
            jw.kc->flops[us.first] = k * pair_upd_flops;
        }
        // a fused round writes the columns of the pairs it rotated, once
        for (auto &us : round_slots) {
            double k = 0.0;
            for (int q = 0; q < npairs; ++q) k += hrot[(size_t)us.second * npairs + q];
            jw.kc->bytes[us.first] += k * 0.5 * pair_upd_bytes;
            jw.kc->flops[us.first] += k * pair_upd_flops;
        }
        if (jw.hflag[1]) {
            note_error_text("fused Jacobi round: a bounded wait ran out");
            return -2;
        }
        if (jw.kc) jw.kc->collect();
        float off = 0.f, smx = 0.f;
        for (int q = 0; q < npairs; ++q) {
            off = fmaxf(off, hoff[q]);
            smx = fmaxf(smx, hsmx[q]);
        }
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
int jacobi_sweeps_cols(hipStream_t s, int N, int ncols, int b, T *Y, T *V, double eps, int maxsweep,
                       int max_inner, JacobiWork &jw, int *conv) {
    if (ncols <= 0 || ncols > N || ncols % (2 * b) != 0) {
        note_hip_error(hipErrorInvalidValue, "jacobi_sweeps_cols: column count");
        return -1;
    }
    // the update works on whole 64-row stripes with 16-byte column accesses
    if (N % 64 != 0) {
        note_hip_error(hipErrorInvalidValue, "jacobi_sweeps_cols: row count not a multiple of 64");
        return -1;
    }
    if constexpr (sizeof(T) == 4) {
        FusedCfg fc;
        if (jw.fused && !V && b == 32 && ncols == N && fused_config(N, 64, &fc, jw.half))
            return sweeps_impl<T, 64, 256>(s, N, ncols, Y, V, eps, maxsweep, max_inner, jw, conv, &fc);
    }
    if (jw.half) {
        note_hip_error(hipErrorInvalidValue, "jacobi_sweeps_cols: BF16 sweeps need the fused round");
        return -1;
    }
    if (b == 16) return sweeps_impl<T, 32, 256>(s, N, ncols, Y, V, eps, maxsweep, max_inner, jw, conv);
    // 64-wide FP64 blocks: 512 threads shorten each round's per-thread work
    // (2 groups of G and 4 rows of W per thread instead of 4 and 8)
    if (sizeof(T) == 8)
        return sweeps_impl<T, 64, 512>(s, N, ncols, Y, V, eps, maxsweep, max_inner, jw, conv);
    return sweeps_impl<T, 64, 256>(s, N, ncols, Y, V, eps, maxsweep, max_inner, jw, conv);
}

bool jacobi_fused_ok(int N, int half) {
    FusedCfg fc;
    return fused_config(N, 64, &fc, half);
}

template <typename T>
int jacobi_sweeps(hipStream_t s, int N, int b, T *Y, T *V, double eps, int maxsweep, int max_inner,
                  JacobiWork &jw, int *conv) {
    return jacobi_sweeps_cols<T>(s, N, N, b, Y, V, eps, maxsweep, max_inner, jw, conv);
}

template int jacobi_sweeps<float>(hipStream_t, int, int, float *, float *, double, int, int,
                                  JacobiWork &, int *);
template int jacobi_sweeps<double>(hipStream_t, int, int, double *, double *, double, int, int,
                                   JacobiWork &, int *);
template int jacobi_sweeps_cols<double>(hipStream_t, int, int, int, double *, double *, double, int,
                                        int, JacobiWork &, int *);

} // namespace mpj
