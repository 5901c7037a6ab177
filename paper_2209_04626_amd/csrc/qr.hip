// Blocked Householder QR in FP64 (the QR factorizations of Sections 2.2 and
// 3.1: the tall reduction A = Q0 R1, the QR of A1 P after the pivots of
// Algorithm 5, the LQ step through the QR of R^T, and the QR of X^T U_low in
// the switch of Section 3.3).
//
// Panel (QR_NB columns): one launch per column.  Each workgroup owns QR_RC
// consecutive rows of the panel, stages them in LDS, applies the reflector
// of the current column and emits partial dot products for the next one
// (rows below the next diagonal), so the norm and the projections of a
// column are a single cross-workgroup reduction, read by every workgroup at
// the start of the next launch.  The row of the next diagonal element (the
// reflector's head) is passed through a separate buffer so no workgroup reads
// a value another one is writing.
// Trailing matrix: compact WY form H_0..H_{nb-1} = I - V T V^T with the LAPACK
// xLARFT recurrence for T, applied with MFMA GEMMs.
#include <atomic>
#include <utility>

#include "common.hpp"
#include "internal.hpp"

namespace mpj {

static_assert(QR_RC == 256, "panel kernels use one thread per row");
constexpr int LROW = QR_RC;  // LDS column stride (all accesses are row-contiguous)

// Load rows [g*RC, g*RC+RC) x columns [c0, nb) of the panel into L[k][r].
// (unrolled over the panel width so that all loads of a thread are in flight)
__device__ __forceinline__ void panel_load(double *L, const double *P, int ld, int mp, int g,
                                           int c0, int nb) {
    const int r = threadIdx.x;
    const int i = g * QR_RC + r;
    double v[QR_NB];
#pragma unroll
    for (int k = 0; k < QR_NB; ++k)
        v[k] = (k >= c0 && k < nb && i < mp) ? P[(size_t)k * ld + i] : 0.0;
#pragma unroll
    for (int k = 0; k < QR_NB; ++k)
        if (k >= c0 && k < nb) L[k * LROW + r] = v[k];
}

__device__ __forceinline__ void panel_store(const double *L, double *P, int ld, int mp, int g,
                                            int c0, int nb) {
    const int r = threadIdx.x;
    const int i = g * QR_RC + r;
    if (i < mp) {
#pragma unroll
        for (int k = 0; k < QR_NB; ++k)
            if (k >= c0 && k < nb) P[(size_t)k * ld + i] = L[k * LROW + r];
    }
}

// Partial dots for the reflector of column jn: over local rows i > jn,
// part[k] = sum x_i P(i, k) for k = jn..nb-1 (k = jn gives the squared norm of
// the part below the diagonal).  Wavefront w takes columns jn + w + 4c; its
// lanes stride the rows.  Head row jn goes to head[k].
__device__ void panel_partials(const double *L, int mp, int g, int jn, int nb,
                               double *part, double *head) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int k = jn + w; k < nb; k += 4) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < QR_RC / 64; ++q) {
            const int r = lane + 64 * q;
            const int i = g * QR_RC + r;
            if (i > jn && i < mp) s += L[jn * LROW + r] * L[k * LROW + r];
        }
        s = wave_sum(s);
        if (lane == 0) part[(size_t)g * QR_NB + k] = s;
    }
    const int rj = jn - g * QR_RC;
    if (rj >= 0 && rj < QR_RC && t >= jn && t < nb) head[t] = L[t * LROW + rj];
}

__global__ __launch_bounds__(QR_RC) void qr_panel_init(int mp, int nb, const double *P, int ld,
                                                      double *part, double *head) {
    __shared__ double L[QR_NB * LROW];
    const int g = blockIdx.x;
    panel_load(L, P, ld, mp, g, 0, nb);
    __syncthreads();
    panel_partials(L, mp, g, 0, nb, part, head);
}

// Cross-workgroup sums of the partial dots for columns j..nb-1, read with all
// threads in parallel (QR_RC / QR_NB workgroup rows at a time) and reduced
// in a fixed order.
__device__ __forceinline__ void reduce_partials(const double *pin, int ngroups, int j, int nb,
                                                double *dsum, double *red) {
    const int t = threadIdx.x;
    constexpr int GR = QR_RC / QR_NB;        // workgroup rows per pass
    const int k = t % QR_NB, q0 = t / QR_NB;
    double a = 0.0;
    for (int q = q0; q < ngroups; q += GR) a += pin[(size_t)q * QR_NB + k];
    red[q0 * QR_NB + k] = a;
    __syncthreads();
    if (t < QR_NB && t >= j && t < nb) {
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q < GR; ++q) sacc += red[q * QR_NB + t];
        dsum[t] = sacc;
    }
}

__global__ __launch_bounds__(QR_RC) void qr_panel_step(int j, int mp, int nb, int ngroups,
                                                      double *P, int ld, double *part,
                                                      double *head, double *tau) {
    __shared__ double L[QR_NB * LROW];
    __shared__ double red[QR_RC];
    __shared__ double wsh[QR_NB];
    __shared__ double dsum[QR_NB];
    __shared__ double hsh[QR_NB];
    __shared__ double prm[3];  // beta, tau, scale
    const int g = blockIdx.x, t = threadIdx.x;
    const double *pin = part + (size_t)(j & 1) * ngroups * QR_NB;
    const double *hin = head + (j & 1) * QR_NB;
    double *pout = part + (size_t)((j + 1) & 1) * ngroups * QR_NB;
    double *hout = head + ((j + 1) & 1) * QR_NB;

    // 1. all global loads first: head row, this chunk, the partial dots
    if (t >= j && t < nb) hsh[t] = hin[t];
    panel_load(L, P, ld, mp, g, j, nb);
    reduce_partials(pin, ngroups, j, nb, dsum, red);
    __syncthreads();
    if (t == 0) {
        const double x0 = hsh[j];
        const double s2 = dsum[j];
        double beta = x0, tv = 0.0, scale = 0.0;
        if (s2 != 0.0) {
            beta = -copysign(sqrt(x0 * x0 + s2), x0);
            tv = (beta - x0) / beta;
            scale = 1.0 / (x0 - beta);
        }
        prm[0] = beta; prm[1] = tv; prm[2] = scale;
        if (g == 0) tau[j] = tv;
    }
    __syncthreads();
    if (t > j && t < nb) wsh[t] = prm[1] * (hsh[t] + prm[2] * dsum[t]);
    __syncthreads();

    // 2. apply H_j to this workgroup's rows
    {
        const int i = g * QR_RC + t;
        if (i == j) {
            L[j * LROW + t] = prm[0];
            for (int k = j + 1; k < nb; ++k) L[k * LROW + t] -= wsh[k];
        } else if (i > j && i < mp) {
            const double v = L[j * LROW + t] * prm[2];
            L[j * LROW + t] = v;
            for (int k = j + 1; k < nb; ++k) L[k * LROW + t] -= wsh[k] * v;
        }
    }
    __syncthreads();

    // 3. partials for column j + 1
    if (j + 1 < nb) panel_partials(L, mp, g, j + 1, nb, pout, hout);
    __syncthreads();
    panel_store(L, P, ld, mp, g, j, nb);
}

// The whole panel in one launch (at most QR_COOP_MAXG workgroups, all
// resident at once): thread t of workgroup g keeps row g*QR_RC + t of the
// panel in registers for all nb columns.  For column j every workgroup
// reduces its rows' products a_ij a_ik (i > j) in LDS and publishes the sums
// (and workgroup 0 the head row j); every workgroup then reads all of them,
// adds them in the same order, so that all build the same reflector, and
// applies it to its rows.
//
// Each published FP64 value travels as two 64-bit words, (tag << 32) | half,
// written and read with device-coherent (relaxed, agent-scope) atomics.  A
// 64-bit atomic is seen whole or not at all, so a reader that finds the
// column's tag (base + j + 1) in both words has the value: no flag, no
// store-completion wait, one memory round trip per column.  Reading is a
// bounded poll; a wait that runs out poisons tau[j] with NaN instead of
// hanging.  Tags are unique within one factorisation (the words are cleared
// before each one), and a workgroup cannot overwrite a buffer of column j + 2
// before every workgroup has read column j (it first needs their column
// j + 1 values).
constexpr int QR_COOP_MAXG = 256;
constexpr int QR_COOP_SPIN = 1 << 22;

__device__ __forceinline__ void tag_store(unsigned long long *p, double v, unsigned tag) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned long long t = (unsigned long long)tag << 32;
    coh_store(p, t | (b & 0xffffffffull));
    coh_store(p + 1, t | (b >> 32));
}

// Up to K tagged values at once, those whose bit is set in `mask` (all
// loads of a pass in flight together); false if the bounded poll ran out
// (spin < 0: give up at once when there is anything to wait for).
template <int K>
__device__ __forceinline__ bool tag_load(const unsigned long long *const (&p)[K], unsigned mask,
                                         unsigned tag, int spin, double (&v)[K]) {
    if (mask == 0) return true;
    if (spin < 0) return false;
    int it = 0;
    for (;;) {
        unsigned long long w0[K], w1[K];
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (mask & (1u << i)) { w0[i] = coh_load(p[i]); w1[i] = coh_load(p[i] + 1); }
        bool ok = true;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (mask & (1u << i)) {
                ok = ok && (unsigned)(w0[i] >> 32) == tag && (unsigned)(w1[i] >> 32) == tag;
                v[i] = __longlong_as_double((long long)((w1[i] << 32) | (w0[i] & 0xffffffffull)));
            }
        if (ok) return true;
        if (++it > spin) return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

struct CoopShared {
    double red[QR_RC * (QR_NB + 1)];
    double s8[(QR_RC / QR_NB) * QR_NB];
    double S[QR_NB], H[QR_NB], tv[QR_NB];
    int bad;
};

// Column J of the one-launch panel (J is a compile-time constant so that the
// row stays in registers).
template <int J>
__device__ __forceinline__ void coop_column(double (&a)[QR_NB], CoopShared &sh, int mp, int nb,
                                            unsigned long long *tpart, unsigned long long *thead,
                                            double *tau, int base, int spin) {
    if (J >= nb) return;
    constexpr int GR = QR_RC / QR_NB;
    const int G = gridDim.x;
    const int g = blockIdx.x, t = threadIdx.x, i = g * QR_RC + t;
    const bool live = i < mp;
    // 1. this workgroup's sums of a_iJ a_ik over its rows i > J
    {
        const double xj = (live && i > J) ? a[J] : 0.0;
#pragma unroll
        for (int k = J; k < QR_NB; ++k) sh.red[t * (QR_NB + 1) + k] = xj * a[k];
    }
    __syncthreads();
    {
        const int k = t % QR_NB, q = t / QR_NB;
        double sacc = 0.0;
#pragma unroll
        for (int r = 0; r < QR_RC / GR; ++r) sacc += sh.red[(q * (QR_RC / GR) + r) * (QR_NB + 1) + k];
        sh.s8[q * QR_NB + k] = sacc;
    }
    __syncthreads();
    // 2. publish this workgroup's sums and (workgroup 0) the head row, tagged;
    // every thread of column k keeps this workgroup's own sum for step 3
    const unsigned tag = (unsigned)(base + J + 1);
    unsigned long long *po = tpart + (size_t)(J & 1) * G * QR_NB * 2;
    unsigned long long *ho = thead + (size_t)(J & 1) * QR_NB * 2;
    double own = 0.0;
    {
        const int k = t % QR_NB;
#pragma unroll
        for (int q = 0; q < GR; ++q) own += sh.s8[q * QR_NB + k];
    }
    if (t < QR_NB) tag_store(po + ((size_t)g * QR_NB + t) * 2, own, tag);
    // (the head row goes out from 32 threads after the barrier: one thread
    // issuing its 64 stores held every other workgroup back)
    if (g == 0 && t == J) {
#pragma unroll
        for (int k = 0; k < QR_NB; ++k) sh.H[k] = a[k];
    }
    __syncthreads();
    if (g == 0 && t < QR_NB) tag_store(ho + 2 * t, sh.H[t], tag);
    // 3. every workgroup's sums of column J, added in workgroup order (the
    // own one from registers), and the head row; up to four values per pass
    // with their loads in flight together
    {
        const int k = t % QR_NB, q0 = t / QR_NB;
        double sacc = 0.0;
        bool ok = true;
        for (int qb = q0; qb < G; qb += 4 * GR) {
            const unsigned long long *pp[4];
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            unsigned mask = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = qb + i * GR;
                pp[i] = po + ((size_t)(q < G ? q : 0) * QR_NB + k) * 2;
                if (q < G && q != g) mask |= 1u << i;
            }
            ok = ok && tag_load<4>(pp, mask, tag, spin, v);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = qb + i * GR;
                if (q < G) sacc += q == g ? own : v[i];
            }
        }
        sh.s8[q0 * QR_NB + k] = sacc;
        if (g != 0 && t < QR_NB) {
            const unsigned long long *hp[1] = {ho + 2 * t};
            double hv[1] = {0.0};
            ok = ok && tag_load<1>(hp, 1u, tag, spin, hv);
            sh.H[t] = hv[0];
        }
        if (!ok) sh.bad = 1;
    }
    __syncthreads();
    if (t < QR_NB) {
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q < GR; ++q) sacc += sh.s8[q * QR_NB + t];
        sh.S[t] = sacc;
    }
    __syncthreads();
    // 4. the reflector of column J (every thread computes the same one)
    const double x0 = sh.H[J], s2 = sh.S[J];
    double beta = x0, tv = 0.0, scale = 0.0;
    if (s2 != 0.0) {
        beta = -copysign(sqrt(x0 * x0 + s2), x0);
        tv = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
    }
    if (g == 0 && t == 0) tau[J] = sh.bad ? __builtin_nan("") : tv;
    if (t == 0) sh.tv[J] = tv;
    // 5. apply it to this thread's row
    if (live && i >= J) {
        const double v = i == J ? 1.0 : a[J] * scale;
#pragma unroll
        for (int k = J + 1; k < QR_NB; ++k) a[k] -= tv * (sh.H[k] + scale * sh.S[k]) * v;
        a[J] = i == J ? beta : v;
    }
}

template <int... J>
__device__ __forceinline__ void coop_columns(std::integer_sequence<int, J...>, double (&a)[QR_NB],
                                             CoopShared &sh, int mp, int nb,
                                             unsigned long long *tpart, unsigned long long *thead,
                                             double *tau, int base, int spin) {
    (coop_column<J>(a, sh, mp, nb, tpart, thead, tau, base, spin), ...);
}

// After the last column: G = V^T V of the panel, each workgroup's rows on
// the matrix cores (wavefront w forms 16 x 16 tile (w % 2, w / 2) over the
// 256 rows held in LDS), published through the same coherent stores and a
// flag raised to base + QR_NB + 1; workgroup 0 alone waits, adds the partial
// tiles in workgroup order and forms T from G as qr_build_t does (lane j
// solves column j of the inverse of diag(1/tau) + striu(G)).  No workgroup
// waits for workgroup 0, so this adds one wait, not a round trip.
__global__ __launch_bounds__(QR_RC) void qr_panel_coop(int mp, int nb, double *P, int ld,
                                                      unsigned long long *tpart,
                                                      unsigned long long *thead, double *tau,
                                                      int *flags, int base, double *Vb,
                                                      double *Gpart, double *T, int ldt, int *err,
                                                      int spin) {
    __shared__ CoopShared sh;
    const int i = blockIdx.x * QR_RC + threadIdx.x;
    const bool live = i < mp;
    double a[QR_NB];
#pragma unroll
    for (int k = 0; k < QR_NB; ++k) a[k] = (live && k < nb) ? P[(size_t)k * ld + i] : 0.0;
    if (threadIdx.x == 0) sh.bad = 0;
    coop_columns(std::make_integer_sequence<int, QR_NB>{}, a, sh, mp, nb, tpart, thead, tau, base,
                 spin);
    // the explicit unit lower trapezoidal V of the panel into LDS (rows past
    // mp and columns past nb are zero); the factored panel and V go out to
    // memory after the V^T V partial has been published, so that the
    // store-completion wait before the flag covers the partial alone
    __syncthreads();
    {
        double *vr = sh.red + threadIdx.x * (QR_NB + 1);
#pragma unroll
        for (int k = 0; k < QR_NB; ++k)
            vr[k] = (live && k < nb) ? (i > k ? a[k] : (i == k ? 1.0 : 0.0)) : 0.0;
    }
    __syncthreads();
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = blockIdx.x, G = gridDim.x;
    {
        const int ti = w & 1, tj = w >> 1;
        dbl4 acc = dbl4{0, 0, 0, 0};
        for (int kk = 0; kk < QR_RC; kk += 4) {
            const double *row = sh.red + (kk + lane / 16) * (QR_NB + 1);
            acc = mfma16(row[16 * ti + lane % 16], row[16 * tj + lane % 16], acc);
        }
        double *pg = Gpart + (size_t)g * QR_NB * QR_NB;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            coh_store(pg + (16 * ti + mfma_row<double>(lane, e)) + (size_t)(16 * tj + lane % 16) * QR_NB, acc[e]);
    }
    publish_fence();
    __syncthreads();
    if (t == 0) coh_store(flags + g, base + QR_NB + 1);
    // the factored panel and V (workgroup 0: after the sum of the V^T V
    // partials, its first wavefront after T)
    auto write_back = [&]() {
#pragma unroll
        for (int k = 0; k < QR_NB; ++k) {
            if (live && k < nb) {
                P[(size_t)k * ld + i] = a[k];
                Vb[(size_t)k * mp + i] = i > k ? a[k] : (i == k ? 1.0 : 0.0);
            }
        }
    };
    // a wait that ran out leaves this panel's factors invalid: report it in
    // the caller's error word (read back with the run's status)
    if (t == 0 && sh.bad && err) *err = 1;
    if (g != 0) {
        write_back();
        return;
    }
    if (t < G && t != 0) {
        int it = 0;
        while (spin < 0 || coh_load(flags + t) < base + QR_NB + 1) {
            if (spin < 0 || ++it > spin) { sh.bad = 1; break; }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    if (t == 0 && sh.bad && err) *err = 1;
    double *Gs = sh.red;   // G (ld QR_NB), the rows of V are no longer needed
    {
        // the four entries of this thread, the loads of eight partials at a
        // time in flight together, added in workgroup order
        constexpr int EPT = QR_NB * QR_NB / QR_RC;
        constexpr int QB = 8;
        double sacc[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) sacc[u] = 0.0;
        for (int q0 = 0; q0 < G; q0 += QB) {
            double v[QB][EPT];
#pragma unroll
            for (int q = 0; q < QB; ++q)
#pragma unroll
                for (int u = 0; u < EPT; ++u)
                    v[q][u] = q0 + q < G ? coh_load(Gpart + (size_t)(q0 + q) * QR_NB * QR_NB + t + u * QR_RC)
                                         : 0.0;
#pragma unroll
            for (int q = 0; q < QB; ++q)
#pragma unroll
                for (int u = 0; u < EPT; ++u)
                    if (q0 + q < G) sacc[u] += v[q][u];
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) Gs[t + u * QR_RC] = sacc[u];
    }
    __syncthreads();
    // the other wavefronts write their rows back while the first solves for T
    if (t >= 64) write_back();
    if (t < QR_NB) {
        const int j = t;
        const double poison = sh.bad ? __builtin_nan("") : 0.0;
        double c[QR_NB];
#pragma unroll
        for (int r = 0; r < QR_NB; ++r) c[r] = (r == j && j < nb) ? sh.tv[r] : 0.0;
#pragma unroll
        for (int r = QR_NB - 2; r >= 0; --r) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int k = r + 1; k < QR_NB; ++k) {
                if ((k - r) & 1) s0 = fma(Gs[k * QR_NB + r], c[k], s0);
                else s1 = fma(Gs[k * QR_NB + r], c[k], s1);
            }
            if (r < j) c[r] = -(r < nb ? sh.tv[r] : 0.0) * (s0 + s1);
        }
#pragma unroll
        for (int r = 0; r < QR_NB; ++r) T[(size_t)j * ldt + r] = (j < nb ? c[r] : 0.0) + poison;
    }
    if (t < 64) write_back();
}

// ---------------------------------------------------------------- in-block update
// C (mp x ncol) <- (I - V T^T V^T) C for a factored panel (V: mp x nb, ld ldv,
// explicit unit lower trapezoidal; T: nb x nb upper, ld ldt; nb <= 32,
// ncol <= 96), in one launch instead of the four of apply_block (split-K
// V^T C, its reduction, T^T W, C - V W).  Workgroup g holds rows 64g .. 64g+63
// of V and C in LDS and forms its partial P_g = V_g^T C_g on the matrix
// cores; the partials go out as tagged words (two per value, as in the
// panel), workgroup g sums a slice of the 32 ncol entries over all
// workgroups in workgroup order (four threads per entry, each a quarter of
// the workgroups, then the four quarters in order) and publishes the slice;
// every workgroup then reads all of W = V^T C, forms T^T W on the matrix
// cores and updates its rows.  Each of the two exchanges is one pass of loads
// with all of a thread's words in flight.  Needs every workgroup resident at
// once; the waits are bounded and one that runs out sets *err.
constexpr int QA_RB = 64;          // rows per workgroup
constexpr int QA_NC = 96;          // most columns of C
constexpr int QA_LDV = QR_NB + 1, QA_LDC = QA_NC + 1;
constexpr int QA_KW = QR_NB * QA_NC / 256;             // words of W per thread
constexpr int QA_K = (QR_NB * QA_NC + 255) / 256 + 1;  // slice words per thread: S G <= 32 QA_NC + G

__global__ __launch_bounds__(256) void qr_apply_coop(int mp, int nb, const double *__restrict__ V, int ldv,
                                                     const double *__restrict__ T, int ldt, int ncol,
                                                     double *__restrict__ C, int ldc,
                                                     unsigned long long *tw1, unsigned long long *tw2,
                                                     unsigned tag, int spin, int *err) {
    __shared__ double Vs[QA_RB * QA_LDV];
    __shared__ double Cs[QA_RB * QA_LDC];
    __shared__ double Ws[QR_NB * QA_LDC];     // W = V^T C, then T^T W
    __shared__ double Ts[QR_NB * QA_LDV];
    __shared__ double Ps[256 * QA_K];         // the slice's words of every workgroup
    __shared__ double red[256];
    __shared__ int bad;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int g = blockIdx.x, G = gridDim.x;
    const int r0 = g * QA_RB;
    if (t == 0) bad = 0;
    // rows of V (columns past nb zero) and of C (columns past ncol zero), T:
    // every load of a thread in flight together, then the LDS stores
    {
        constexpr int NV = QA_RB * QR_NB / 256, NC = QA_RB * QA_NC / 256, NT = QR_NB * QR_NB / 256;
        double rv[NV], rc[NC], rt[NT];
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int e = t + 256 * u, i = e % QA_RB, k = e / QA_RB;
            rv[u] = (r0 + i < mp && k < nb) ? V[(size_t)k * ldv + r0 + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int e = t + 256 * u, i = e % QA_RB, c = e / QA_RB;
            rc[u] = (r0 + i < mp && c < ncol) ? C[(size_t)c * ldc + r0 + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int e = t + 256 * u, i = e % QR_NB, k = e / QR_NB;
            rt[u] = (i < nb && k < nb) ? T[(size_t)k * ldt + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int e = t + 256 * u;
            Vs[(e % QA_RB) * QA_LDV + e / QA_RB] = rv[u];
        }
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int e = t + 256 * u;
            Cs[(e % QA_RB) * QA_LDC + e / QA_RB] = rc[u];
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int e = t + 256 * u;
            Ts[(e % QR_NB) * QA_LDV + e / QR_NB] = rt[u];
        }
    }
    for (int e = t; e < QR_NB * QA_LDC; e += 256) Ws[e] = 0.0;   // columns past ncol stay zero
    __syncthreads();
    const int nct = cdiv(ncol, 16);   // 16-column tiles of C
    // 1. P_g = V_g^T C_g (32 x ncol), 2 x nct tiles over the four wavefronts
    for (int tile = w; tile < 2 * nct; tile += 4) {
        const int ti = tile & 1, tj = tile >> 1;
        dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < QA_RB; s4 += 4) {
            const int k = s4 + lane / 16;
            acc = mfma16(Vs[k * QA_LDV + 16 * ti + lane % 16], Cs[k * QA_LDC + 16 * tj + lane % 16], acc);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 16 * ti + mfma_row<double>(lane, e), c = 16 * tj + lane % 16;
            if (c < ncol) tag_store(tw1 + ((size_t)g * QR_NB * QA_NC + r * QA_NC + c) * 2, acc[e], tag);
        }
    }
    // 2. this workgroup's slice of the 32 ncol entries of W, summed over the
    // workgroups.  Every (workgroup, entry) word of the slice is loaded in
    // one pass (entries fastest, so the loads of a wavefront are contiguous),
    // kept in LDS, then four threads per entry sum a quarter of the
    // workgroups each and the four quarters are added in order.
    const int E = QR_NB * ncol;
    const int S = cdiv(E, G);
    const int e_lo = g * S;
    const int SL = min(S, E - e_lo);   // entries of this slice (none past E)
    {
        const unsigned long long *pp[QA_K];
        double v[QA_K];
        unsigned mask = 0;
#pragma unroll
        for (int u = 0; u < QA_K; ++u) {
            const int i = t + 256 * u, q = i / S, el = i - q * S;
            const bool ok = q < G && el < SL;
            const int e = ok ? e_lo + el : 0, r = e / ncol, c = e - r * ncol;
            pp[u] = tw1 + ((size_t)(ok ? q : 0) * QR_NB * QA_NC + r * QA_NC + c) * 2;
            if (ok) mask |= 1u << u;
            v[u] = 0.0;
        }
        if (!tag_load<QA_K>(pp, mask, tag, spin, v)) bad = 1;
#pragma unroll
        for (int u = 0; u < QA_K; ++u)
            if (mask & (1u << u)) Ps[t + 256 * u] = v[u];
    }
    __syncthreads();
    const int Gq = cdiv(G, 4);
    for (int e0 = 0; e0 < SL; e0 += 64) {
        const int el = e0 + (t >> 2), h = t & 3;
        double part = 0.0;
        if (el < SL)
            for (int q = h * Gq; q < min(G, (h + 1) * Gq); ++q) part += Ps[q * S + el];
        red[t] = part;
        __syncthreads();
        if (h == 0 && el < SL) {
            const double sum = ((red[t] + red[t + 1]) + red[t + 2]) + red[t + 3];
            tag_store(tw2 + (size_t)(e_lo + el) * 2, sum, tag);
        }
        __syncthreads();
    }
    // 3. all of W in one pass, then T^T W on the matrix cores
    {
        const unsigned long long *pp[QA_KW];
        double v[QA_KW];
        unsigned mask = 0;
#pragma unroll
        for (int u = 0; u < QA_KW; ++u) {
            const int e = t + 256 * u;
            pp[u] = tw2 + (size_t)(e < E ? e : 0) * 2;
            if (e < E) mask |= 1u << u;
            v[u] = 0.0;
        }
        if (!tag_load<QA_KW>(pp, mask, tag, spin, v)) bad = 1;
#pragma unroll
        for (int u = 0; u < QA_KW; ++u) {
            const int e = t + 256 * u;
            if (e < E) Ws[(e / ncol) * QA_LDC + e % ncol] = v[u];
        }
    }
    __syncthreads();
    {
        constexpr int TPW = (2 * (QA_NC / 16) + 3) / 4;   // tiles of T^T W per wavefront
        dbl4 acc[TPW];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int tile = w + 4 * u, ti = tile & 1, tj = tile >> 1;
            acc[u] = dbl4{0, 0, 0, 0};
            if (tile < 2 * nct) {
#pragma unroll
                for (int s4 = 0; s4 < QR_NB; s4 += 4) {
                    const int k = s4 + lane / 16;
                    acc[u] = mfma16(Ts[k * QA_LDV + 16 * ti + lane % 16], Ws[k * QA_LDC + 16 * tj + lane % 16],
                                    acc[u]);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int tile = w + 4 * u, ti = tile & 1, tj = tile >> 1;
            if (tile < 2 * nct) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = 16 * ti + mfma_row<double>(lane, e), c = 16 * tj + lane % 16;
                    Ws[i * QA_LDC + c] = acc[u][e];
                }
            }
        }
    }
    __syncthreads();
    // 4. C_g <- C_g - V_g (T^T W): 4 x nct tiles over the wavefronts
    for (int tile = w; tile < 4 * nct; tile += 4) {
        const int ri = tile & 3, tj = tile >> 2;
        dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < QR_NB; s4 += 4) {
            const int k = s4 + lane / 16;
            acc = mfma16(Vs[(16 * ri + lane % 16) * QA_LDV + k], Ws[k * QA_LDC + 16 * tj + lane % 16], acc);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 16 * ri + mfma_row<double>(lane, e), c = 16 * tj + lane % 16;
            if (r0 + i < mp && c < ncol) C[(size_t)c * ldc + r0 + i] = Cs[i * QA_LDC + c] - acc[e];
        }
    }
    if (t == 0 && bad && err) *err = 1;
}

// Clears the one-launch panel's flags and tagged words, and those of the
// one-launch in-block update, before a factorisation.
__global__ void qr_flags_zero(int n, int *flags, int nt, unsigned long long *tp, int nh,
                              unsigned long long *th, int na, unsigned long long *ta) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) flags[e] = 0;
    if (e < nt) tp[e] = 0ull;
    if (e < nh) th[e] = 0ull;
    if (e < na) ta[e] = 0ull;
}

// T (nb x nb upper, zeros below, ld ldt) of the compact-WY form
// H_0 ... H_{nb-1} = I - V T V^T, from G = V^T V (ld QR_NB) and tau.  T is the
// inverse of diag(1/tau) + striu(G); the columns of that triangular system
// are independent, so lane j solves for column j by back substitution,
// T_jj = tau_j, T_ij = -tau_i sum_{i<k<=j} G_ik T_kj for i = j-1 .. 0, with
// no exchange between lanes.  A zero tau (an identity reflector) gives a zero
// row and column, with no division.  The sums run in registers, over the
// whole column with masked terms, so every lane follows the same unrolled
// sequence and reads the same entry of G at a time.
__global__ __launch_bounds__(64) void qr_build_t(int nb, const double *vtv, const double *tau,
                                                 double *T, int ldt) {
    __shared__ double G[QR_NB * QR_NB];
    __shared__ double ts[QR_NB];
    const int t = threadIdx.x;
    // entries of G outside nb x nb are never written by the product: zero them
#pragma unroll
    for (int k = 0; k < QR_NB * QR_NB / 64; ++k) {
        const int e = t + 64 * k;
        G[e] = (e % QR_NB < nb && e / QR_NB < nb) ? vtv[e] : 0.0;
    }
    if (t < QR_NB) ts[t] = t < nb ? tau[t] : 0.0;
    __syncthreads();
    const int j = t;
    double c[QR_NB];
#pragma unroll
    for (int i = 0; i < QR_NB; ++i) c[i] = (i == j && j < nb) ? ts[i] : 0.0;
#pragma unroll
    for (int i = QR_NB - 2; i >= 0; --i) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = i + 1; k < QR_NB; ++k) {
            // c[k] is zero for k > j, so the masked terms add nothing
            if ((k - i) & 1) s0 = fma(G[k * QR_NB + i], c[k], s0);
            else s1 = fma(G[k * QR_NB + i], c[k], s1);
        }
        if (i < j) c[i] = -ts[i] * (s0 + s1);
    }
    if (j < QR_NB) {
#pragma unroll
        for (int i = 0; i < QR_NB; ++i) T[(size_t)j * ldt + i] = j < nb ? c[i] : 0.0;
    }
}

// Vb (mp x nb, ld ldv) = explicit unit lower trapezoidal V of the panel.
__global__ __launch_bounds__(256) void qr_extract_v(int mp, int nb, const double *P, int ld,
                                                    double *Vb, int ldv) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)mp * nb) return;
    const int i = (int)(e % mp), k = (int)(e / mp);
    const double v = (i < k) ? 0.0 : (i == k ? 1.0 : P[(size_t)k * ld + i]);
    Vb[(size_t)k * ldv + i] = v;
}

size_t qr_t_doubles(int n) { return (size_t)cdiv(n, QR_NBO) * QR_NBO * QR_NBO; }

size_t qr_scratch_doubles(int m, int ncols_max, size_t *split_elems) {
    const int G = cdiv(m, QR_RC);
    const size_t se = (size_t)8 * QR_NBO * (size_t)ncols_max;
    if (split_elems) *split_elems = se;
    const int GA = cdiv(m, QA_RB);
    const size_t ta = GA <= 256 ? (size_t)2 * (GA + 1) * QR_NB * QA_NC : 0;   // in-block update words
    return (size_t)2 * G * QR_NB + 2 * QR_NB + (size_t)4 * G * QR_NB + 4 * QR_NB + ta +
           (size_t)G * QR_NB * QR_NB + (size_t)m * QR_NB +
           (size_t)m * QR_NBO + (size_t)QR_NBO * QR_NBO + (size_t)QR_NB * QR_NB +
           2 * (size_t)QR_NBO * ncols_max + se + (size_t)(G + 63) / 2 + 128;
}

void qr_scratch_carve(QRScratch &q, double *base, int m, int ncols_max) {
    const int G = cdiv(m, QR_RC);
    size_t se;
    qr_scratch_doubles(m, ncols_max, &se);
    double *p = base;
    q.part = p; p += (size_t)2 * G * QR_NB;
    q.head = p; p += 2 * QR_NB;
    q.tpart = (unsigned long long *)p; p += (size_t)4 * G * QR_NB;
    q.thead = (unsigned long long *)p; p += 4 * QR_NB;
    {
        const int GA = cdiv(m, QA_RB);
        if (GA <= 256) {
            q.tw1 = (unsigned long long *)p; p += (size_t)2 * GA * QR_NB * QA_NC;
            q.tw2 = (unsigned long long *)p; p += (size_t)2 * QR_NB * QA_NC;
            q.tw_words = 2 * (GA + 1) * QR_NB * QA_NC;
        } else {
            q.tw1 = q.tw2 = nullptr;
            q.tw_words = 0;
        }
    }
    q.vtv = p; p += (size_t)G * QR_NB * QR_NB;
    q.vb = p; p += (size_t)m * QR_NB;
    q.vbo = p; p += (size_t)m * QR_NBO;
    q.go = p; p += (size_t)QR_NBO * QR_NBO;
    q.tp = p; p += (size_t)QR_NB * QR_NB;
    q.w1 = p; p += (size_t)QR_NBO * ncols_max;
    q.w2 = p; p += (size_t)QR_NBO * ncols_max;
    q.split = p; p += se;
    q.split_elems = se;
    q.flags = (int *)(p + 32);
}

static void extract_v(hipStream_t s, int mp, int nb, const double *P, int ld, double *vb) {
    const size_t tot = (size_t)mp * nb;
    hipLaunchKernelGGL(qr_extract_v, dim3((unsigned)cdivl((long long)tot, 256)), dim3(256), 0, s,
                       mp, nb, P, ld, vb, mp);
}

// Factor one panel (mp x nb at P), leave its explicit V in Vb and build its T
// from V^T V (FP64 matrix-core product).
// Workgroups of qr_panel_coop that the current device holds at once (its
// compute units times the kernel's occupancy per unit); cached per device.
static int coop_capacity() {
    static std::atomic<int> cap[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 0;
    }
    int c = cap[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
    int ncu = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)qr_panel_coop, QR_RC, 0) !=
            hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    c = ncu * per_cu;
    cap[dev].store(c, std::memory_order_relaxed);
    return c;
}

// Workgroups of qr_apply_coop that the current device holds at once; cached.
static int apply_capacity() {
    static std::atomic<int> cap[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 0;
    }
    int c = cap[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
    int ncu = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)qr_apply_coop, 256, 0) !=
            hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    c = ncu * per_cu;
    cap[dev].store(c, std::memory_order_relaxed);
    return c;
}

// The in-block update C <- (I - V T^T V^T) C of a panel in one launch, when
// its row blocks (8 to 256 of them) all fit on the device; false otherwise
// (nothing launched, the caller takes apply_block).
static bool apply_inblock(hipStream_t s, int mp, int nb, const double *T, int ldt, int ncol, double *C,
                          int ldc, const double *vb, QRScratch &q, unsigned tag) {
    const int G = cdiv(mp, QA_RB);
    if (!q.tw1 || G < 8 || G > 256 || ncol > QA_NC || nb > QR_NB || G > apply_capacity()) return false;
    if (q.kc) q.kc->begin(s, 8, (2.0 * mp * ncol + (double)mp * nb) * sizeof(double),
                          4.0 * mp * nb * ncol + 2.0 * nb * nb * ncol);
    hipLaunchKernelGGL(qr_apply_coop, dim3(G), dim3(256), 0, s, mp, nb, vb, mp, T, ldt, ncol, C, ldc,
                       q.tw1, q.tw2, tag, q.spin == 0 ? QR_COOP_SPIN : q.spin, q.err);
    if (q.kc) q.kc->end(s);
    return true;
}

static void panel_factor(hipStream_t s, int mp, int nb, double *P, int ld, double *tau,
                         double *T, int ldt, QRScratch &q, int panel) {
    const int G = cdiv(mp, QR_RC);
    // the one-launch panel waits on every one of its workgroups, so it runs
    // only when all of them fit on the device at once; its waits are bounded
    // all the same (another stream may hold compute units), and one that runs
    // out is reported through q.err
    if (G <= QR_COOP_MAXG && G <= coop_capacity()) {
        // algorithmic work: the panel read and written once, 2 mp nb^2 flops
        if (q.kc) q.kc->begin(s, 7, 2.0 * mp * nb * sizeof(double), 2.0 * mp * nb * nb);
        // the panel, its explicit V and its T in one launch
        hipLaunchKernelGGL(qr_panel_coop, dim3(G), dim3(QR_RC), 0, s, mp, nb, P, ld, q.tpart, q.thead,
                           tau, q.flags, panel * 64, q.vb, q.vtv, T, ldt, q.err,
                           q.spin == 0 ? QR_COOP_SPIN : q.spin);
        if (q.kc) q.kc->end(s);
    } else {
        hipLaunchKernelGGL(qr_panel_init, dim3(G), dim3(QR_RC), 0, s, mp, nb, P, ld, q.part, q.head);
        for (int j = 0; j < nb; ++j)
            hipLaunchKernelGGL(qr_panel_step, dim3(G), dim3(QR_RC), 0, s, j, mp, nb, G, P, ld,
                               q.part, q.head, tau);
        extract_v(s, mp, nb, P, ld, q.vb);
        gemm<double>(s, true, false, nb, nb, mp, 1.0, q.vb, mp, q.vb, mp, 0.0, q.vtv, QR_NB, q.split,
                     q.split_elems, q.kc);
        hipLaunchKernelGGL(qr_build_t, dim3(1), dim3(64), 0, s, nb, q.vtv, tau, T, ldt);
    }
}

// C (mp x ncol) <- (I - V T' V^T) C with T' = T (trans = false) or T^T; V
// explicit in vb (ld mp), T with ld ldt.
static void apply_block(hipStream_t s, bool transT, int mp, int nb, const double *T, int ldt,
                        int ncol, double *C, int ldc, const double *vb, QRScratch &q) {
    gemm<double>(s, true, false, nb, ncol, mp, 1.0, vb, mp, C, ldc, 0.0, q.w1, nb, q.split,
                 q.split_elems, q.kc);
    gemm<double>(s, transT, false, nb, ncol, nb, 1.0, T, ldt, q.w1, nb, 0.0, q.w2, nb, nullptr, 0,
                 q.kc);
    gemm<double>(s, false, false, mp, ncol, nb, -1.0, vb, mp, q.w2, nb, 1.0, C, ldc, nullptr, 0,
                 q.kc);
}

// Two-level blocked Householder QR: 32-wide panels (one launch each) update
// the rest of their 128-column outer block with the panel's compact-WY form;
// the outer block's T is assembled from the panel T's on its diagonal and
// the blocks above them, T(0:r, c) = -T(0:r, 0:r) (V(:, 0:r)^T V_c) T_c (the
// column recurrence of the compact-WY form taken a panel at a time), and the
// trailing columns take one compact-WY product of depth 128.
void qr_factor(hipStream_t s, int m, int n, double *A, int lda, double *tau, double *Tall,
               QRScratch &q) {
    const int gmax = cdiv(m, QR_RC);
    if (gmax <= QR_COOP_MAXG) {
        const int nt = 4 * gmax * QR_NB;   // tagged sums of both column parities
        const int na = q.tw1 ? q.tw_words : 0;       // tw2 sits after the carve's tw1, not the call's
        hipLaunchKernelGGL(qr_flags_zero, dim3(cdiv(nt > na ? nt : na, 256)), dim3(256), 0, s, gmax,
                           q.flags, nt, q.tpart, 4 * QR_NB, q.thead, na, q.tw1);
    }
    int panel = 0;
    for (int c0o = 0, ob = 0; c0o < n; c0o += QR_NBO, ++ob) {
        const int nbo = min(QR_NBO, n - c0o);
        const int mpo = m - c0o;
        double *To = Tall + (size_t)ob * QR_NBO * QR_NBO;
        zero_pad_fill(s, QR_NBO, QR_NBO, To, QR_NBO);
        for (int c0 = c0o; c0 < c0o + nbo; c0 += QR_NB, ++panel) {
            const int nb = min(QR_NB, c0o + nbo - c0);
            const int mp = m - c0;
            double *P = A + (size_t)c0 * lda + c0;
            double *Tp = To + (size_t)(c0 - c0o) * QR_NBO + (c0 - c0o);
            panel_factor(s, mp, nb, P, lda, tau + c0, Tp, QR_NBO, q, panel);
            const int nin = c0o + nbo - c0 - nb;   // the rest of the outer block
            if (nin > 0 && !apply_inblock(s, mp, nb, Tp, QR_NBO, nin, P + (size_t)nb * lda, lda, q.vb, q,
                                          (unsigned)(panel * 64 + 48)))
                apply_block(s, true, mp, nb, Tp, QR_NBO, nin, P + (size_t)nb * lda, lda, q.vb, q);
        }
        double *Po = A + (size_t)c0o * lda + c0o;
        extract_v(s, mpo, nbo, Po, lda, q.vbo);
        if (nbo > QR_NB) {
            gemm<double>(s, true, false, nbo, nbo, mpo, 1.0, q.vbo, mpo, q.vbo, mpo, 0.0, q.go, QR_NBO,
                         q.split, q.split_elems, q.kc);
            for (int r = QR_NB; r < nbo; r += QR_NB) {
                const int cb = min(QR_NB, nbo - r);
                gemm<double>(s, false, false, r, cb, r, 1.0, To, QR_NBO, q.go + (size_t)r * QR_NBO,
                             QR_NBO, 0.0, q.w1, r, nullptr, 0, q.kc);
                gemm<double>(s, false, false, r, cb, cb, -1.0, q.w1, r, To + (size_t)r * QR_NBO + r,
                             QR_NBO, 0.0, To + (size_t)r * QR_NBO, QR_NBO, nullptr, 0, q.kc);
            }
        }
        const int nt = n - c0o - nbo;
        if (nt > 0)
            apply_block(s, true, mpo, nbo, To, QR_NBO, nt, Po + (size_t)nbo * lda, lda, q.vbo, q);
    }
}

void qr_apply_left(hipStream_t s, bool trans, int m, int k, const double *Qf, int ldq,
                   const double *Tall, int ncol, double *C, int ldc, QRScratch &q) {
    const int nob = cdiv(k, QR_NBO);
    for (int t = 0; t < nob; ++t) {
        const int ob = trans ? t : nob - 1 - t;
        const int c0 = ob * QR_NBO;
        const int nb = min(QR_NBO, k - c0);
        const int mp = m - c0;
        extract_v(s, mp, nb, Qf + (size_t)c0 * ldq + c0, ldq, q.vbo);
        apply_block(s, trans, mp, nb, Tall + (size_t)ob * QR_NBO * QR_NBO, QR_NBO, ncol, C + c0, ldc,
                    q.vbo, q);
    }
}

} // namespace mpj
