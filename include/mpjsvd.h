/*
 * mpjsvd — mixed-precision one-sided Jacobi SVD for AMD Instinct MI355X (gfx950).
 *
 * Computes A = U diag(S) V^T for a dense FP64 matrix A (m x n, m >= n) to high
 * relative accuracy, following Gao, Ma and Shao, "A mixed precision Jacobi SVD
 * algorithm" (arXiv 2209.04626):
 *   svd_plain  — Algorithm 2 + Algorithm 1: QR with column pivoting, an LQ
 *                step, FP64 one-sided Jacobi sweeps with accumulated V.
 *   svd_mixed  — Algorithm 4: the same QR preconditioning with pivots chosen in
 *                FP32 (Algorithm 5), the branch tests of Section 3.5, an FP32
 *                one-sided Jacobi SVD without V (Section 3.2), the switch
 *                Q = qr(X^T U_low), Y = X Q (Section 3.3), and FP64 one-sided
 *                Jacobi refinement on Y (Section 3.4).
 *   svd_batched — the mixed path over many small matrices of uneven size in
 *                one persistent-kernel launch.
 *   svd_backward — the adjoint of the SVD (not in the paper): gA from U, S, V
 *                and cotangents gU, gS, gV.
 *
 * Conventions shared by every entry point:
 *   - Matrices are FP64, column-major, with a leading dimension (ld >= rows).
 *   - All matrix/vector pointers are DEVICE pointers owned by the caller.  The
 *     library never allocates device memory inside these calls: scratch space
 *     is the caller's `work` buffer, sized by the matching *_workspace_size
 *     query.  A is never modified.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on that stream.  By default svd_plain / svd_mixed read
 *     convergence and branch flags back to the host between sweeps, so they
 *     return only when the result is complete; with svd_opts.capture = 1
 *     they are stream-ordered and graph-capturable like svd_batched and
 *     svd_backward (every decision on the device, svd_info written there).
 *   - The return value checks arguments only, LAPACK style: 0 on success,
 *     -k when argument k is invalid (k counts from 1), -100 on a HIP runtime
 *     error.  The numerical outcome is in svd_info.status.
 *   - Calls on different streams with different workspaces may run
 *     concurrently; the library keeps no mutable global state.
 */
#ifndef MPJSVD_H
#define MPJSVD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* svd_info.status values */
#define SVD_OK 0
#define SVD_WARN_NOCONV 1        /* the FP64 sweeps hit their cap (the FP32
                                    stage may stop at its cap: it only
                                    preconditions, Section 4) */
#define SVD_ERR_NONFINITE 2      /* A holds NaN or Inf; outputs undefined   */
#define SVD_WARN_RANK_DEFICIENT 3 /* some sigma_i == 0; U(:, i) set to zero */
#define EIG_ERR_CLUSTER 4        /* eig_mixed: a block of equal |eigenvalue|
                                    larger than 64; outputs undefined       */
#define SVD_ERR_WAIT_TIMEOUT 5   /* a bounded wait between the workgroups of
                                    a one-launch kernel (the Householder
                                    panel) ran out, e.g. because another
                                    stream held compute units; outputs
                                    undefined (the one-launch pivot pass
                                    instead falls back to per-step launches
                                    and does not report this)              */
#define SVD_ERR_BREAKDOWN 6      /* a singular value came out NaN or Inf
                                    from finite input; outputs undefined    */
#define SVD_WARN_VSOLVE 7        /* svd_opts.capture = 1, v_method 1: the
                                    solved V_X = X^{-1} Y failed its
                                    orthogonality test and the fallback
                                    (which the host drives) did not run; S
                                    and U are valid, V is not accurate      */

/* svd_opts.branch / svd_info.branch_taken (Algorithm 4's special cases) */
#define SVD_BRANCH_AUTO 0
#define SVD_BRANCH_LOW 1         /* run the FP32 stage and the switch       */
#define SVD_BRANCH_SKIP 2        /* Q = I: go straight to FP64 sweeps       */

#define SVD_ERR_HIP (-100)
#define SVD_ERR_SCRATCH_LIMIT (-101) /* svd_backward_noalloc: the problem needs
                                        more than its fixed scratch array     */

typedef struct {
    /* Section 7.1 parameters.  tol_alg is recorded only: the low-precision
       SVD is always the FP32 one-sided Jacobi method. */
    double tol_alg;        /* 1e-2 */
    double tol_orth;       /* 1e-5: skip the FP32 stage when
                              max|X_t^T X_t - I| <= tol_orth (Section 3.5) */
    double tol_cond_coef;  /* 1.5: skip when max|r_ii|/min|r_ii| <=
                              tol_cond_coef * n^(1/4) (Section 3.5) */
    double small_col_rel;  /* a column of X is "small" when its norm is
                              <= small_col_rel * max column norm; 2^-53 */
    double small_col_frac; /* skip when at least ceil(frac * n) trailing
                              columns of X are small; 0.25 */
    double eps_work;       /* FP64 rotation threshold; 0 -> sqrt(n) 2^-53 */
    double eps_low;        /* FP32 rotation threshold; 0 -> sqrt(n) 2^-24 */
    int maxsweep_low;      /* FP32 sweep cap (30) */
    int maxsweep_work;     /* FP64 sweep cap (30) */
    int want_u;            /* 1: form U (m x n) */
    int want_v;            /* 1: form V (n x n); 0 skips V accumulation */
    int branch;            /* SVD_BRANCH_AUTO / _LOW / _SKIP */
    int switch_method;     /* 1: Q = qr(X^T U_low), the switch of Algorithm 4
                              (Section 3.3, default); 2: Q = qr(fp64(V_low))
                              with V_low accumulated in the FP32 stage (the
                              switch of Algorithm 3, compared in Section 6),
                              Y = X Q; 3: Algorithm 3 itself, Q =
                              qr(P Q2^T fp64(V_low)) and the FP64 sweeps on
                              Y = A1 Q (A1 = A, or R1 when m > n) with V
                              accumulated; the workspace query depends on it */
    int pivot_precision;   /* 32 (Algorithm 5) or 64 (plain xGEQP3) */
    int sign_normalize;    /* 1: make the largest |V(k, i)| of each column
                              positive (first k on ties), negating U(:, i)
                              with it */
    int block_cols;        /* Jacobi block width b (16 or 32) of both stages;
                              0 = per stage (block_cols_low / _work) */
    int inner_sweeps;      /* cap on the Jacobi sweeps run on each 2b x 2b
                              Gram block per block pair; 0 = auto (1) */
    int kernel_timing;     /* 1: time the QRCP pivot pass as one interval
                              (class SVD_K_QRCP, negligible overhead);
                              2: bracket every launch of the Jacobi, pivot,
                              QR panel and GEMM kernels with HIP events
                              (per-class totals; adds host work and a little
                              time); 100 + c: bracket only the launches of
                              class c (SVD_K_*), the others run without
                              events.  Results in svd_info.kern_*. */
    double low_stop_off;   /* end the FP32 stage after a sweep in which
                              every |g_pq| met was <= low_stop_off
                              sqrt(g_pp g_qq): the next sweep would only
                              rotate at the FP32 rounding level.  0 (default)
                              -> sqrt(n) eps_low; < 0: only the eps_low rule */
    int block_cols_low;    /* b of the FP32 stage (16 or 32), over block_cols;
                              0 = block_cols, else the tuning table, else 16 */
    int block_cols_work;   /* b of the FP64 stage (16 or 32), over block_cols;
                              0 = block_cols, else the tuning table, else
                              32 for n >= 512 and 16 below */
    int v_method;          /* right singular vectors (Section 3.4):
                              0: rotations accumulated through every FP64
                              sweep (the plain path's default);
                              1: FP64 sweeps without V, then V_X = X^{-1} Y by
                              a triangular solve with X = L, accepted when
                              max|V_X^T V_X - I| <= tol_vsolve, else V_X from
                              the QR of X^T U_X followed by FP64 sweeps with
                              accumulation (the mixed path's default) */
    int diagnostics;       /* 1: also measure svd_info.orth_y (one more FP64
                              Gram product); 2: that, and leave a copy of Y
                              as the FP64 sweeps start (after the switch,
                              before the Y2 safeguard; n x n, ld = n rounded
                              up to a multiple of 64) in the workspace at
                              byte offset svd_diag_y_offset(); 0 (default):
                              skip */
    double tol_vsolve;     /* acceptance bound of v_method 1; 0 -> n 2^-50 */
    int inner_pairs;       /* pairs rotated in a block pair's inner solve:
                              0 (default): all pairs of its 2b columns in the
                              first round of a sweep, then only the b^2 pairs
                              between the two blocks (each pair of columns is
                              rotated about once per sweep, as in Algorithm 1);
                              1: all pairs in every round */
    double tol_cluster;    /* eig_mixed only: consecutive singular values of
                              A Q with relative gap <= tol_cluster form one
                              block of U^T A U; 0 -> 1e-8 */
    int y2_safeguard;      /* 1 (default): after the switch, the columns j
                              of Y whose normalised Gram row has an
                              off-diagonal max|c_ij| > tol_y2 form Y2; if there
                              are two or more, FP64 sweeps run on Y2 alone
                              before the sweeps over all of Y (Section 3.4);
                              costs one FP64 Gram product; 0: off */
    double tol_y2;         /* 0 -> 64 sqrt(n) 2^-24 */
    int kernel_timing_every; /* with kernel_timing >= 2: clock only every
                              k-th launch of each kernel class (the first
                              launch always; a sample that keeps the events'
                              cost out of the rest of the launches); 0 or 1 =
                              every launch */
    int wait_polls;        /* polls of each bounded cross-workgroup wait
                              (one-launch pivot pass, Householder panel)
                              before it gives up: 0 = default (2^22);
                              -1 = give up at the first check (a test hook
                              for the time-out paths: the pivot pass then
                              falls back to per-step launches, the panel
                              reports SVD_ERR_WAIT_TIMEOUT, the fused FP32
                              round restarts the FP32 stage with separate
                              kernels); < -1 invalid */
    int fused_rounds;      /* FP32 stage without V_low (switch method 1):
                              0 (default) = one launch per block-Jacobi round
                              (Gram, inner solve and update fused, 32-column
                              blocks) for n > 2048 when the device holds the
                              whole grid at once, else separate kernels;
                              1 = the fused round at any n where it fits;
                              -1 = always the separate kernels */
    int capture;           /* 1: stream-ordered, with no host
                              synchronisation inside the call, so it can be
                              captured in a HIP graph and replayed.  The
                              branch tests of Section 3.5, the stopping rules
                              of every sweep stage and v_method 1's
                              acceptance test are decided on the device;
                              info must then be DEVICE memory (or NULL) and
                              is written by the call's last kernel.  Every
                              sweep up to maxsweep_low / maxsweep_work is
                              enqueued and those after the stop exit at
                              once, so the caps set the launch count.  The
                              FP32 stage and the switch are enqueued even
                              when the tests choose the skip branch (their
                              result is then replaced by Y = X); all three
                              tests are measured.  Not available here:
                              kernel_timing (must be 0), stage_ms (0), the
                              Y2 safeguard (not run), v_method 1's fallback
                              (SVD_WARN_VSOLVE instead), restarting the FP32
                              stage after a fused round's wait ran out (the
                              stage stops there: fused_fallback = 2, still a
                              valid preconditioner by Proposition 1) and the
                              step-by-step pivot pass after the one-launch
                              pass's wait ran out (SVD_ERR_WAIT_TIMEOUT);
                              switch_method 3 needs branch = SVD_BRANCH_LOW.
                              0 (default): the host-synchronised call. */
    int half_sweeps;       /* three-precision variant (the GPU outlook of
                              the paper's conclusions): the first sweeps of
                              the FP32 stage form their Gram blocks with
                              BF16 matrix-core products (operands rounded
                              to BF16, FP32 sums); rotation angles, tests,
                              the update and Y stay FP32 (FP64 angles).  At
                              most half_sweeps such sweeps, fewer once a
                              sweep ends with every relative off-diagonal
                              <= half_stop_off; then the FP32 sweeps
                              continue on the same Y.  Only where the fused
                              round runs (see fused_rounds); default 4;
                              0 = off */
    double half_stop_off;  /* 0 -> 2^-6 */
    int half_storage;      /* 1: those sweeps also keep Y in BF16 (the
                              update's result rounded to BF16, Y widened to
                              FP32 after them); 0 (default): Y stays FP32 */
} svd_opts;

/* Kernel classes reported by svd_info.kern_* (kernel_timing 1: SVD_K_QRCP
   only; 2: all of them) */
#define SVD_K_GRAM32 0     /* Jacobi Gram blocks, FP32 stage          */
#define SVD_K_INNER32 1    /* Jacobi 2b x 2b inner solve, FP32 stage  */
#define SVD_K_UPDATE32 2   /* Jacobi block rotation update, FP32      */
#define SVD_K_GRAM64 3
#define SVD_K_INNER64 4
#define SVD_K_UPDATE64 5
#define SVD_K_QRCP 6       /* pivot pass launches (one, or one per step) */
#define SVD_K_QRPANEL 7    /* Householder panel factorisations        */
#define SVD_K_GEMM 8       /* matrix-core GEMMs (with their split-K sums) */
#define SVD_K_ROUND32 9    /* fused FP32 Jacobi round (Gram, inner solve
                              and update in one launch)               */
#define SVD_K_TRSM 10      /* diagonal-block solves of V_X = X^-1 Y     */
#define SVD_K_ROUND16 11   /* fused round of the BF16 sweeps (BF16 Gram
                              products; Y in BF16 with half_storage)   */
#define SVD_K_NCLASS 12

typedef struct {
    int status;            /* SVD_OK / SVD_WARN_* / SVD_ERR_* */
    int branch_taken;      /* SVD_BRANCH_LOW or SVD_BRANCH_SKIP */
    int sweeps_low;        /* FP32 sweeps executed */
    int sweeps_work;       /* FP64 sweeps executed */
    int n_small;           /* trailing small columns of X */
    double orth;           /* max|X_t^T X_t - I| (FP32), -1 if not computed */
    double cond_r;         /* max|r_ii| / min|r_ii| of the pivoted R */
    float stage_ms[8];     /* ingest+tall QR, pivots, QR, LQ, tests,
                              FP32 sweeps, switch, FP64 sweeps+finalise */
    float off_low[32];     /* per FP32 sweep: max |g_pq| / sqrt(g_pp g_qq)
                              on the fresh Gram blocks (convergence trace) */
    float off_work[32];    /* the same for the FP64 sweeps */
    float kern_ms[SVD_K_NCLASS];   /* summed kernel durations per class */
    int kern_calls[SVD_K_NCLASS];  /* launches per class */
    double kern_bytes[SVD_K_NCLASS]; /* algorithmic HBM bytes of those launches */
    double kern_flops[SVD_K_NCLASS]; /* algorithmic flops of those launches */
    int v_method_taken;    /* -1: V not wanted; 0: accumulated; 1: triangular
                              solve accepted; 2: solve rejected, V_X from the
                              QR of X^T U_X and further sweeps; 3 (capture =
                              1): solve rejected, no fallback */
    int sweeps_vfix;       /* FP64 sweeps of that fallback */
    double orth_vx;        /* max|V_X^T V_X - I| of the solve, -1 if none */
    double orth_y;         /* diagnostics: max|D^-1 Y^T Y D^-1 - I| of Y
                              after the switch (D = column norms), -1 if not
                              measured */
    int n_y2;              /* columns in Y2 (0: the safeguard did not act) */
    int sweeps_y2;         /* FP64 sweeps run on Y2 alone */
    int fused_fallback;    /* 1: a fused FP32 round gave up waiting and the
                              FP32 stage was run again with separate kernels;
                              2 (capture = 1): the FP32 stage stopped there */
    int sweeps_half;       /* BF16 sweeps run before the FP32 sweeps */
} svd_info;

/* Load the tuning table measured by the autotuner (not part of the paper's
   method): JSON text of the form
     {"arch": "gfx950",
      "single":  [{"nmax": N, "b_low": 16|32, "b_work": 16|32}, ...],
      "batched": [{"nmax": N, "wg_per_cu": W}, ...]}
   An entry applies to problems with n <= nmax; the smallest such nmax wins.
   "single" sets the Jacobi block widths of the two stages where svd_opts
   leaves them at 0; "batched" sets the persistent grid of svd_batched (W
   workgroups per compute unit, 1..16; default 2).  json = NULL clears the
   table.  Returns 0, -2 on malformed JSON, -3 on an invalid entry (the
   table is then unchanged).  The text is copied; thread-safe. */
int svd_set_tuning(const char *json);

/* The table's entries for size n (0 where the table has none).  Returns 1
   if any entry applies, else 0.  Any output pointer may be NULL. */
int svd_tuning_lookup(int n, int *b_low, int *b_work, int *wg_per_cu);

/* Fill *o with the defaults above; mixed = 1 selects pivot_precision 32,
   mixed = 0 selects 64. */
void svd_default_opts(svd_opts *o, int mixed);

/* Bytes of device workspace svd_plain / svd_mixed need for an m x n problem
   with options o (NULL = defaults).  Returns 0 for invalid sizes. */
size_t svd_workspace_size(int m, int n, const svd_opts *o);

/* Byte offset in the workspace of the copy of Y that diagnostics = 2 leaves
   (the switch study of Section 6); 0 when o->diagnostics != 2 or the sizes
   are invalid. */
size_t svd_diag_y_offset(int m, int n, const svd_opts *o);

/*
 * svd_plain: Algorithm 2 (preconditioned one-sided Jacobi) in FP64:
 *   A = Q0 R1 if m > n (Algorithm 4, first lines), A1 P = Q1 R with FP64
 *   Businger-Golub pivots, R = L Q2, FP64 Jacobi sweeps on X = L with V_X = I,
 *   U = Q0 Q1 U_X, V = P Q2^T V_X.
 * Arguments:
 *   1 m, 2 n        sizes, m >= n >= 0
 *   3 A, 4 lda      input, lda >= max(1, m); not modified
 *   5 S             output, n singular values, descending, >= 0
 *   6 U, 7 ldu      output m x n (ignored when want_u = 0; may be NULL then)
 *   8 V, 9 ldv      output n x n (ignored when want_v = 0; may be NULL then)
 *   10 work, 11 work_bytes  device scratch, >= svd_workspace_size(m, n, o)
 *   12 o            options (NULL = svd_default_opts(.., 0))
 *   13 info         HOST pointer, filled before return (may be NULL); with
 *                   o->capture = 1 a DEVICE pointer written on the stream
 *   14 stream       hipStream_t
 */
int svd_plain(int m, int n, const double *A, int lda, double *S,
              double *U, int ldu, double *V, int ldv,
              void *work, size_t work_bytes, const svd_opts *o,
              svd_info *info, void *stream);

/*
 * svd_mixed: Algorithm 4 with Algorithm 5 pivots.  Same arguments as
 * svd_plain (NULL options = svd_default_opts(.., 1)).  Section 4 (Proposition
 * 1) makes the result as accurate as svd_plain's whatever the FP32 stage
 * delivers; the FP32 stage changes only the number of FP64 sweeps.
 */
int svd_mixed(int m, int n, const double *A, int lda, double *S,
              double *U, int ldu, double *V, int ldv,
              void *work, size_t work_bytes, const svd_opts *o,
              svd_info *info, void *stream);

/* Per-matrix result of svd_batched, written on the device. */
typedef struct {
    int status;
    int branch_taken;
    int sweeps_low;
    int sweeps_work;
} svd_batch_info;

/*
 * Ragged batch, packed layout: matrix j is m_j x n_j (16 <= ... ; any
 * 1 <= n_j <= m_j <= 256 is accepted), stored column-major with ld = m_j at
 *   A_base + offA[j],  offA[j] = sum_{i<j} m_i n_i   (same offsets for U)
 *   S_base + offS[j],  offS[j] = sum_{i<j} n_i
 *   V_base + offV[j],  offV[j] = sum_{i<j} n_i^2       (ld = n_j)
 * svd_batched_plan_create (host only) validates the sizes, orders the work
 * longest-first, picks per-size kernel parameters and reports the workspace
 * size.  svd_batched enqueues one persistent kernel that runs the whole mixed
 * path for every matrix (U and V are always formed).  info: device array of
 * `batch` svd_batch_info.  The plan is immutable after creation and may be
 * shared between streams.
 * Returns -k for a bad argument k, as above.
 */
int svd_batched_plan_create(int batch, const int *h_m, const int *h_n,
                            const svd_opts *o, void **plan, size_t *work_bytes);
int svd_batched(void *plan, const double *A_base, double *S_base,
                double *U_base, double *V_base, void *work, size_t work_bytes,
                svd_batch_info *info, void *stream);
void svd_batched_plan_destroy(void *plan);

/*
 * svd_backward: the SVD adjoint for a strided batch of equal shapes (not in
 * the paper; the standard result for distinct singular values):
 *   gA = U [ (F o (J - J^T)) S + diag(gS) + S (F o (K - K^T)) ] V^T
 *        + (I - U U^T) gU S^-1 V^T,
 *   J = U^T gU, K = V^T gV, F_ij = d / (d^2 + eta^2), d = S_j^2 - S_i^2,
 *   eta = eps_deg * S_1^2, F_ii = 0.
 * U (m x n, ld m) at U + b*sU, S at S + b*sS, V (n x n, ld n) at V + b*sV,
 * gU / gV with the strides of U / V, gS with the stride of S, gA (m x n,
 * ld m) at gA + b*sA.  Any of gU, gS, gV may be NULL (zero).  eps_deg <= 0
 * selects 1e-12.  work >= svd_backward_workspace_size(batch, m, n) bytes.
 * Requires m >= n >= 1; if m > n and some S_i == 0 the S^-1 term is undefined
 * (those columns are left at zero contribution).
 */
size_t svd_backward_workspace_size(int batch, int m, int n);
int svd_backward(int batch, int m, int n,
                 const double *U, long long sU, const double *S, long long sS,
                 const double *V, long long sV,
                 const double *gU, const double *gS, const double *gV,
                 double *gA, long long sA, double eps_deg,
                 void *work, size_t work_bytes, void *stream);

/*
 * svd_backward_noalloc: svd_backward for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  It computes exactly what svd_backward computes, with the
 * same kernel, but takes no workspace: its scratch is a fixed array of
 * SVD_BACKWARD_NOALLOC_SCRATCH_BYTES in device memory inside the library
 * (one per GPU, held from the library's first use on that GPU until the
 * process ends).  Arguments 1-15 and `stream` as for svd_backward; call it
 * with the stream's device current.
 * Returns 0; -k for an invalid argument k as svd_backward; SVD_ERR_SCRATCH_LIMIT
 * (nothing launched) when svd_backward_workspace_size(batch, m, n) exceeds the
 * array; SVD_ERR_HIP on a runtime failure (svd_last_error() says which).
 * The call allocates nothing (no hipMalloc, no hipFree, no allocating library
 * routine) and is stream-ordered.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (different streams, or host threads
 * without ordering) race and give undefined results; calls ordered on one
 * stream are safe.  The kernel writes every scratch word before reading it,
 * so the previous call's contents do not matter.
 */
#define SVD_BACKWARD_NOALLOC_SCRATCH_BYTES (64u << 20)
int svd_backward_noalloc(int batch, int m, int n,
                         const double *U, long long sU, const double *S, long long sS,
                         const double *V, long long sV,
                         const double *gU, const double *gS, const double *gV,
                         double *gA, long long sA, double eps_deg, void *stream);

/*
 * Mixed-precision symmetric eigensolver (Section 8, Algorithm 6):
 *   A = X diag(W) X^T for a symmetric n x n A (both triangles are read as
 *   given; symmetry is not checked).
 *   1-3. the low-precision decomposition, its orthogonalisation and the FP64
 *      one-sided Jacobi refinement without V: the mixed-precision SVD of A
 *      (svd_mixed with want_v = 0), A = U Sigma V^T;
 *   4. blocks of U^T A U over runs of sigma with relative gap <= tol_cluster
 *      (sigma and -sigma may both be eigenvalues);
 *   5. blocks of two or more diagonalised by FP64 two-sided Jacobi (at most
 *      64 columns each), a block of one takes the sign of u_i^T A u_i;
 *   6. W ascending, X's columns with it; sign rule of svd_opts.sign_normalize.
 * Options: those of svd_mixed (want_u, want_v and kernel_timing are set
 * internally), sign_normalize for X, and tol_cluster.  NULL =
 * svd_default_opts(.., 1).
 * Arguments:
 *   1 n (0 <= n <= 8192), 2 A, 3 lda >= max(1, n)   device, not modified
 *   4 W        device output, n eigenvalues ascending
 *   5 X, 6 ldx device output n x n, ldx >= max(1, n), eigenvectors in columns
 *   7 work, 8 work_bytes   device scratch, >= eig_workspace_size(n, o)
 *   9 o        options (host)
 *   10 info    HOST pointer, filled before return (may be NULL)
 *   11 stream  hipStream_t
 * Returns 0, or -k for an invalid argument k (-9: an option out of range).
 * The numerical outcome is info->status: SVD_OK, SVD_WARN_NOCONV,
 * SVD_ERR_NONFINITE, SVD_WARN_RANK_DEFICIENT (a zero singular value: the
 * matching columns of X are zero) or EIG_ERR_CLUSTER.  The call reads
 * results back and synchronises the stream before it returns.
 */
typedef struct {
    int status;
    int sweeps_low;        /* FP32 sweeps of the SVD                     */
    int sweeps_work;       /* FP64 sweeps of the SVD                     */
    int n_clusters;        /* blocks of two or more diagonalised         */
    int max_cluster;       /* largest block                              */
    float stage_ms[4];     /* SVD of A, A U and signs, blocks, sort and
                              output                                     */
} eig_info;

size_t eig_workspace_size(int n, const svd_opts *o);
int eig_mixed(int n, const double *A, int lda, double *W, double *X, int ldx,
              void *work, size_t work_bytes, const svd_opts *o, eig_info *info,
              void *stream);

/* Human-readable name of a status or return code. */
const char *svd_status_string(int code);

/* Description of the HIP failure behind the last SVD_ERR_HIP return of a
   call made on this thread ("" if none). */
const char *svd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MPJSVD_H */
