/*
 * FP64 CPU oracle for the one-sided Jacobi SVD.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load.  The GPU library never links, includes or calls it, and it
 * shares no code with the GPU library.
 *
 * What it computes is the plain definition of the problem: the SVD
 * A = U diag(S) V^T of an m x n matrix, m >= n, to high relative accuracy,
 * by the preconditioned one-sided Jacobi method of the paper (Section 2:
 * Algorithm 1 for the sweeps, Algorithm 2 for the QR preconditioning, with the
 * tall-matrix reduction of Algorithm 4 / Section 3.1).  The mixed-precision
 * method reaches this same result (Section 4, Proposition 1), so the oracle is
 * plain FP64 throughout.
 *
 * Conventions: column-major storage, IEEE double, no BLAS or LAPACK, every
 * dot product summed sequentially in index order, no FMA contraction (the
 * build uses -ffp-contract=off).  Column norms are plain square roots of sums
 * of squares: entries must stay within about 1e-150 .. 1e150 in magnitude.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IX(i, j, ld) ((size_t)(j) * (size_t)(ld) + (size_t)(i))

enum { ORC_OK = 0, ORC_NOCONV = 1, ORC_RANKDEF = 3, ORC_BADARG = -1 };

void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Progress lines on stderr (phase ends, sweeps) for long timed runs; no
   effect on what is computed. */
static int g_verbose = 0;
void oracle_set_verbose(int v) { g_verbose = v; }
#define ORC_PROGRESS(...)                                                     \
    do {                                                                      \
        if (g_verbose) { fprintf(stderr, "[oracle] " __VA_ARGS__); fflush(stderr); } \
    } while (0)

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static double dot(int len, const double *x, const double *y)
{
    double s = 0.0;
    for (int i = 0; i < len; ++i) s += x[i] * y[i];
    return s;
}

static double nrm2(int len, const double *x) { return sqrt(dot(len, x, x)); }

/*
 * Householder reflector H = I - tau v v^T with v[0] = 1 such that
 * H x = beta e_1 (the elementary reflector of QR, Section 2.2).
 * On return x[0] = beta and x[1..len-1] = v[1..len-1].
 */
void oracle_house(int len, double *x, double *tau)
{
    if (len <= 1) { *tau = 0.0; return; }
    double alpha = x[0];
    double xnorm = nrm2(len - 1, x + 1);
    if (xnorm == 0.0) { *tau = 0.0; return; }
    double beta = -copysign(hypot(alpha, xnorm), alpha);
    *tau = (beta - alpha) / beta;
    double scal = 1.0 / (alpha - beta);
    for (int i = 1; i < len; ++i) x[i] *= scal;
    x[0] = beta;
}

/* Apply H = I - tau v v^T (v[0] = 1 implied, v[1..] in vt) to the len x ncol
   block C from the left. */
static void apply_house_left(int len, const double *vt, double tau,
                             int ncol, double *C, int ldc)
{
    if (tau == 0.0) return;
    for (int j = 0; j < ncol; ++j) {
        double *c = C + IX(0, j, ldc);
        double w = c[0];
        for (int i = 1; i < len; ++i) w += vt[i] * c[i];
        w *= tau;
        c[0] -= w;
        for (int i = 1; i < len; ++i) c[i] -= w * vt[i];
    }
}

/*
 * Unpivoted Householder QR, A = Q R (m x n, m >= n): the tall reduction
 * A = Q0 R1 of Algorithm 4 and the plain QR of Algorithm 5.
 * R overwrites the upper triangle, the reflectors the strict lower part,
 * tau[0..n-1] their scalars.
 */
int oracle_geqr2(int m, int n, double *A, int lda, double *tau)
{
    if (m < 0 || n < 0 || lda < (m > 1 ? m : 1)) return ORC_BADARG;
    int k = m < n ? m : n;
    for (int j = 0; j < k; ++j) {
        double *col = A + IX(j, j, lda);
        oracle_house(m - j, col, &tau[j]);
        double beta = col[0];
        col[0] = 1.0;
        apply_house_left(m - j, col, tau[j], n - j - 1, A + IX(j, j + 1, lda), lda);
        col[0] = beta;
    }
    return ORC_OK;
}

/*
 * Businger-Golub QR with column pivoting, A P = Q R (the rank-revealing QR of
 * Algorithm 2, computed as LAPACK's xGEQP3 would; Section 3.1).  At step k the
 * remaining column whose trailing part A(k:m-1, j) has the largest 2-norm,
 * recomputed from scratch (no downdating), is swapped into position k; ties go
 * to the column with the smallest original index.  jpvt[k] = original index of
 * the column in position k.
 */
int oracle_geqp3(int m, int n, double *A, int lda, int *jpvt, double *tau)
{
    if (m < 0 || n < 0 || lda < (m > 1 ? m : 1)) return ORC_BADARG;
    for (int j = 0; j < n; ++j) jpvt[j] = j;
    int k = m < n ? m : n;
    for (int s = 0; s < k; ++s) {
        int p = s;
        double best = -1.0;
        for (int j = s; j < n; ++j) {
            double nj = nrm2(m - s, A + IX(s, j, lda));
            if (nj > best || (nj == best && jpvt[j] < jpvt[p])) { best = nj; p = j; }
        }
        if (p != s) {
            for (int i = 0; i < m; ++i) {
                double t = A[IX(i, s, lda)];
                A[IX(i, s, lda)] = A[IX(i, p, lda)];
                A[IX(i, p, lda)] = t;
            }
            int t = jpvt[s]; jpvt[s] = jpvt[p]; jpvt[p] = t;
        }
        double *col = A + IX(s, s, lda);
        oracle_house(m - s, col, &tau[s]);
        double beta = col[0];
        col[0] = 1.0;
        apply_house_left(m - s, col, tau[s], n - s - 1, A + IX(s, s + 1, lda), lda);
        col[0] = beta;
    }
    return ORC_OK;
}

/*
 * C <- Q C (trans = 0) or C <- Q^T C (trans = 1), where Q = H_0 H_1 ... H_{k-1}
 * is held as reflectors in the strict lower part of the m x k matrix Qf (as
 * left by oracle_geqr2 / oracle_geqp3).  C is m x ncol.
 */
int oracle_apply_q(int trans, int m, int k, const double *Qf, int ldq,
                   const double *tau, int ncol, double *C, int ldc)
{
    double *v = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    if (!v) return ORC_BADARG;
    for (int s = 0; s < k; ++s) {
        int j = trans ? s : k - 1 - s;
        int len = m - j;
        v[0] = 1.0;
        for (int i = 1; i < len; ++i) v[i] = Qf[IX(j + i, j, ldq)];
        apply_house_left(len, v, tau[j], ncol, C + IX(j, 0, ldc), ldc);
    }
    free(v);
    return ORC_OK;
}

/*
 * The 2x2 Jacobi rotation of Section 2.1 for the Gram entries
 * alpha = x_p^T x_p, beta = x_q^T x_q, gamma = x_p^T x_q (gamma != 0):
 * J = [c s; -s c] with c real, the root with |theta| <= pi/4 (the choice
 * closest to the identity).  [x_p, x_q] J has orthogonal columns in exact
 * arithmetic.  zeta = (beta - alpha) / (2 gamma),
 * t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) with sign(0) = +1.
 */
void oracle_rotation(double alpha, double beta, double gamma, double *c, double *s)
{
    double zeta = (beta - alpha) / (2.0 * gamma);
    double sg = zeta >= 0.0 ? 1.0 : -1.0;
    double t = sg / (fabs(zeta) + hypot(1.0, zeta));
    *c = 1.0 / sqrt(1.0 + t * t);
    *s = t * (*c);
}

/* One pair step of Algorithm 1: test and, if needed, rotate columns p < q of
   X (m rows) and of V (nv rows, may be NULL).  Returns 1 if rotated. */
static int pair_step(int m, double *X, int ldx, int nv, double *V, int ldv,
                     int p, int q, double eps)
{
    double *xp = X + IX(0, p, ldx), *xq = X + IX(0, q, ldx);
    double alpha = dot(m, xp, xp);
    double beta = dot(m, xq, xq);
    double gamma = dot(m, xp, xq);
    if (!(fabs(gamma) > eps * sqrt(alpha) * sqrt(beta))) return 0;
    double c, s;
    oracle_rotation(alpha, beta, gamma, &c, &s);
    for (int i = 0; i < m; ++i) {
        double a = xp[i], b = xq[i];
        xp[i] = c * a - s * b;
        xq[i] = s * a + c * b;
    }
    if (V) {
        double *vp = V + IX(0, p, ldv), *vq = V + IX(0, q, ldv);
        for (int i = 0; i < nv; ++i) {
            double a = vp[i], b = vq[i];
            vp[i] = c * a - s * b;
            vq[i] = s * a + c * b;
        }
    }
    return 1;
}

/* Round-robin (circle method) pairing on nn = n rounded up to even: in round
   r (0 <= r < nn-1) slot 0 pairs r with nn-1 and slot k pairs (r+k) mod (nn-1)
   with (r-k) mod (nn-1).  Every unordered pair appears exactly once per sweep.
   Pairs involving the padding index n (odd n) are reported as (-1, -1). */
void oracle_rr_pair(int n, int r, int k, int *p, int *q)
{
    int nn = n + (n & 1);
    int a, b;
    if (k == 0) { a = r; b = nn - 1; }
    else {
        a = (r + k) % (nn - 1);
        b = ((r - k) % (nn - 1) + (nn - 1)) % (nn - 1);
    }
    if (a > b) { int t = a; a = b; b = t; }
    if (b >= n) { *p = -1; *q = -1; return; }
    *p = a; *q = b;
}

/*
 * Algorithm 1 (one-sided Jacobi, without the final normalisation): sweeps over
 * the column pairs of the m x n matrix X, rotating a pair when
 * |x_q^T x_p| > eps ||x_p|| ||x_q||, until a sweep rotates nothing or maxiter
 * sweeps have run.  Rotations are accumulated into V (nv x n, caller
 * initialised, may be NULL).  order 0 = the row-cyclic order (eq. cyclic);
 * order 1 = round-robin rounds of disjoint pairs, run in parallel with OpenMP.
 * *sweeps receives the number of sweeps executed (the last one rotating
 * nothing when converged).  Returns ORC_OK or ORC_NOCONV.
 */
int oracle_gesvj(int m, int n, double *X, int ldx, int nv, double *V, int ldv,
                 double eps, int maxiter, int order, int *sweeps)
{
    int it = 0, converged = 0;
    while (it < maxiter && !converged) {
        int rotated = 0;
        if (order == 0) {
            for (int p = 0; p < n - 1; ++p)
                for (int q = p + 1; q < n; ++q)
                    rotated |= pair_step(m, X, ldx, nv, V, ldv, p, q, eps);
        } else {
            int nn = n + (n & 1);
            for (int r = 0; r < nn - 1; ++r) {
                int rr = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : rr)
                for (int k = 0; k < nn / 2; ++k) {
                    int p, q;
                    oracle_rr_pair(n, r, k, &p, &q);
                    if (p >= 0) rr |= pair_step(m, X, ldx, nv, V, ldv, p, q, eps);
                }
                rotated |= rr;
            }
        }
        ++it;
        converged = !rotated;
        ORC_PROGRESS("sweep %d done\n", it);
    }
    if (sweeps) *sweeps = it;
    return converged ? ORC_OK : ORC_NOCONV;
}

/*
 * Final step of Algorithm 1: S[i] = ||x_i||, U(:, i) = x_i / S[i], then a stable
 * sort of S descending (equal values keep their order) applied to the columns
 * of U and of V (nv x n, may be NULL).  X is overwritten by U.  A zero column
 * gives S[i] = 0 and a zero U column; the return value counts them.
 */
int oracle_finalize(int m, int n, double *X, int ldx, double *S,
                    int nv, double *V, int ldv)
{
    int zeros = 0;
    for (int i = 0; i < n; ++i) {
        double *x = X + IX(0, i, ldx);
        double s = nrm2(m, x);
        S[i] = s;
        if (s == 0.0) { ++zeros; continue; }
        for (int r = 0; r < m; ++r) x[r] /= s;
    }
    /* stable insertion sort of the permutation by descending S */
    int *ord = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    for (int i = 0; i < n; ++i) ord[i] = i;
    for (int i = 1; i < n; ++i) {
        int v = ord[i], j = i - 1;
        while (j >= 0 && S[ord[j]] < S[v]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = v;
    }
    double *tmpS = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *tmp = (double *)malloc((size_t)(m > nv ? m : nv > 0 ? nv : 1) * (size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int i = 0; i < n; ++i) tmpS[i] = S[ord[i]];
    memcpy(S, tmpS, (size_t)n * sizeof(double));
    for (int i = 0; i < n; ++i) memcpy(tmp + IX(0, i, m), X + IX(0, ord[i], ldx), (size_t)m * sizeof(double));
    for (int i = 0; i < n; ++i) memcpy(X + IX(0, i, ldx), tmp + IX(0, i, m), (size_t)m * sizeof(double));
    if (V) {
        for (int i = 0; i < n; ++i) memcpy(tmp + IX(0, i, nv), V + IX(0, ord[i], ldv), (size_t)nv * sizeof(double));
        for (int i = 0; i < n; ++i) memcpy(V + IX(0, i, ldv), tmp + IX(0, i, nv), (size_t)nv * sizeof(double));
    }
    free(ord); free(tmpS); free(tmp);
    return zeros;
}

/* Sign rule for the singular vectors: for each i let k be the first row index
   of the largest |V(k, i)|; if V(k, i) < 0, negate U(:, i) and V(:, i). */
void oracle_sign_normalize(int m, int n, double *U, int ldu, double *V, int ldv)
{
    for (int i = 0; i < n; ++i) {
        int k = 0;
        double best = -1.0;
        for (int j = 0; j < n; ++j) {
            double a = fabs(V[IX(j, i, ldv)]);
            if (a > best) { best = a; k = j; }
        }
        if (V[IX(k, i, ldv)] < 0.0) {
            for (int j = 0; j < n; ++j) V[IX(j, i, ldv)] = -V[IX(j, i, ldv)];
            for (int j = 0; j < m; ++j) U[IX(j, i, ldu)] = -U[IX(j, i, ldu)];
        }
    }
}

/*
 * The full SVD A = U diag(S) V^T, m >= n.
 *
 * precondition = 1 (Algorithm 2 with the tall reduction of Algorithm 4):
 *   1. if m > n: A = Q0 R1 (oracle_geqr2), A1 = R1; else A1 = A.
 *   2. A1 P = Q1 R (oracle_geqp3).
 *   3. R = L Q2 through the QR of R^T: R^T = Q2' R2, L = R2^T, Q2 = Q2'^T;
 *      X = L.  (The LQ step is always taken.)
 *   4. Algorithm 1 on X with V_X = I.
 *   5. S, U_X sorted (oracle_finalize).
 *   6. U = Q0 Q1 U_X and V = P Q2^T V_X = P Q2' V_X.
 * precondition = 0: Algorithm 1 directly on A (m x n) with V = I.
 * Then the sign rule (oracle_sign_normalize) when sign_norm != 0.
 *
 * eps <= 0 selects sqrt(rows) * 2^-53, rows being the row count of the
 * matrix the sweeps act on.  U is m x n, V is n x n.
 * Returns ORC_OK, ORC_NOCONV, ORC_RANKDEF (a zero singular value) or
 * ORC_BADARG.  sweeps / jpvt_out may be NULL.
 */
int oracle_svd(int m, int n, const double *A, int lda, double *S,
               double *U, int ldu, double *V, int ldv,
               int precondition, int order, double eps, int maxiter,
               int sign_norm, int *sweeps, int *jpvt_out)
{
    if (n < 0 || m < n || lda < (m > 1 ? m : 1) || ldu < (m > 1 ? m : 1) ||
        ldv < (n > 1 ? n : 1))
        return ORC_BADARG;
    if (sweeps) *sweeps = 0;
    if (n == 0) return ORC_OK;
    int status = ORC_OK;

    if (!precondition) {
        double *X = (double *)malloc((size_t)m * n * sizeof(double));
        for (int j = 0; j < n; ++j) memcpy(X + IX(0, j, m), A + IX(0, j, lda), (size_t)m * sizeof(double));
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) V[IX(i, j, ldv)] = (i == j) ? 1.0 : 0.0;
        double e = eps > 0 ? eps : sqrt((double)m) * ldexp(1.0, -53);
        status = oracle_gesvj(m, n, X, m, n, V, ldv, e, maxiter, order, sweeps);
        int z = oracle_finalize(m, n, X, m, S, n, V, ldv);
        for (int j = 0; j < n; ++j) memcpy(U + IX(0, j, ldu), X + IX(0, j, m), (size_t)m * sizeof(double));
        free(X);
        if (status == ORC_OK && z) status = ORC_RANKDEF;
        if (jpvt_out) for (int j = 0; j < n; ++j) jpvt_out[j] = j;
        if (sign_norm) oracle_sign_normalize(m, n, U, ldu, V, ldv);
        return status;
    }

    /* 1. tall reduction */
    double *Qt = NULL, *tau0 = NULL;
    double *A1 = (double *)calloc((size_t)n * n, sizeof(double));
    if (m > n) {
        Qt = (double *)malloc((size_t)m * n * sizeof(double));
        tau0 = (double *)malloc((size_t)n * sizeof(double));
        for (int j = 0; j < n; ++j) memcpy(Qt + IX(0, j, m), A + IX(0, j, lda), (size_t)m * sizeof(double));
        oracle_geqr2(m, n, Qt, m, tau0);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i <= j; ++i) A1[IX(i, j, n)] = Qt[IX(i, j, m)];
    } else {
        for (int j = 0; j < n; ++j) memcpy(A1 + IX(0, j, n), A + IX(0, j, lda), (size_t)n * sizeof(double));
    }
    /* 2. QRCP */
    int *jpvt = (int *)malloc((size_t)n * sizeof(int));
    double *tau1 = (double *)malloc((size_t)n * sizeof(double));
    ORC_PROGRESS("tall reduction done\n");
    oracle_geqp3(n, n, A1, n, jpvt, tau1);
    ORC_PROGRESS("QRCP done\n");
    /* 3. LQ of R via QR of R^T */
    double *Rt = (double *)calloc((size_t)n * n, sizeof(double));
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; ++i) Rt[IX(j, i, n)] = A1[IX(i, j, n)];
    double *tau2 = (double *)malloc((size_t)n * sizeof(double));
    oracle_geqr2(n, n, Rt, n, tau2);
    ORC_PROGRESS("LQ done\n");
    double *X = (double *)calloc((size_t)n * n, sizeof(double));
    for (int j = 0; j < n; ++j)
        for (int i = j; i < n; ++i) X[IX(i, j, n)] = Rt[IX(j, i, n)];
    /* 4. Jacobi with V_X = I */
    double *VX = (double *)calloc((size_t)n * n, sizeof(double));
    for (int j = 0; j < n; ++j) VX[IX(j, j, n)] = 1.0;
    double e = eps > 0 ? eps : sqrt((double)n) * ldexp(1.0, -53);
    status = oracle_gesvj(n, n, X, n, n, VX, n, e, maxiter, order, sweeps);
    /* 5. normalise and sort */
    int z = oracle_finalize(n, n, X, n, S, n, VX, n);
    if (status == ORC_OK && z) status = ORC_RANKDEF;
    /* 6. U = Q0 Q1 U_X */
    oracle_apply_q(0, n, n, A1, n, tau1, n, X, n);
    ORC_PROGRESS("U back-transform done\n");
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) U[IX(i, j, ldu)] = X[IX(i, j, n)];
        for (int i = n; i < m; ++i) U[IX(i, j, ldu)] = 0.0;
    }
    if (m > n) oracle_apply_q(0, m, n, Qt, m, tau0, n, U, ldu);
    /*    V = P Q2' V_X */
    oracle_apply_q(0, n, n, Rt, n, tau2, n, VX, n);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) V[IX(jpvt[k], j, ldv)] = VX[IX(k, j, n)];
    if (jpvt_out) memcpy(jpvt_out, jpvt, (size_t)n * sizeof(int));
    if (sign_norm) oracle_sign_normalize(m, n, U, ldu, V, ldv);

    free(Qt); free(tau0); free(A1); free(jpvt); free(tau1); free(Rt);
    free(tau2); free(X); free(VX);
    return status;
}

/*
 * Symmetric eigendecomposition A = X diag(w) X^T (n x n, A symmetric; only
 * what is stored is used, both triangles are read as given) by the cyclic
 * two-sided Jacobi method: the textbook computation of the spectral
 * decomposition that the mixed-precision eigensolver of Section 8
 * (Algorithm 6) also delivers.
 *
 * Each sweep visits the pairs (p, q), p < q, in row-cyclic order.  A pair is
 * rotated when |a_pq| > eps sqrt(|a_pp| |a_qq|) (and a_pq != 0); the rotation
 * is the 2 x 2 symmetric Schur rotation (the formula of oracle_rotation with
 * alpha = a_pp, beta = a_qq, gamma = a_pq), applied as
 * A <- J^T A J on rows and columns p, q, with a_pp <- a_pp - t a_pq,
 * a_qq <- a_qq + t a_pq and a_pq <- 0; X <- X J accumulates the rotations.
 * The method stops after a sweep without rotations, or after maxiter sweeps.
 * w is then sorted ascending (stable) with X's columns, and, when sign_norm
 * is set, each column of X is negated if its largest-magnitude entry (first
 * on ties) is negative.
 *
 * eps <= 0 selects sqrt(n) 2^-53.  Returns ORC_OK, ORC_NOCONV or ORC_BADARG.
 */
int oracle_syevj(int n, const double *A, int lda, double *w, double *X, int ldx,
                 double eps, int maxiter, int sign_norm, int *sweeps)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || ldx < (n > 1 ? n : 1)) return ORC_BADARG;
    if (sweeps) *sweeps = 0;
    if (n == 0) return ORC_OK;
    double *M = (double *)malloc((size_t)n * n * sizeof(double));
    for (int j = 0; j < n; ++j) memcpy(M + IX(0, j, n), A + IX(0, j, lda), (size_t)n * sizeof(double));
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) X[IX(i, j, ldx)] = (i == j) ? 1.0 : 0.0;
    const double e = eps > 0 ? eps : sqrt((double)n) * ldexp(1.0, -53);
    int status = ORC_NOCONV, sw = 0;
    for (; sw < maxiter; ++sw) {
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double app = M[IX(p, p, n)], aqq = M[IX(q, q, n)], apq = M[IX(p, q, n)];
                if (apq == 0.0 || !(fabs(apq) > e * sqrt(fabs(app) * fabs(aqq)))) continue;
                /* the root t of t^2 + 2 zeta t - 1 = 0 with |t| <= 1 */
                const double zeta = (aqq - app) / (2.0 * apq);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                rotated = 1;
                for (int r = 0; r < n; ++r) {
                    if (r == p || r == q) continue;
                    const double arp = M[IX(r, p, n)], arq = M[IX(r, q, n)];
                    const double np_ = c * arp - s * arq, nq_ = s * arp + c * arq;
                    M[IX(r, p, n)] = np_; M[IX(p, r, n)] = np_;
                    M[IX(r, q, n)] = nq_; M[IX(q, r, n)] = nq_;
                }
                M[IX(p, p, n)] = app - t * apq;
                M[IX(q, q, n)] = aqq + t * apq;
                M[IX(p, q, n)] = 0.0;
                M[IX(q, p, n)] = 0.0;
                for (int r = 0; r < n; ++r) {
                    const double xp = X[IX(r, p, ldx)], xq = X[IX(r, q, ldx)];
                    X[IX(r, p, ldx)] = c * xp - s * xq;
                    X[IX(r, q, ldx)] = s * xp + c * xq;
                }
            }
        }
        if (!rotated) { status = ORC_OK; ++sw; break; }
    }
    if (sweeps) *sweeps = sw;
    for (int i = 0; i < n; ++i) w[i] = M[IX(i, i, n)];
    free(M);
    /* stable ascending sort of w with the columns of X (insertion sort) */
    double *col = (double *)malloc((size_t)n * sizeof(double));
    for (int i = 1; i < n; ++i) {
        const double wi = w[i];
        for (int r = 0; r < n; ++r) col[r] = X[IX(r, i, ldx)];
        int j = i - 1;
        while (j >= 0 && w[j] > wi) {
            w[j + 1] = w[j];
            for (int r = 0; r < n; ++r) X[IX(r, j + 1, ldx)] = X[IX(r, j, ldx)];
            --j;
        }
        w[j + 1] = wi;
        for (int r = 0; r < n; ++r) X[IX(r, j + 1, ldx)] = col[r];
    }
    free(col);
    if (sign_norm) {
        for (int i = 0; i < n; ++i) {
            int k = 0;
            double best = -1.0;
            for (int r = 0; r < n; ++r) {
                const double a = fabs(X[IX(r, i, ldx)]);
                if (a > best) { best = a; k = r; }
            }
            if (X[IX(k, i, ldx)] < 0.0)
                for (int r = 0; r < n; ++r) X[IX(r, i, ldx)] = -X[IX(r, i, ldx)];
        }
    }
    return status;
}
