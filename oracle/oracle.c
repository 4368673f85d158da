/*
 * oracle.c -- plain FP64 reference for the batched regularised contact solve,
 * its implicit-function-theorem VJP and the unrolled-trace VJP.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two meet only through the
 * seeded input generator.  Everything here is plain loops in double precision,
 * one instance at a time (OpenMP only distributes whole instances).
 *
 * Problem (paper Sec. III-A, reduced objective eq. 5, with pyramidal rows so
 * that the regulariser is s(u) = 1/2 sum_i D_i min(u_i, 0)^2):
 *
 *   L(a) = 1/2 (a - a0)^T M (a - a0) + 1/2 sum_i D_i min(r_i, 0)^2,
 *   r    = J a - aref,   A = 1[r < 0],   w = D o A o r.
 *
 *   stationarity residual (eq. 6):   F(a) = M (a - a0) + J^T w
 *   Newton matrix (eq. 9):           H    = M + J^T diag(D o A) J
 *   Newton step + line search (eq. 10): p = -H^{-1} F, a <- a + alpha p,
 *       alpha the exact minimiser of phi(alpha) = L(a + alpha p).
 *   IFT adjoint (eq. 17):  H^T lambda = abar,  theta_bar = -F_theta^T lambda.
 *
 * Linear systems are solved with Householder QR (the dense QR the paper uses
 * for the transposed adjoint solve), never with Cholesky.
 *
 * Stopping rule (reading of "tolerance-converged" with a max-iteration cap,
 * Sec. III-C): iterate a_k is converged when
 *   ||F(a_k)||_2 <= tol * tr(M)          (gradient scaled by mean inertia * n)
 * or, for k >= 1, the step that produced it was negligible and did not change
 * the active set,
 *   ||a_k - a_{k-1}||_inf <= tol * (1 + ||a_k||_inf)  and  A(a_k) = A(a_{k-1}).
 * At most max_iter steps are taken; the returned active set and residual are
 * those of the returned iterate.
 *
 * A second forward solver, preconditioned nonlinear conjugate gradients with
 * the same exact line search (oracle_forward_cg), reaches the same minimiser
 * by another path (Sec. III-B names Newton and nonlinear CG as the two
 * solvers; eqs. 11-14: the derivative does not depend on which).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ST_CONVERGED 1
#define ST_MAXITER 2
#define ST_NONFINITE 4
#define ST_NOTSPD 8
#define ST_LSFAIL 16

/* ------------------------------------------------------------------ */
/* small dense helpers (row-major)                                      */
/* ------------------------------------------------------------------ */

static double dot(int n, const double *x, const double *y) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* y = A x, A is rows x cols */
static void matvec(int rows, int cols, const double *A, const double *x, double *y) {
    for (int i = 0; i < rows; ++i) y[i] = dot(cols, A + (size_t)i * cols, x);
}

/* y = A^T x, A is rows x cols */
static void matvec_t(int rows, int cols, const double *A, const double *x, double *y) {
    for (int j = 0; j < cols; ++j) y[j] = 0.0;
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) y[j] += A[(size_t)i * cols + j] * x[i];
}

static int all_finite(size_t len, const double *x) {
    for (size_t i = 0; i < len; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* Householder QR solve of A x = b (A n x n, row-major, not modified).
 * Returns 0 on success, -1 if R has a zero pivot. */
static int qr_solve(int n, const double *A, const double *b, double *x) {
    double *R = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    memcpy(R, A, sizeof(double) * (size_t)n * n);
    memcpy(y, b, sizeof(double) * (size_t)n);
    for (int k = 0; k < n; ++k) {
        /* reflector for column k, rows k..n-1 */
        double norm = 0.0;
        for (int i = k; i < n; ++i) norm += R[i * n + k] * R[i * n + k];
        norm = sqrt(norm);
        if (norm == 0.0) continue;
        double alpha = R[k * n + k] > 0 ? -norm : norm;
        for (int i = 0; i < n; ++i) v[i] = 0.0;
        v[k] = R[k * n + k] - alpha;
        for (int i = k + 1; i < n; ++i) v[i] = R[i * n + k];
        double vv = 0.0;
        for (int i = k; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        /* apply I - 2 v v^T / (v^T v) to R (columns k..n-1) and to y */
        for (int j = k; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < n; ++i) s += v[i] * R[i * n + j];
            s = 2.0 * s / vv;
            for (int i = k; i < n; ++i) R[i * n + j] -= s * v[i];
        }
        double s = 0.0;
        for (int i = k; i < n; ++i) s += v[i] * y[i];
        s = 2.0 * s / vv;
        for (int i = k; i < n; ++i) y[i] -= s * v[i];
    }
    /* back substitution R x = Q^T b */
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int j = i + 1; j < n; ++j) s -= R[i * n + j] * x[j];
        if (R[i * n + i] == 0.0) { rc = -1; x[i] = NAN; continue; }
        x[i] = s / R[i * n + i];
    }
    free(R); free(y); free(v);
    return rc;
}

/* Plain Cholesky attempt, used only to classify M as SPD or not. */
static int is_spd(int n, const double *M) {
    double *L = (double *)calloc((size_t)n * n, sizeof(double));
    int ok = 1;
    for (int j = 0; j < n && ok; ++j) {
        double s = M[j * n + j];
        for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) { ok = 0; break; }
        L[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = M[i * n + j];
            for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / L[j * n + j];
        }
    }
    free(L);
    return ok;
}

/* ------------------------------------------------------------------ */
/* the method's pieces                                                  */
/* ------------------------------------------------------------------ */

/* r = J a - aref, A = 1[r < 0], F = M (a - a0) + J^T (D o A o r)   (eq. 6) */
static void eval_residual(int n, int m, const double *M, const double *J, const double *a0,
                          const double *aref, const double *D, const double *a,
                          double *r, unsigned char *A, double *F) {
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int j = 0; j < n; ++j) d[j] = a[j] - a0[j];
    matvec(n, n, M, d, F);
    for (int i = 0; i < m; ++i) {
        r[i] = dot(n, J + (size_t)i * n, a) - aref[i];
        A[i] = r[i] < 0.0;
        if (A[i]) {
            double w = D[i] * r[i];
            for (int j = 0; j < n; ++j) F[j] += J[(size_t)i * n + j] * w;
        }
    }
    free(d);
}

/* H = M + J^T diag(D o A) J   (eq. 9) */
static void assemble_H(int n, int m, const double *M, const double *J, const double *D,
                       const unsigned char *A, double *H) {
    memcpy(H, M, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < m; ++i) {
        if (!A[i]) continue;
        const double *Ji = J + (size_t)i * n;
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) H[j * n + k] += D[i] * Ji[j] * Ji[k];
    }
}

typedef struct { double t; int i; } bp_t;

static int bp_cmp(const void *x, const void *y) {
    double a = ((const bp_t *)x)->t, b = ((const bp_t *)y)->t;
    return (a > b) - (a < b);
}

/* Exact line search along p from a (eq. 10 with the exact minimiser of
 * phi(alpha) = L(a + alpha p)).
 *
 * phi'(alpha) = alpha p^T M p + p^T M (a - a0) + sum_i D_i q_i min(r_i + alpha q_i, 0),
 * q = J p, is continuous, piecewise linear and strictly increasing.  Its
 * breakpoints t_i = -r_i / q_i (t_i > 0) are sorted and the pieces scanned
 * from alpha = 0+; the first piece that contains its own root -b/c (closed
 * endpoints) gives alpha.  On return Ap holds the active rows of that piece.
 */
static double exact_line_search(int n, int m, const double *M, const double *J,
                                const double *a0, const double *D, const double *a,
                                const double *p, const double *r, double *q,
                                unsigned char *Ap, double *c_out) {
    double *Mp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    bp_t *bps = (bp_t *)malloc(sizeof(bp_t) * (size_t)(m > 0 ? m : 1));
    for (int j = 0; j < n; ++j) d[j] = a[j] - a0[j];
    matvec(n, n, M, p, Mp);
    double c = dot(n, p, Mp);            /* p^T M p */
    double b = 0.0;                      /* p^T M (a - a0) */
    {
        double *Md = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        matvec(n, n, M, d, Md);
        b = dot(n, p, Md);
        free(Md);
    }
    int nb = 0;
    for (int i = 0; i < m; ++i) {
        q[i] = dot(n, J + (size_t)i * n, p);
        /* piece at alpha = 0+ */
        Ap[i] = (r[i] < 0.0) || (r[i] == 0.0 && q[i] < 0.0);
        if (Ap[i]) { c += D[i] * q[i] * q[i]; b += D[i] * q[i] * r[i]; }
        if (q[i] != 0.0) {
            double t = -r[i] / q[i];
            if (t > 0.0) { bps[nb].t = t; bps[nb].i = i; ++nb; }
        }
    }
    qsort(bps, (size_t)nb, sizeof(bp_t), bp_cmp);
    double alpha = -b / c;
    int k = 0;
    while (k < nb) {
        double t = bps[k].t;
        alpha = -b / c;
        if (alpha <= t) break;           /* root lies in the current piece */
        /* cross every breakpoint equal to t: those rows change activity */
        while (k < nb && bps[k].t == t) {
            int i = bps[k].i;
            double s = Ap[i] ? -1.0 : 1.0;
            Ap[i] = !Ap[i];
            c += s * D[i] * q[i] * q[i];
            b += s * D[i] * q[i] * r[i];
            ++k;
        }
        alpha = -b / c;
    }
    if (c_out) *c_out = c;
    free(Mp); free(d); free(bps);
    return alpha;
}

static double inf_norm(int n, const double *x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s = fmax(s, fabs(x[i]));
    return s;
}

/* step_inf: ||a_k - a_{k-1}||_inf of the step that produced a, or < 0 at k = 0;
 * same_set: A(a_k) equals A(a_{k-1}) */
static int converged(int n, const double *M, const double *F, double step_inf, int same_set,
                     const double *a, double tol) {
    double trM = 0.0;
    for (int j = 0; j < n; ++j) trM += M[j * n + j];
    double g = sqrt(dot(n, F, F));
    if (g <= tol * trM) return 1;
    if (step_inf >= 0.0 && same_set && step_inf <= tol * (1.0 + inf_norm(n, a))) return 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* one instance                                                         */
/* ------------------------------------------------------------------ */

/* Forward solve.  a_init may be NULL (start at a0).  Outputs: a (n),
 * active (m, A at the returned iterate), *iters (steps taken), *status.
 * Optional trace (may be NULL): alphas[max_iter], trA[max_iter*m] (A_k),
 * trAp[max_iter*m] (line-search piece A'_k). */
int oracle_forward(int n, int m, const double *M, const double *J, const double *a0,
                   const double *aref, const double *D, const double *a_init,
                   int max_iter, double tol,
                   double *a, unsigned char *active, int *iters, int *status,
                   double *alphas, unsigned char *trA, unsigned char *trAp) {
    size_t nn = (size_t)n * n, mn = (size_t)m * n;
    *iters = 0;
    if (!all_finite(nn, M) || !all_finite(mn, J) || !all_finite(n, a0) ||
        !all_finite(m, aref) || !all_finite(m, D) || (a_init && !all_finite(n, a_init))) {
        for (int j = 0; j < n; ++j) a[j] = NAN;
        for (int i = 0; i < m; ++i) active[i] = 0;
        *status = ST_NONFINITE;
        return 0;
    }
    if (!is_spd(n, M)) {
        for (int j = 0; j < n; ++j) a[j] = NAN;
        for (int i = 0; i < m; ++i) active[i] = 0;
        *status = ST_NOTSPD;
        return 0;
    }
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1;
    double *r = (double *)malloc(sizeof(double) * mm);
    double *q = (double *)malloc(sizeof(double) * mm);
    double *F = (double *)malloc(sizeof(double) * n1);
    double *negF = (double *)malloc(sizeof(double) * n1);
    double *p = (double *)malloc(sizeof(double) * n1);
    double *H = (double *)malloc(sizeof(double) * (size_t)n1 * n1);
    unsigned char *Ap = (unsigned char *)malloc(mm);
    for (int j = 0; j < n; ++j) a[j] = a_init ? a_init[j] : a0[j];
    int st = ST_MAXITER;
    double step_inf = -1.0;
    unsigned char *Aprev = (unsigned char *)malloc(mm);
    for (int k = 0;; ++k) {
        if (k > 0) memcpy(Aprev, active, m);
        eval_residual(n, m, M, J, a0, aref, D, a, r, active, F);
        int same = k > 0 && (m == 0 || memcmp(Aprev, active, m) == 0);
        if (converged(n, M, F, step_inf, same, a, tol)) { st = ST_CONVERGED; break; }
        if (k == max_iter) { st = ST_MAXITER; break; }
        assemble_H(n, m, M, J, D, active, H);
        for (int j = 0; j < n; ++j) negF[j] = -F[j];
        qr_solve(n, H, negF, p);
        double alpha = exact_line_search(n, m, M, J, a0, D, a, p, r, q, Ap, NULL);
        if (alphas) alphas[k] = alpha;
        if (trA) memcpy(trA + (size_t)k * m, active, m);
        if (trAp) memcpy(trAp + (size_t)k * m, Ap, m);
        step_inf = 0.0;
        for (int j = 0; j < n; ++j) {
            a[j] += alpha * p[j];
            step_inf = fmax(step_inf, fabs(alpha * p[j]));
        }
        *iters = k + 1;
    }
    *status = st;
    free(r); free(q); free(F); free(negF); free(p); free(H); free(Ap); free(Aprev);
    return 0;
}

/* Forward solve by preconditioned nonlinear conjugate gradients (a second
 * solver for the same minimiser; Sec. III-B: any update a - P F with
 * nonsingular P shares the root and its derivative, eqs. 11-14):
 *   z_k = M^{-1} F_k (M preconditions),
 *   p_k = -z_k + beta_k p_{k-1},  beta_k = max(0, F_k . (z_k - z_{k-1}) / (F_{k-1} . z_{k-1}))
 *   (Polak-Ribiere, restarted (beta = 0) at k = 0, when the active set changed,
 *   and whenever p_k is not a descent direction),
 *   a_{k+1} = a_k + alpha_k p_k with the exact line search of the Newton solver.
 * Converged when ||F|| <= tol tr(M) (the Newton rule's gradient test), or when
 *   sqrt(F . M^{-1} F) <= tol sqrt(tr(M)) (1 + ||a||_inf).
 * The second test bounds the distance to the minimiser: L is M-strongly convex
 * (its curvature is H >= M everywhere), so ||a - a*||_M <= sqrt(F . M^{-1} F).
 * The Newton rule's small-step test is not used: a short CG step says little
 * about the distance to the root.  Outputs as oracle_forward. */
int oracle_forward_cg(int n, int m, const double *M, const double *J, const double *a0,
                      const double *aref, const double *D, int max_iter, double tol,
                      double *a, unsigned char *active, int *iters, int *status) {
    size_t nn = (size_t)n * n, mn = (size_t)m * n;
    *iters = 0;
    if (!all_finite(nn, M) || !all_finite(mn, J) || !all_finite(n, a0) ||
        !all_finite(m, aref) || !all_finite(m, D)) {
        for (int j = 0; j < n; ++j) a[j] = NAN;
        for (int i = 0; i < m; ++i) active[i] = 0;
        *status = ST_NONFINITE;
        return 0;
    }
    if (!is_spd(n, M)) {
        for (int j = 0; j < n; ++j) a[j] = NAN;
        for (int i = 0; i < m; ++i) active[i] = 0;
        *status = ST_NOTSPD;
        return 0;
    }
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1;
    double *r = (double *)malloc(sizeof(double) * mm);
    double *q = (double *)malloc(sizeof(double) * mm);
    double *F = (double *)malloc(sizeof(double) * n1);
    double *z = (double *)malloc(sizeof(double) * n1);
    double *zprev = (double *)malloc(sizeof(double) * n1);
    double *p = (double *)calloc(n1, sizeof(double));
    unsigned char *Ap = (unsigned char *)malloc(mm);
    unsigned char *Aprev = (unsigned char *)malloc(mm);
    for (int j = 0; j < n; ++j) a[j] = a0[j];
    int st = ST_MAXITER;
    double fz_prev = 0.0, trM = 0.0;
    for (int j = 0; j < n; ++j) trM += M[j * n + j];
    for (int k = 0;; ++k) {
        if (k > 0) memcpy(Aprev, active, m);
        eval_residual(n, m, M, J, a0, aref, D, a, r, active, F);
        int same = k > 0 && (m == 0 || memcmp(Aprev, active, m) == 0);
        qr_solve(n, M, F, z);
        double fz = dot(n, F, z), beta = 0.0;
        if (sqrt(dot(n, F, F)) <= tol * trM ||
            sqrt(fmax(fz, 0.0)) <= tol * sqrt(trM) * (1.0 + inf_norm(n, a))) {
            st = ST_CONVERGED;
            break;
        }
        if (k == max_iter) { st = ST_MAXITER; break; }
        if (k > 0 && same && fz_prev > 0.0) {
            double num = 0.0;
            for (int j = 0; j < n; ++j) num += F[j] * (z[j] - zprev[j]);
            beta = fmax(0.0, num / fz_prev);
        }
        for (int j = 0; j < n; ++j) p[j] = -z[j] + beta * p[j];
        if (dot(n, F, p) >= 0.0)
            for (int j = 0; j < n; ++j) p[j] = -z[j];
        double alpha = exact_line_search(n, m, M, J, a0, D, a, p, r, q, Ap, NULL);
        for (int j = 0; j < n; ++j) a[j] += alpha * p[j];
        memcpy(zprev, z, sizeof(double) * n);
        fz_prev = fz;
        *iters = k + 1;
    }
    *status = st;
    free(r); free(q); free(F); free(z); free(zprev); free(p); free(Ap); free(Aprev);
    return 0;
}

void oracle_forward_cg_batch(int B, const int32_t *nv, const int32_t *nrows,
                             const int64_t *off_nn, const int64_t *off_mn, const int64_t *off_n,
                             const int64_t *off_m, const double *M, const double *J,
                             const double *a0, const double *aref, const double *D,
                             int max_iter, double tol, double *a, unsigned char *active,
                             int32_t *iters, int32_t *status, int threads);

/* IFT VJP at the returned solution (eq. 17, pyramidal rows):
 *   H(A*)^T lambda = abar,  sigma = J lambda,
 *   a0bar = M^T lambda,  arefbar = D o A* o sigma,  Dbar = -A* o r* o sigma,
 *   Jbar = -(w* lambda^T + arefbar a*^T),  Mbar = -lambda (a* - a0)^T.
 * active may be NULL (then A* = 1[r(a) < 0]).  Every output may be NULL.
 * lambda_out (n) may be NULL. */
int oracle_ift_vjp(int n, int m, const double *M, const double *J, const double *a0,
                   const double *aref, const double *D, const double *a,
                   const unsigned char *active, const double *abar,
                   double *a0bar, double *arefbar, double *Jbar, double *Dbar, double *Mbar,
                   double *lambda_out) {
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1;
    double *r = (double *)malloc(sizeof(double) * mm);
    double *sig = (double *)malloc(sizeof(double) * mm);
    double *H = (double *)malloc(sizeof(double) * (size_t)n1 * n1);
    double *Ht = (double *)malloc(sizeof(double) * (size_t)n1 * n1);
    double *lam = (double *)malloc(sizeof(double) * n1);
    unsigned char *A = (unsigned char *)calloc(mm, 1);
    for (int i = 0; i < m; ++i) {
        r[i] = dot(n, J + (size_t)i * n, a) - aref[i];
        A[i] = active ? active[i] : (r[i] < 0.0);
    }
    assemble_H(n, m, M, J, D, A, H);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) Ht[j * n + k] = H[k * n + j];
    int rc = qr_solve(n, Ht, abar, lam);
    for (int i = 0; i < m; ++i) sig[i] = dot(n, J + (size_t)i * n, lam);
    if (a0bar) matvec_t(n, n, M, lam, a0bar);
    for (int i = 0; i < m; ++i) {
        double w = A[i] ? D[i] * r[i] : 0.0;
        double ar = A[i] ? D[i] * sig[i] : 0.0;
        if (arefbar) arefbar[i] = ar;
        if (Dbar) Dbar[i] = A[i] ? -r[i] * sig[i] : 0.0;
        if (Jbar)
            for (int j = 0; j < n; ++j) Jbar[(size_t)i * n + j] = -(w * lam[j] + ar * a[j]);
    }
    if (Mbar)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) Mbar[j * n + k] = -lam[j] * (a[k] - a0[k]);
    if (lambda_out) memcpy(lambda_out, lam, sizeof(double) * (size_t)n);
    free(r); free(sig); free(H); free(Ht); free(lam); free(A);
    return rc;
}

/* IFT Jacobian-vector products (Sec. III-C, eq. 15, forward mode): for each of
 * k tangent directions (da0_j, daref_j) of the inputs a0 and aref, the
 * directional derivative of the solution,
 *   da_j = -F_a^{-1} F_theta (da0_j, daref_j) = H^{-1} (M da0_j + J^T (D o A* o daref_j)),
 * since F = M (a - a0) + J^T (D o A o (J a - aref)) gives F_a0 = -M and
 * F_aref = -J^T diag(D o A).  H = M + J^T diag(D o A*) J is solved by QR for
 * every direction.  da0 (k x n) and daref (k x m), direction-major, may be
 * NULL (zero); da is k x n. */
int oracle_ift_jvp(int n, int m, const double *M, const double *J, const double *D,
                   const unsigned char *active, int k, const double *da0, const double *daref,
                   double *da) {
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1;
    double *H = (double *)malloc(sizeof(double) * (size_t)n1 * n1);
    double *rhs = (double *)malloc(sizeof(double) * n1);
    double *t = (double *)malloc(sizeof(double) * mm);
    assemble_H(n, m, M, J, D, active, H);
    int rc = 0;
    for (int d = 0; d < k; ++d) {
        for (int j = 0; j < n; ++j) rhs[j] = 0.0;
        if (da0) matvec(n, n, M, da0 + (size_t)d * n, rhs);
        if (daref) {
            for (int i = 0; i < m; ++i) t[i] = active[i] ? D[i] * daref[(size_t)d * m + i] : 0.0;
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < n; ++j) rhs[j] += J[(size_t)i * n + j] * t[i];
        }
        rc |= qr_solve(n, H, rhs, da + (size_t)d * n);
    }
    free(H); free(rhs); free(t);
    return rc;
}

/* Unrolled VJP: the gradient of abar . a_K through the executed K-step trace.
 * Steps after the stopping rule fires are the identity (not recorded).  The
 * line-search step alpha = -b/c is differentiated on its accepted piece A'_k
 * with A_k and A'_k held fixed (reverse-mode AD of the recorded trace). */
int oracle_unrolled_vjp(int n, int m, const double *M, const double *J, const double *a0,
                        const double *aref, const double *D, const double *abar,
                        int K, double tol, double *a_out,
                        double *a0bar, double *arefbar, double *Jbar, double *Dbar,
                        double *Mbar, int *iters, int *status) {
    size_t nn = (size_t)n * n, mn = (size_t)m * n;
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1, K1 = K > 0 ? K : 1;
    /* zero every gradient: the sweep accumulates */
    if (a0bar) memset(a0bar, 0, sizeof(double) * n);
    if (arefbar) memset(arefbar, 0, sizeof(double) * m);
    if (Jbar) memset(Jbar, 0, sizeof(double) * mn);
    if (Dbar) memset(Dbar, 0, sizeof(double) * m);
    if (Mbar) memset(Mbar, 0, sizeof(double) * nn);
    *iters = 0;
    if (!all_finite(nn, M) || !all_finite(mn, J) || !all_finite(n, a0) ||
        !all_finite(m, aref) || !all_finite(m, D) || !all_finite(n, abar)) {
        for (int j = 0; j < n; ++j) a_out[j] = NAN;
        *status = ST_NONFINITE;
        return 0;
    }
    if (!is_spd(n, M)) {
        for (int j = 0; j < n; ++j) a_out[j] = NAN;
        *status = ST_NOTSPD;
        return 0;
    }
    /* tape */
    double *tA = (double *)malloc(sizeof(double) * (size_t)K1 * n1);   /* a_k */
    double *tP = (double *)malloc(sizeof(double) * (size_t)K1 * n1);   /* p_k */
    double *tR = (double *)malloc(sizeof(double) * (size_t)K1 * mm);   /* r_k */
    double *tQ = (double *)malloc(sizeof(double) * (size_t)K1 * mm);   /* q_k */
    double *tH = (double *)malloc(sizeof(double) * (size_t)K1 * n1 * n1);
    unsigned char *tAk = (unsigned char *)malloc((size_t)K1 * mm);
    unsigned char *tAp = (unsigned char *)malloc((size_t)K1 * mm);
    double *tAlpha = (double *)malloc(sizeof(double) * K1);
    double *tC = (double *)malloc(sizeof(double) * K1);
    double *a = (double *)calloc(n1, sizeof(double));
    double *F = (double *)malloc(sizeof(double) * n1);
    double *negF = (double *)malloc(sizeof(double) * n1);
    double *p = (double *)malloc(sizeof(double) * n1);
    double *H = (double *)malloc(sizeof(double) * (size_t)n1 * n1);
    double *r = (double *)malloc(sizeof(double) * mm);
    unsigned char *Ak = (unsigned char *)malloc(mm);
    for (int j = 0; j < n; ++j) a[j] = a0[j];
    int steps = 0, st = ST_MAXITER;
    double step_inf = -1.0;
    unsigned char *Aprev = (unsigned char *)malloc(mm);
    for (int k = 0; k < K; ++k) {
        if (k > 0) memcpy(Aprev, Ak, m);
        eval_residual(n, m, M, J, a0, aref, D, a, r, Ak, F);
        int same = k > 0 && (m == 0 || memcmp(Aprev, Ak, m) == 0);
        if (converged(n, M, F, step_inf, same, a, tol)) { st = ST_CONVERGED; break; }
        assemble_H(n, m, M, J, D, Ak, H);
        for (int j = 0; j < n; ++j) negF[j] = -F[j];
        qr_solve(n, H, negF, p);
        memcpy(tA + (size_t)k * n, a, sizeof(double) * n);
        memcpy(tP + (size_t)k * n, p, sizeof(double) * n);
        memcpy(tR + (size_t)k * m, r, sizeof(double) * m);
        memcpy(tH + (size_t)k * nn, H, sizeof(double) * nn);
        memcpy(tAk + (size_t)k * m, Ak, m);
        double c;
        double alpha = exact_line_search(n, m, M, J, a0, D, a, p, r, tQ + (size_t)k * m,
                                         tAp + (size_t)k * m, &c);
        tAlpha[k] = alpha;
        tC[k] = c;
        step_inf = 0.0;
        for (int j = 0; j < n; ++j) {
            a[j] += alpha * p[j];
            step_inf = fmax(step_inf, fabs(alpha * p[j]));
        }
        steps = k + 1;
    }
    if (st != ST_CONVERGED) {
        /* the K-th iterate is returned; classify it like the forward does */
        if (K > 0) memcpy(Aprev, Ak, m);
        eval_residual(n, m, M, J, a0, aref, D, a, r, Ak, F);
        int same = K > 0 && (m == 0 || memcmp(Aprev, Ak, m) == 0);
        st = converged(n, M, F, step_inf, same, a, tol) ? ST_CONVERGED : ST_MAXITER;
    }
    free(Aprev);
    memcpy(a_out, a, sizeof(double) * n);
    *iters = steps;
    *status = st;

    /* reverse sweep over the recorded steps */
    double *ab = (double *)malloc(sizeof(double) * n1);      /* adjoint of a_{k+1} then a_k */
    double *akb = (double *)malloc(sizeof(double) * n1);
    double *pb = (double *)malloc(sizeof(double) * n1);
    double *d = (double *)malloc(sizeof(double) * n1);
    double *Mp = (double *)malloc(sizeof(double) * n1);
    double *MTp = (double *)malloc(sizeof(double) * n1);
    double *Md = (double *)malloc(sizeof(double) * n1);
    double *u = (double *)malloc(sizeof(double) * n1);
    double *gb = (double *)malloc(sizeof(double) * n1);
    double *tmp = (double *)malloc(sizeof(double) * n1);
    double *Ht = (double *)malloc(sizeof(double) * (size_t)n1 * n1);
    double *qb = (double *)malloc(sizeof(double) * mm);
    double *rb = (double *)malloc(sizeof(double) * mm);
    double *Ju = (double *)malloc(sizeof(double) * mm);
    double *t = (double *)malloc(sizeof(double) * mm);
    /* private accumulators so a NULL output still lets the sweep run */
    double *g_a0 = (double *)calloc(n1, sizeof(double));
    double *g_aref = (double *)calloc(mm, sizeof(double));
    double *g_J = (double *)calloc(mn > 0 ? mn : 1, sizeof(double));
    double *g_D = (double *)calloc(mm, sizeof(double));
    double *g_M = (double *)calloc((size_t)n1 * n1, sizeof(double));
    memcpy(ab, abar, sizeof(double) * n);
    for (int k = steps - 1; k >= 0; --k) {
        const double *ak = tA + (size_t)k * n, *pk = tP + (size_t)k * n;
        const double *rk = tR + (size_t)k * m, *qk = tQ + (size_t)k * m;
        const double *Hk = tH + (size_t)k * nn;
        const unsigned char *Ak_ = tAk + (size_t)k * m, *Apk = tAp + (size_t)k * m;
        double alpha = tAlpha[k], c = tC[k];
        for (int j = 0; j < n; ++j) d[j] = ak[j] - a0[j];
        /* a_{k+1} = a_k + alpha p */
        double alphab = dot(n, ab, pk);
        for (int j = 0; j < n; ++j) { pb[j] = alpha * ab[j]; akb[j] = ab[j]; }
        /* alpha = -b / c */
        double bb = -alphab / c;
        double cb = -alphab * alpha / c;
        matvec(n, n, M, pk, Mp);
        matvec_t(n, n, M, pk, MTp);
        matvec(n, n, M, d, Md);
        /* c = p^T M p + sum_{A'} D q^2 */
        for (int j = 0; j < n; ++j) pb[j] += cb * (Mp[j] + MTp[j]);
        for (int j = 0; j < n; ++j)
            for (int l = 0; l < n; ++l) g_M[j * n + l] += cb * pk[j] * pk[l];
        for (int i = 0; i < m; ++i) { qb[i] = 0.0; rb[i] = 0.0; }
        for (int i = 0; i < m; ++i) {
            if (!Apk[i]) continue;
            g_D[i] += cb * qk[i] * qk[i];
            qb[i] += 2.0 * cb * D[i] * qk[i];
        }
        /* b = p^T M (a_k - a0) + sum_{A'} D q r */
        for (int j = 0; j < n; ++j) pb[j] += bb * Md[j];
        for (int j = 0; j < n; ++j) { akb[j] += bb * MTp[j]; g_a0[j] -= bb * MTp[j]; }
        for (int j = 0; j < n; ++j)
            for (int l = 0; l < n; ++l) g_M[j * n + l] += bb * pk[j] * d[l];
        for (int i = 0; i < m; ++i) {
            if (!Apk[i]) continue;
            g_D[i] += bb * qk[i] * rk[i];
            qb[i] += bb * D[i] * rk[i];
            rb[i] += bb * D[i] * qk[i];
        }
        /* q = J p */
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) {
                pb[j] += J[(size_t)i * n + j] * qb[i];
                g_J[(size_t)i * n + j] += qb[i] * pk[j];
            }
        /* p = -H^{-1} g  ->  u = H^{-T} pbar, gbar = -u, Hbar = -u p^T */
        for (int j = 0; j < n; ++j)
            for (int l = 0; l < n; ++l) Ht[j * n + l] = Hk[l * n + j];
        qr_solve(n, Ht, pb, u);
        for (int j = 0; j < n; ++j) gb[j] = -u[j];
        /* H = M + J^T diag(D o A_k) J */
        for (int j = 0; j < n; ++j)
            for (int l = 0; l < n; ++l) g_M[j * n + l] -= u[j] * pk[l];
        for (int i = 0; i < m; ++i) {
            Ju[i] = dot(n, J + (size_t)i * n, u);
            if (!Ak_[i]) continue;
            for (int j = 0; j < n; ++j)
                g_J[(size_t)i * n + j] -= D[i] * Ju[i] * pk[j] + D[i] * qk[i] * u[j];
            g_D[i] -= Ju[i] * qk[i];
        }
        /* g = M (a_k - a0) + J^T (D o A_k o r_k) */
        matvec_t(n, n, M, gb, tmp);
        for (int j = 0; j < n; ++j) { akb[j] += tmp[j]; g_a0[j] -= tmp[j]; }
        for (int j = 0; j < n; ++j)
            for (int l = 0; l < n; ++l) g_M[j * n + l] += gb[j] * d[l];
        for (int i = 0; i < m; ++i) {
            t[i] = dot(n, J + (size_t)i * n, gb);
            if (!Ak_[i]) continue;
            double w = D[i] * rk[i];
            for (int j = 0; j < n; ++j) g_J[(size_t)i * n + j] += w * gb[j];
            rb[i] += D[i] * t[i];
            g_D[i] += rk[i] * t[i];
        }
        /* r = J a_k - aref */
        matvec_t(m, n, J, rb, tmp);
        for (int j = 0; j < n; ++j) akb[j] += tmp[j];
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < n; ++j) g_J[(size_t)i * n + j] += rb[i] * ak[j];
            g_aref[i] -= rb[i];
        }
        memcpy(ab, akb, sizeof(double) * n);
    }
    /* the first iterate is a0 itself */
    for (int j = 0; j < n; ++j) g_a0[j] += ab[j];
    if (a0bar) memcpy(a0bar, g_a0, sizeof(double) * n);
    if (arefbar) memcpy(arefbar, g_aref, sizeof(double) * m);
    if (Jbar) memcpy(Jbar, g_J, sizeof(double) * mn);
    if (Dbar) memcpy(Dbar, g_D, sizeof(double) * m);
    if (Mbar) memcpy(Mbar, g_M, sizeof(double) * nn);

    free(tA); free(tP); free(tR); free(tQ); free(tH); free(tAk); free(tAp); free(tAlpha);
    free(tC); free(a); free(F); free(negF); free(p); free(H); free(r); free(Ak);
    free(ab); free(akb); free(pb); free(d); free(Mp); free(MTp); free(Md); free(u); free(gb);
    free(tmp); free(Ht); free(qb); free(rb); free(Ju); free(t);
    free(g_a0); free(g_aref); free(g_J); free(g_D); free(g_M);
    return 0;
}

/* Line search alone (for its own tests): returns alpha; Ap (m) and q (m) out. */
double oracle_line_search(int n, int m, const double *M, const double *J, const double *a0,
                          const double *aref, const double *D, const double *a,
                          const double *p, double *q, unsigned char *Ap) {
    double *r = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    for (int i = 0; i < m; ++i) r[i] = dot(n, J + (size_t)i * n, a) - aref[i];
    double alpha = exact_line_search(n, m, M, J, a0, D, a, p, r, q, Ap, NULL);
    free(r);
    return alpha;
}

/* ------------------------------------------------------------------ */
/* packed batches: instance i uses off_*[i]; OpenMP over instances      */
/* ------------------------------------------------------------------ */

/* ------------------------------------------------------------------ */
/* elliptic (round) Coulomb cone                                        */
/* ------------------------------------------------------------------ */
/*
 * Contact c owns rows 3c (normal), 3c+1, 3c+2 (tangential) of J and aref; its
 * regularisation weights are R^{-1} = diag(dn, dt, dt) (D = 1/R per row, the
 * two tangential rows sharing one weight) and its friction coefficient mu
 * (Sec. III-A, eqs. 2, 3 and 5).  The dual of K = {l_N >= 0, |l_T| <= mu l_N}
 * is K* = {z_N >= mu |z_T|}, and
 *   s_c(u) = min over z in K* of 1/2 (u - z)^T R^{-1} (u - z).
 * In the scaled coordinates x = (sqrt(dn) u_N, sqrt(dt) u_T) the weighted
 * projection is the Euclidean projection onto the second-order cone
 * {x_N >= mh |x_T|}, mh = mu sqrt(dn / dt).  With nn = x_N, t = |x_T|:
 *   zone 0 (inside):  nn >= mh t            s = 0;
 *   zone 2 (polar):   mh nn + t <= 0        s = 1/2 (nn^2 + t^2)  (all three rows act);
 *   zone 1 (between): s = 1/2 (mh t - nn)^2 / (1 + mh^2)  (distance to the cone's edge).
 * ell_block returns s, w = ds/du (3) and G = d^2 s / du^2 (3 x 3, row-major).
 */
static int ell_block(const double *u, double dn, double dt, double mu, double *w, double *G,
                     double *sval) {
    const double sn = sqrt(dn), st = sqrt(dt), mh = mu * sn / st;
    const double nn = sn * u[0], x1 = st * u[1], x2 = st * u[2];
    const double t = sqrt(x1 * x1 + x2 * x2);
    double gh[3] = {0, 0, 0}, Gh[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, sv = 0.0;
    int zone;
    if (nn >= mh * t) {
        zone = 0;
    } else if (mh * nn + t <= 0.0) {
        zone = 2;
        sv = 0.5 * (nn * nn + t * t);
        gh[0] = nn; gh[1] = x1; gh[2] = x2;
        Gh[0] = Gh[4] = Gh[8] = 1.0;
    } else {
        zone = 1;   /* t > 0 here */
        const double k = 1.0 + mh * mh, h = mh * t - nn;
        const double e[3] = {-1.0, mh * x1 / t, mh * x2 / t};
        sv = 0.5 * h * h / k;
        for (int i = 0; i < 3; ++i) gh[i] = h / k * e[i];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Gh[3 * i + j] = e[i] * e[j] / k;
        /* curvature of t: (I - tau tau^T) / t on the tangential block */
        const double c = h * mh / (k * t), t1 = x1 / t, t2 = x2 / t;
        Gh[4] += c * (1.0 - t1 * t1);
        Gh[5] += c * (-t1 * t2);
        Gh[7] += c * (-t1 * t2);
        Gh[8] += c * (1.0 - t2 * t2);
    }
    const double S[3] = {sn, st, st};
    for (int i = 0; i < 3; ++i) {
        w[i] = S[i] * gh[i];
        for (int j = 0; j < 3; ++j) G[3 * i + j] = S[i] * Gh[3 * i + j] * S[j];
    }
    if (sval) *sval = sv;
    return zone;
}

/* F = M (a - a0) + J^T w (eq. 6 with the round cone), the zones and the
 * contact blocks (w: m values, G: 9 per contact) at a; returns L(a). */
static double ell_eval(int n, int nc, const double *M, const double *J, const double *a0,
                       const double *aref, const double *dn, const double *dt, const double *mu,
                       const double *a, double *u, double *w, double *G, unsigned char *zone,
                       double *F) {
    const int m = 3 * nc;
    double *d = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int j = 0; j < n; ++j) d[j] = a[j] - a0[j];
    matvec(m, n, J, a, u);
    for (int i = 0; i < m; ++i) u[i] -= aref[i];
    double Lv = 0.0;
    for (int c = 0; c < nc; ++c) {
        double sv;
        zone[c] = (unsigned char)ell_block(u + 3 * c, dn[c], dt[c], mu[c], w + 3 * c, G + 9 * c, &sv);
        Lv += sv;
    }
    matvec(n, n, M, d, F);
    Lv += 0.5 * dot(n, d, F);
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += J[(size_t)i * n + j] * w[i];
        F[j] += s;
    }
    free(d);
    return Lv;
}

/* H = M + sum_c J_c^T G_c J_c (eq. 9 with 3 x 3 blocks) */
static void ell_assemble_H(int n, int nc, const double *M, const double *J, const double *G,
                           double *H) {
    memcpy(H, M, sizeof(double) * (size_t)n * n);
    for (int c = 0; c < nc; ++c)
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                const double g = G[9 * c + 3 * r + q];
                if (g == 0.0) continue;
                const double *Jr = J + (size_t)(3 * c + r) * n, *Jq = J + (size_t)(3 * c + q) * n;
                for (int j = 0; j < n; ++j)
                    for (int l = 0; l < n; ++l) H[(size_t)j * n + l] += Jr[j] * g * Jq[l];
            }
}

/* Exact line search along p: phi(alpha) = L(a + alpha p) is convex and C^1
 * (piecewise C^2), so its minimiser is the root of the increasing phi'.  From
 * alpha = 1: Newton steps on phi' while no upper end of the bracket is known;
 * then Newton steps that stay inside the bracket and at least halve the step
 * before last, else a secant step on the bracket's ends (bisection instead
 * when the bracket is not at most half as wide as two evaluations before, or
 * the secant point falls outside); until
 * phi' = 0, |phi'| is at its rounding level (1e-13 of the sum of its terms'
 * magnitudes), the bracket is within rounding of its upper end, or a step no
 * longer moves alpha.  *fail is set when 100 evaluations do not get there. */
static double ell_line_search(int n, int nc, const double *M, const double *J, const double *a0,
                              const double *aref, const double *dn, const double *dt,
                              const double *mu, const double *a, const double *p, int *fail) {
    const int m = 3 * nc;
    int mm = m > 0 ? m : 1;
    double *u0 = (double *)malloc(sizeof(double) * mm), *q = (double *)malloc(sizeof(double) * mm);
    double *Mp = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *d = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    matvec(m, n, J, a, u0);
    for (int i = 0; i < m; ++i) u0[i] -= aref[i];
    matvec(m, n, J, p, q);
    matvec(n, n, M, p, Mp);
    for (int j = 0; j < n; ++j) d[j] = a[j] - a0[j];
    const double c0 = dot(n, p, Mp), b0 = dot(n, Mp, d);
    /* phi'(0) from the blocks at u0 */
    double glo = b0;
    for (int c = 0; c < nc; ++c) {
        double w[3], G[9];
        ell_block(u0 + 3 * c, dn[c], dt[c], mu[c], w, G, NULL);
        for (int r = 0; r < 3; ++r) glo += w[r] * q[3 * c + r];
    }
    double lo = 0.0, hi = -1.0, ghi = 0.0, al = 1.0, best = 1.0, dxold = INFINITY, dx = INFINITY;
    double wid1 = INFINITY, wid2 = INFINITY;
    *fail = 1;
    for (int it = 0; it < 100; ++it) {
        double g = c0 * al + b0, h = c0, sabs = fabs(c0 * al) + fabs(b0);
        for (int c = 0; c < nc; ++c) {
            double uu[3], w[3], G[9];
            for (int r = 0; r < 3; ++r) uu[r] = u0[3 * c + r] + al * q[3 * c + r];
            ell_block(uu, dn[c], dt[c], mu[c], w, G, NULL);
            double wq = 0.0;
            for (int r = 0; r < 3; ++r) {
                wq += w[r] * q[3 * c + r];
                for (int s2 = 0; s2 < 3; ++s2) h += q[3 * c + r] * G[3 * r + s2] * q[3 * c + s2];
            }
            g += wq;
            sabs += fabs(wq);
        }
        best = al;
        if (g == 0.0) { *fail = 0; break; }
        if (g < 0.0) { lo = al; glo = g; } else { hi = al; ghi = g; }
        if (fabs(g) <= 1e-13 * sabs) { *fail = 0; break; }
        double nx = al - g / h;
        if (hi < 0.0) {
            if (!(nx > al)) nx = 2.0 * al;
        } else {
            const double wid = hi - lo;
            if (wid <= 4e-16 * hi) { *fail = 0; break; }
            const int slow = wid > 0.5 * wid2;
            wid2 = wid1;
            wid1 = wid;
            if (!(nx > lo && nx < hi && fabs(nx - al) < 0.5 * fabs(dxold))) {
                nx = lo - glo * (hi - lo) / (ghi - glo);
                if (slow || !(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
            }
        }
        dxold = dx;
        dx = nx - al;
        if (nx == al) { *fail = 0; break; }
        al = nx;
    }
    free(u0); free(q); free(Mp); free(d);
    return best;
}

/* Forward solve with the round cone: Newton steps p = -H^{-1} F with the
 * exact line search; the stopping rule of oracle_forward with the zone
 * pattern in place of the active set.  Outputs a (n), zone (nc), iters,
 * status. */
int oracle_forward_ell(int n, int nc, const double *M, const double *J, const double *a0,
                       const double *aref, const double *dn, const double *dt, const double *mu,
                       int max_iter, double tol, double *a, unsigned char *zone, int *iters,
                       int *status) {
    const int m = 3 * nc;
    *iters = 0;
    if (!all_finite((size_t)n * n, M) || !all_finite((size_t)m * n, J) || !all_finite(n, a0) ||
        !all_finite(m, aref) || !all_finite(nc, dn) || !all_finite(nc, dt) || !all_finite(nc, mu)) {
        for (int j = 0; j < n; ++j) a[j] = NAN;
        for (int c = 0; c < nc; ++c) zone[c] = 0;
        *status = ST_NONFINITE;
        return 0;
    }
    if (!is_spd(n, M)) {
        for (int j = 0; j < n; ++j) a[j] = NAN;
        for (int c = 0; c < nc; ++c) zone[c] = 0;
        *status = ST_NOTSPD;
        return 0;
    }
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1, nc1 = nc > 0 ? nc : 1;
    double *u = (double *)malloc(sizeof(double) * mm), *w = (double *)malloc(sizeof(double) * mm);
    double *G = (double *)malloc(sizeof(double) * 9 * nc1), *F = (double *)malloc(sizeof(double) * n1);
    double *H = (double *)malloc(sizeof(double) * n1 * n1), *p = (double *)malloc(sizeof(double) * n1);
    double *mf = (double *)malloc(sizeof(double) * n1);
    unsigned char *zprev = (unsigned char *)malloc(nc1);
    for (int j = 0; j < n; ++j) a[j] = a0[j];
    double step_inf = -1.0;
    int st = ST_MAXITER, lsfail = 0;
    for (int k = 0;; ++k) {
        if (k > 0) memcpy(zprev, zone, nc);
        ell_eval(n, nc, M, J, a0, aref, dn, dt, mu, a, u, w, G, zone, F);
        const int same = k > 0 && (nc == 0 || memcmp(zprev, zone, nc) == 0);
        if (converged(n, M, F, step_inf, same, a, tol)) { st = ST_CONVERGED; break; }
        if (k == max_iter) { st = ST_MAXITER; break; }
        ell_assemble_H(n, nc, M, J, G, H);
        for (int j = 0; j < n; ++j) mf[j] = -F[j];
        qr_solve(n, H, mf, p);
        int fl = 0;
        const double al = ell_line_search(n, nc, M, J, a0, aref, dn, dt, mu, a, p, &fl);
        lsfail |= fl;
        step_inf = 0.0;
        for (int j = 0; j < n; ++j) {
            a[j] += al * p[j];
            step_inf = fmax(step_inf, fabs(al * p[j]));
        }
        *iters = k + 1;
    }
    *status = st | (lsfail ? ST_LSFAIL : 0);
    free(u); free(w); free(G); free(F); free(H); free(p); free(mf); free(zprev);
    return 0;
}

/* IFT VJP with the round cone (eq. 17): H lambda = abar with H = M + sum_c
 * J_c^T G_c J_c at a; sigma = J lambda;
 *   a0bar = M^T lambda,  arefbar_c = G_c sigma_c,  Jbar = -(w lambda^T + arefbar a^T),
 *   Mbar = -lambda (a - a0)^T,  theta_bar = -sigma_c . dw_c/dtheta for theta in
 *   (dn_c, dt_c, mu_c), dw/dtheta at fixed u (w = S g(S u, mh), S = diag(sqrt dn,
 *   sqrt dt, sqrt dt), mh = mu sqrt(dn / dt)).  Any output may be NULL. */
int oracle_ift_vjp_ell(int n, int nc, const double *M, const double *J, const double *a0,
                       const double *aref, const double *dn, const double *dt, const double *mu,
                       const double *a, const double *abar, double *a0bar, double *arefbar,
                       double *Jbar, double *dnbar, double *dtbar, double *mubar, double *Mbar) {
    const int m = 3 * nc;
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1, nc1 = nc > 0 ? nc : 1;
    double *u = (double *)malloc(sizeof(double) * mm), *w = (double *)malloc(sizeof(double) * mm);
    double *G = (double *)malloc(sizeof(double) * 9 * nc1), *F = (double *)malloc(sizeof(double) * n1);
    double *H = (double *)malloc(sizeof(double) * n1 * n1), *lam = (double *)malloc(sizeof(double) * n1);
    double *sg = (double *)malloc(sizeof(double) * mm), *ab = (double *)malloc(sizeof(double) * mm);
    unsigned char *zone = (unsigned char *)malloc(nc1);
    ell_eval(n, nc, M, J, a0, aref, dn, dt, mu, a, u, w, G, zone, F);
    ell_assemble_H(n, nc, M, J, G, H);
    qr_solve(n, H, abar, lam);   /* H is symmetric */
    matvec(m, n, J, lam, sg);
    for (int c = 0; c < nc; ++c)
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += G[9 * c + 3 * r + q] * sg[3 * c + q];
            ab[3 * c + r] = s;
        }
    if (a0bar) matvec_t(n, n, M, lam, a0bar);
    if (arefbar) memcpy(arefbar, ab, sizeof(double) * m);
    if (Jbar)
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) Jbar[(size_t)i * n + j] = -(w[i] * lam[j] + ab[i] * a[j]);
    if (Mbar)
        for (int j = 0; j < n; ++j)
            for (int l = 0; l < n; ++l) Mbar[(size_t)j * n + l] = -lam[j] * (a[l] - a0[l]);
    for (int c = 0; c < nc; ++c) {
        /* dw/dtheta at fixed u, theta = (dn, dt, mu) */
        const double sn = sqrt(dn[c]), st = sqrt(dt[c]), mh = mu[c] * sn / st;
        const double *uc = u + 3 * c;
        const double x[3] = {sn * uc[0], st * uc[1], st * uc[2]};
        double gh[3], Gh[9], S[3] = {sn, st, st};
        /* g and its Jacobian in scaled coordinates: from the unscaled block */
        for (int i = 0; i < 3; ++i) {
            gh[i] = w[3 * c + i] / S[i];
            for (int j = 0; j < 3; ++j) Gh[3 * i + j] = G[9 * c + 3 * i + j] / (S[i] * S[j]);
        }
        double dgm[3] = {0, 0, 0};   /* dg/dmh */
        if (zone[c] == 1) {
            const double t = sqrt(x[1] * x[1] + x[2] * x[2]), k = 1.0 + mh * mh, h = mh * t - x[0];
            const double e[3] = {-1.0, mh * x[1] / t, mh * x[2] / t};
            const double f = t / k - 2.0 * mh * h / (k * k);
            dgm[0] = f * e[0];
            dgm[1] = f * e[1] + h / k * x[1] / t;
            dgm[2] = f * e[2] + h / k * x[2] / t;
        }
        /* theta = dn: dS = diag(1/(2 sn), 0, 0), dmh = mu / (2 sn st)
         * theta = dt: dS = diag(0, 1/(2 st), 1/(2 st)), dmh = -mu sn / (2 st^3)
         * theta = mu: dS = 0, dmh = sn / st */
        double dS[3][3] = {{0.5 / sn, 0, 0}, {0, 0.5 / st, 0.5 / st}, {0, 0, 0}};
        double dmh[3] = {mu[c] / (2.0 * sn * st), -mu[c] * sn / (2.0 * st * st * st), sn / st};
        double out[3];
        for (int th = 0; th < 3; ++th) {
            double dx[3], dw[3];
            for (int i = 0; i < 3; ++i) dx[i] = dS[th][i] * uc[i];
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += Gh[3 * i + j] * dx[j];
                dw[i] = dS[th][i] * gh[i] + S[i] * (s + dgm[i] * dmh[th]);
            }
            out[th] = -(sg[3 * c] * dw[0] + sg[3 * c + 1] * dw[1] + sg[3 * c + 2] * dw[2]);
        }
        if (dnbar) dnbar[c] = out[0];
        if (dtbar) dtbar[c] = out[1];
        if (mubar) mubar[c] = out[2];
    }
    free(u); free(w); free(G); free(F); free(H); free(lam); free(sg); free(ab); free(zone);
    return 0;
}

/* s_c, w_c, G_c and the zone of one contact (for the pins) */
int oracle_ell_block(const double *u, double dn, double dt, double mu, double *w, double *G,
                     double *sval) {
    return ell_block(u, dn, dt, mu, w, G, sval);
}

/* L(a) with the round cone (for the pins) */
double oracle_ell_objective(int n, int nc, const double *M, const double *J, const double *a0,
                            const double *aref, const double *dn, const double *dt,
                            const double *mu, const double *a, double *F) {
    const int m = 3 * nc;
    int mm = m > 0 ? m : 1, nc1 = nc > 0 ? nc : 1;
    double *u = (double *)malloc(sizeof(double) * mm), *w = (double *)malloc(sizeof(double) * mm);
    double *G = (double *)malloc(sizeof(double) * 9 * nc1);
    unsigned char *zone = (unsigned char *)malloc(nc1);
    const double Lv = ell_eval(n, nc, M, J, a0, aref, dn, dt, mu, a, u, w, G, zone, F);
    free(u); free(w); free(G); free(zone);
    return Lv;
}

/* ------------------------------------------------------------------ */
/* mixed regularised rows: one-sided, equality, friction loss           */
/* ------------------------------------------------------------------ */
/*
 * Row i has a kind (Sec. III-A: the frictional block and "other regularised
 * constraint rows"):
 *   0  one-sided (a pyramid edge or a limit):  s_i = 1/2 D_i min(r_i, 0)^2;
 *   1  equality:                               s_i = 1/2 D_i r_i^2;
 *   2  friction loss with bound f_i >= 0 (its force saturates at +-f_i):
 *      s_i = 1/2 D_i r_i^2 for |r_i| <= f_i / D_i, else f_i |r_i| - f_i^2 / (2 D_i).
 * Each s_i is C^1 and piecewise quadratic in r_i.  Zone codes of a row at r:
 * 0 no force, 1 quadratic (w = D r, curvature D), 2 saturated at +f (w = f),
 * 3 saturated at -f (w = -f).
 */
static int row_zone(int kind, double r, double D, double f) {
    if (kind == 0) return r < 0.0 ? 1 : 0;
    if (kind == 1) return 1;
    const double d = f / D;
    if (r > d) return 2;
    if (r < -d) return 3;
    return 1;
}

static double row_w(int zone, double r, double D, double f) {
    return zone == 1 ? D * r : (zone == 2 ? f : (zone == 3 ? -f : 0.0));
}

static double row_s(int zone, double r, double D, double f) {
    if (zone == 1) return 0.5 * D * r * r;
    if (zone == 2 || zone == 3) return f * fabs(r) - 0.5 * f * f / D;
    return 0.0;
}

/* F, zones and L at a; returns L(a) */
static double rows_eval(int n, int m, const double *M, const double *J, const double *a0,
                        const double *aref, const double *D, const unsigned char *kind,
                        const double *fl, const double *a, double *r, unsigned char *zone,
                        double *w, double *F) {
    double *d = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int j = 0; j < n; ++j) d[j] = a[j] - a0[j];
    matvec(m, n, J, a, r);
    double Lv = 0.0;
    for (int i = 0; i < m; ++i) {
        r[i] -= aref[i];
        zone[i] = (unsigned char)row_zone(kind[i], r[i], D[i], fl[i]);
        w[i] = row_w(zone[i], r[i], D[i], fl[i]);
        Lv += row_s(zone[i], r[i], D[i], fl[i]);
    }
    matvec(n, n, M, d, F);
    Lv += 0.5 * dot(n, d, F);
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += J[(size_t)i * n + j] * w[i];
        F[j] += s;
    }
    free(d);
    return Lv;
}

static int dbl_cmp(const void *x, const void *y) {
    const double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

/* Exact line search: phi'(t) = c0 t + b0 + sum_i q_i w_i(r_i + t q_i) is
 * continuous, increasing and piecewise linear.  Its breakpoints (t > 0 where a
 * row changes zone) are sorted; on each piece in turn the zones at the
 * piece's midpoint give the line phi' = c t + b, and the first piece whose
 * line has its root before the piece's end holds the minimiser. */
static double rows_line_search(int n, int m, const double *M, const double *J, const double *a0,
                               const double *D, const unsigned char *kind, const double *fl,
                               const double *a, const double *p, const double *r) {
    int mm = m > 0 ? m : 1;
    double *q = (double *)malloc(sizeof(double) * mm), *bp = (double *)malloc(sizeof(double) * 2 * mm);
    double *Mp = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *d = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    matvec(m, n, J, p, q);
    matvec(n, n, M, p, Mp);
    for (int j = 0; j < n; ++j) d[j] = a[j] - a0[j];
    const double c0 = dot(n, p, Mp), b0 = dot(n, Mp, d);
    int nb = 0;
    for (int i = 0; i < m; ++i) {
        if (q[i] == 0.0) continue;
        if (kind[i] == 0) {
            const double t = -r[i] / q[i];
            if (t > 0.0) bp[nb++] = t;
        } else if (kind[i] == 2) {
            const double dd = fl[i] / D[i];
            const double t1 = (dd - r[i]) / q[i], t2 = (-dd - r[i]) / q[i];
            if (t1 > 0.0) bp[nb++] = t1;
            if (t2 > 0.0) bp[nb++] = t2;
        }
    }
    qsort(bp, (size_t)nb, sizeof(double), dbl_cmp);
    double lo = 0.0, alpha = 0.0;
    for (int k = 0; k <= nb; ++k) {
        const double hi = k < nb ? bp[k] : INFINITY;
        if (hi <= lo) continue;
        const double mid = k < nb ? 0.5 * (lo + hi) : lo + 1.0 + fabs(lo);
        double c = c0, b = b0;
        for (int i = 0; i < m; ++i) {
            const int z = row_zone(kind[i], r[i] + mid * q[i], D[i], fl[i]);
            if (z == 1) { c += D[i] * q[i] * q[i]; b += D[i] * q[i] * r[i]; }
            else if (z == 2) b += fl[i] * q[i];
            else if (z == 3) b -= fl[i] * q[i];
        }
        alpha = -b / c;
        if (alpha <= hi) break;
        lo = hi;
    }
    free(q); free(bp); free(Mp); free(d);
    return alpha;
}

/* Forward solve with mixed rows: Newton steps with H = M + J^T diag(g) J
 * (g_i = D_i in zone 1, else 0), the exact line search above, and the stopping
 * rule of oracle_forward with the zone pattern in place of the active set.
 * Outputs a, zone (m), iters, status. */
int oracle_forward_rows(int n, int m, const double *M, const double *J, const double *a0,
                        const double *aref, const double *D, const unsigned char *kind,
                        const double *fl, int max_iter, double tol, double *a,
                        unsigned char *zone, int *iters, int *status) {
    *iters = 0;
    if (!all_finite((size_t)n * n, M) || !all_finite((size_t)m * n, J) || !all_finite(n, a0) ||
        !all_finite(m, aref) || !all_finite(m, D) || !all_finite(m, fl)) {
        for (int j = 0; j < n; ++j) a[j] = NAN;
        for (int i = 0; i < m; ++i) zone[i] = 0;
        *status = ST_NONFINITE;
        return 0;
    }
    if (!is_spd(n, M)) {
        for (int j = 0; j < n; ++j) a[j] = NAN;
        for (int i = 0; i < m; ++i) zone[i] = 0;
        *status = ST_NOTSPD;
        return 0;
    }
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1;
    double *r = (double *)malloc(sizeof(double) * mm), *w = (double *)malloc(sizeof(double) * mm);
    double *F = (double *)malloc(sizeof(double) * n1), *H = (double *)malloc(sizeof(double) * n1 * n1);
    double *p = (double *)malloc(sizeof(double) * n1), *mf = (double *)malloc(sizeof(double) * n1);
    double *g = (double *)malloc(sizeof(double) * mm);
    unsigned char *zprev = (unsigned char *)malloc(mm);
    for (int j = 0; j < n; ++j) a[j] = a0[j];
    double step_inf = -1.0;
    int st = ST_MAXITER;
    for (int k = 0;; ++k) {
        if (k > 0) memcpy(zprev, zone, m);
        rows_eval(n, m, M, J, a0, aref, D, kind, fl, a, r, zone, w, F);
        const int same = k > 0 && (m == 0 || memcmp(zprev, zone, m) == 0);
        if (converged(n, M, F, step_inf, same, a, tol)) { st = ST_CONVERGED; break; }
        if (k == max_iter) { st = ST_MAXITER; break; }
        for (int i = 0; i < m; ++i) g[i] = zone[i] == 1 ? D[i] : 0.0;
        assemble_H(n, m, M, J, g, zone, H);
        for (int j = 0; j < n; ++j) mf[j] = -F[j];
        qr_solve(n, H, mf, p);
        const double al = rows_line_search(n, m, M, J, a0, D, kind, fl, a, p, r);
        step_inf = 0.0;
        for (int j = 0; j < n; ++j) {
            a[j] += al * p[j];
            step_inf = fmax(step_inf, fabs(al * p[j]));
        }
        *iters = k + 1;
    }
    *status = st;
    free(r); free(w); free(F); free(H); free(p); free(mf); free(g); free(zprev);
    return 0;
}

/* IFT VJP with mixed rows (eq. 17) at a: H lambda = abar, sigma = J lambda,
 *   a0bar = M^T lambda, arefbar_i = g_i sigma_i, Dbar_i = -r_i sigma_i in zone 1
 *   (0 elsewhere), fbar_i = -sign(r_i) sigma_i in zones 2, 3 (0 elsewhere),
 *   Jbar = -(w lambda^T + arefbar a^T), Mbar = -lambda (a - a0)^T.
 * Any output may be NULL. */
int oracle_ift_vjp_rows(int n, int m, const double *M, const double *J, const double *a0,
                        const double *aref, const double *D, const unsigned char *kind,
                        const double *fl, const double *a, const double *abar, double *a0bar,
                        double *arefbar, double *Jbar, double *Dbar, double *flbar,
                        double *Mbar) {
    int mm = m > 0 ? m : 1, n1 = n > 0 ? n : 1;
    double *r = (double *)malloc(sizeof(double) * mm), *w = (double *)malloc(sizeof(double) * mm);
    double *F = (double *)malloc(sizeof(double) * n1), *H = (double *)malloc(sizeof(double) * n1 * n1);
    double *lam = (double *)malloc(sizeof(double) * n1), *sg = (double *)malloc(sizeof(double) * mm);
    double *g = (double *)malloc(sizeof(double) * mm);
    unsigned char *zone = (unsigned char *)malloc(mm);
    rows_eval(n, m, M, J, a0, aref, D, kind, fl, a, r, zone, w, F);
    for (int i = 0; i < m; ++i) g[i] = zone[i] == 1 ? D[i] : 0.0;
    assemble_H(n, m, M, J, g, zone, H);
    qr_solve(n, H, abar, lam);
    matvec(m, n, J, lam, sg);
    if (a0bar) matvec_t(n, n, M, lam, a0bar);
    for (int i = 0; i < m; ++i) {
        const double ab = g[i] * sg[i];
        if (arefbar) arefbar[i] = ab;
        if (Dbar) Dbar[i] = zone[i] == 1 ? -r[i] * sg[i] : 0.0;
        if (flbar) flbar[i] = zone[i] == 2 ? -sg[i] : (zone[i] == 3 ? sg[i] : 0.0);
        if (Jbar)
            for (int j = 0; j < n; ++j) Jbar[(size_t)i * n + j] = -(w[i] * lam[j] + ab * a[j]);
    }
    if (Mbar)
        for (int j = 0; j < n; ++j)
            for (int l = 0; l < n; ++l) Mbar[(size_t)j * n + l] = -lam[j] * (a[l] - a0[l]);
    free(r); free(w); free(F); free(H); free(lam); free(sg); free(g); free(zone);
    return 0;
}

static void set_threads(int threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_forward_batch(int B, const int32_t *nv, const int32_t *nrows,
                          const int64_t *off_nn, const int64_t *off_mn, const int64_t *off_n,
                          const int64_t *off_m, const double *M, const double *J,
                          const double *a0, const double *aref, const double *D,
                          int max_iter, double tol, double *a, unsigned char *active,
                          int32_t *iters, int32_t *status, int threads) {
    set_threads(threads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < B; ++b) {
        int it = 0, st = 0;
        oracle_forward(nv[b], nrows[b], M + off_nn[b], J + off_mn[b], a0 + off_n[b],
                       aref + off_m[b], D + off_m[b], NULL, max_iter, tol, a + off_n[b],
                       active + off_m[b], &it, &st, NULL, NULL, NULL);
        iters[b] = it;
        status[b] = st;
    }
}

void oracle_forward_cg_batch(int B, const int32_t *nv, const int32_t *nrows,
                             const int64_t *off_nn, const int64_t *off_mn, const int64_t *off_n,
                             const int64_t *off_m, const double *M, const double *J,
                             const double *a0, const double *aref, const double *D,
                             int max_iter, double tol, double *a, unsigned char *active,
                             int32_t *iters, int32_t *status, int threads) {
    set_threads(threads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < B; ++b) {
        int it = 0, st = 0;
        oracle_forward_cg(nv[b], nrows[b], M + off_nn[b], J + off_mn[b], a0 + off_n[b],
                          aref + off_m[b], D + off_m[b], max_iter, tol, a + off_n[b],
                          active + off_m[b], &it, &st);
        iters[b] = it;
        status[b] = st;
    }
}

void oracle_ift_vjp_batch(int B, const int32_t *nv, const int32_t *nrows,
                          const int64_t *off_nn, const int64_t *off_mn, const int64_t *off_n,
                          const int64_t *off_m, const double *M, const double *J,
                          const double *a0, const double *aref, const double *D,
                          const double *a, const unsigned char *active, const double *abar,
                          double *a0bar, double *arefbar, double *Jbar, double *Dbar,
                          double *Mbar, int threads) {
    set_threads(threads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < B; ++b) {
        oracle_ift_vjp(nv[b], nrows[b], M + off_nn[b], J + off_mn[b], a0 + off_n[b],
                       aref + off_m[b], D + off_m[b], a + off_n[b],
                       active ? active + off_m[b] : NULL, abar + off_n[b],
                       a0bar ? a0bar + off_n[b] : NULL, arefbar ? arefbar + off_m[b] : NULL,
                       Jbar ? Jbar + off_mn[b] : NULL, Dbar ? Dbar + off_m[b] : NULL,
                       Mbar ? Mbar + off_nn[b] : NULL, NULL);
    }
}

void oracle_ift_jvp_batch(int B, const int32_t *nv, const int32_t *nrows,
                          const int64_t *off_nn, const int64_t *off_mn, const int64_t *off_n,
                          const int64_t *off_m, const double *M, const double *J,
                          const double *D, const unsigned char *active, int k,
                          const double *da0, const double *daref, double *da, int threads) {
    set_threads(threads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < B; ++b) {
        oracle_ift_jvp(nv[b], nrows[b], M + off_nn[b], J + off_mn[b], D + off_m[b],
                       active + off_m[b], k, da0 ? da0 + (size_t)k * off_n[b] : NULL,
                       daref ? daref + (size_t)k * off_m[b] : NULL, da + (size_t)k * off_n[b]);
    }
}

void oracle_unrolled_vjp_batch(int B, const int32_t *nv, const int32_t *nrows,
                               const int64_t *off_nn, const int64_t *off_mn,
                               const int64_t *off_n, const int64_t *off_m, const double *M,
                               const double *J, const double *a0, const double *aref,
                               const double *D, const double *abar, int K, double tol,
                               double *a, double *a0bar, double *arefbar, double *Jbar,
                               double *Dbar, double *Mbar, int32_t *iters, int32_t *status,
                               int threads) {
    set_threads(threads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < B; ++b) {
        int it = 0, st = 0;
        oracle_unrolled_vjp(nv[b], nrows[b], M + off_nn[b], J + off_mn[b], a0 + off_n[b],
                            aref + off_m[b], D + off_m[b], abar + off_n[b], K, tol,
                            a + off_n[b], a0bar ? a0bar + off_n[b] : NULL,
                            arefbar ? arefbar + off_m[b] : NULL, Jbar ? Jbar + off_mn[b] : NULL,
                            Dbar ? Dbar + off_m[b] : NULL, Mbar ? Mbar + off_nn[b] : NULL,
                            &it, &st);
        iters[b] = it;
        status[b] = st;
    }
}
