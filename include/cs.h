/*
 * cs.h -- C ABI of the batched contact-solve library (libcs.so, gfx950).
 *
 * Each instance i of a batch is one regularised contact block with pyramidal
 * friction rows (the reduced problem of Sec. III-A, eq. 5):
 *
 *   a*_i = argmin_a 1/2 (a - a0)^T M (a - a0) + 1/2 sum_r D_r min(r_r, 0)^2,
 *          r = J a - aref,
 *
 * with M (n x n, symmetric positive definite), J (m x n, m = 4 x contacts,
 * rows per contact ordered [J_n + mu J_t1, J_n - mu J_t1, J_n + mu J_t2,
 * J_n - mu J_t2]), a0 (n), aref (m) and D = 1/R (m, D > 0).
 *
 * Conventions for every entry point:
 *  - All arrays are device pointers, row-major, of the batch's dtype (float for
 *    CS_F32, double for CS_F64), except where stated.  The caller allocates and
 *    owns every buffer (including `state` and `tape`); the library never
 *    allocates or frees device memory on a call.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *    stream).  The return code reports argument and launch errors only; the
 *    per-instance `status` words are valid once the stream has synchronised.
 *  - Outputs must not alias inputs.
 *  - Uniform batches: `nv`, `nrows` and every `off_*` pointer are NULL and
 *    instance i occupies elements [i n^2, (i+1) n^2) of M, [i m n, ...) of J,
 *    [i n, ...) of n-vectors and [i m, ...) of m-vectors.
 *  - Packed (uneven) batches: `nv`, `nrows` [B] and the four offset arrays
 *    [B+1] (element offsets, off[B] = total) are device arrays, and the host
 *    fields `nv_max`, `nrows_max`, `total_*` must describe them.
 *
 * Error codes: CS_OK, CS_EINVAL (bad argument: sizes, NULL required pointer,
 * dtype, unsupported shape), CS_ENOSPC (caller buffer too small), CS_EHIP (HIP
 * launch error), CS_EUNSUPPORTED.  cs_strerror() names them.
 */
#ifndef CS_H
#define CS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CS_OK 0
#define CS_EINVAL (-1)
#define CS_ENOSPC (-2)
#define CS_EHIP (-3)
#define CS_EUNSUPPORTED (-4)

#define CS_F32 0
#define CS_F64 1

/* per-instance status bits (status[i]) */
#define CS_ST_CONVERGED 1   /* stopping rule met at the returned iterate */
#define CS_ST_MAXITER 2     /* max_iter steps taken without meeting it */
#define CS_ST_NONFINITE 4   /* an input was NaN/Inf; outputs are NaN */
#define CS_ST_NOTSPD 8      /* M (or a Newton matrix) is not positive definite; outputs NaN */
#define CS_ST_LSFAIL 16     /* the line search hit its safeguard cap (step still taken) */
#define CS_ST_BADDESC 32    /* packed descriptor malformed: 1 <= n <= nv_max, 0 <= m <= nrows_max,
                             * offsets >= 0 and offset + extent <= total_* must hold; the
                             * instance is skipped (no output written; cs_ift_vjp leaves its
                             * outputs untouched).  An order[] entry outside [0, B) is skipped
                             * with no status written. */

/* Kernel families (cs_batch.path), chosen from the batch's (or subset's)
 * largest n and m.  SMALL: 16 lanes per instance with the instance held in
 * registers (FP32 n <= 12, FP64 n <= 6, m <= 64).  CHUNK: one workgroup per
 * instance, rows of J streamed through LDS in 64-row chunks, Newton matrix
 * on the matrix cores in FP32 (n <= 128, m <= 2048).  TEAM: one workgroup per
 * instance, any supported shape.  WAVE (FP32 forward, n <= 31, m <= 1024):
 * one wave per instance with J resident in LDS and the Newton matrix and
 * J^T w from one matrix-core pass per step; its VJP runs on the CHUNK (else
 * TEAM) family.  AUTO takes the first that fits of SMALL, WAVE, CHUNK,
 * TEAM (the unrolled VJP has SMALL and TEAM only).  A forced family that
 * does not fit returns CS_EUNSUPPORTED.  Every family writes the same state layout, so any
 * cs_ift_vjp family can read any cs_forward state. */
#define CS_PATH_AUTO 0
#define CS_PATH_TEAM 1
#define CS_PATH_SMALL 2
#define CS_PATH_CHUNK 3
#define CS_PATH_WAVE 4

/* Largest sizes the library supports per instance. */
#define CS_NV_MAX 128
#define CS_NROWS_MAX 4096

typedef struct cs_batch {
    int32_t B;              /* number of instances (>= 0) */
    int32_t dtype;          /* CS_F32 or CS_F64 */
    int32_t nv_uniform;     /* n when nv == NULL */
    int32_t nrows_uniform;  /* m when nrows == NULL */
    const int32_t *nv;      /* device [B] or NULL */
    const int32_t *nrows;   /* device [B] or NULL */
    const int64_t *off_nn;  /* device [B+1]: offsets into M, Mbar and the state factors */
    const int64_t *off_mn;  /* device [B+1]: offsets into J, Jbar */
    const int64_t *off_n;   /* device [B+1]: offsets into a0, a, abar, a0bar */
    const int64_t *off_m;   /* device [B+1]: offsets into aref, D, arefbar, Dbar */
    const int32_t *order;   /* device [B] processing order (a permutation), or NULL */
    int32_t nv_max;         /* packed: max n over the batch */
    int32_t nrows_max;      /* packed: max m over the batch */
    int64_t total_nn;       /* packed: off_nn[B] */
    int64_t total_mn;       /* packed: off_mn[B] */
    int64_t total_n;        /* packed: off_n[B] */
    int64_t total_m;        /* packed: off_m[B] */
    int32_t path;           /* kernel family: CS_PATH_AUTO, _TEAM, _SMALL, _CHUNK or _WAVE */
    int32_t count;          /* solve only order[0 .. count-1] (0: all B; > 0 needs order).
                             * nv_max / nrows_max may then describe that subset only */
} cs_batch;

typedef struct cs_solver_params {
    int32_t max_iter;  /* cap on Newton steps (>= 0); the unrolled VJP takes exactly this K */
    int32_t flags;     /* 0; for cs_forward 0 or CS_FORWARD_CG; for cs_unrolled_vjp
                        * 0, CS_UNROLLED_RECORD or CS_UNROLLED_REPLAY */
    double tol;        /* stopping tolerance (>= 0), see cs_forward */
} cs_solver_params;

/* cs_unrolled_vjp phases (cs_solver_params.flags).  0 runs both.  RECORD runs
 * the K-step solve, fills the tape and writes a_out, status and iters (iters
 * required); gradient outputs are not touched and may be NULL.  REPLAY runs
 * only the reverse sweep over a tape written by a RECORD call with the same
 * inputs and K, reading status and iters as that call left them (abar and
 * every gradient output required); a_out is not touched and may be NULL.
 * This is how a reverse-mode AD of the solver trace holds the trace from the
 * forward pass to the backward pass. */
#define CS_UNROLLED_RECORD 1
#define CS_UNROLLED_REPLAY 2

/* cs_forward solver (cs_solver_params.flags).  0: Newton steps.
 * CS_FORWARD_CG: preconditioned nonlinear conjugate gradients for the same
 * minimiser (Sec. III-B names Newton and nonlinear CG as the two solvers; by
 * eqs. 11-14 the IFT derivative depends on the root only, so cs_ift_vjp and
 * cs_ift_jvp take its state unchanged).  Directions p_k = -z_k + beta_k p_{k-1},
 * z = M^{-1} F, Polak-Ribiere beta_k = max(0, F_k . (z_k - z_{k-1}) /
 * (F_{k-1} . z_{k-1})), restarted when the active set changes or p_k is not a
 * descent direction; the same exact line search.  Converged when
 * ||F|| <= tol tr(M) or sqrt(F . M^{-1} F) <= tol sqrt(tr(M)) (1 + ||a||_inf);
 * since L is M-strongly convex (H >= M), the second test bounds the distance
 * to the minimiser, ||a - a*||_M <= sqrt(F . M^{-1} F).  max_iter caps CG
 * steps, which a solve needs many more of than Newton steps.  The iterate and
 * every sum are FP64 for either dtype (FP32 storage: the a written is the FP64
 * iterate rounded, then refined as the Newton solve's is).  The state holds
 * the factor of H(A) at the returned iterate.  SMALL family only (batches it
 * supports; CS_EUNSUPPORTED otherwise). */
#define CS_FORWARD_CG 4

/* Bytes of the `state` buffer cs_forward writes and cs_ift_vjp reads: the
 * Cholesky factor of H(A*) as a packed lower triangle per instance (n (n+1)/2
 * values, instance i at element (off_nn[i] + off_n[i]) / 2), then, 256-byte
 * aligned, the active set A* (one byte per row, instance i at off_m[i]).
 * 0 on invalid arguments. */
size_t cs_state_bytes(const cs_batch *batch);

/* Bytes of the tape cs_unrolled_vjp needs for K recorded steps: per instance
 * and step (a_k, p_k, the packed factor of H_k, r_k, q_k, alpha_k, c_k) in the
 * batch's dtype plus the step's active set and line-search piece (one byte per
 * row each).  Grows linearly in K. */
size_t cs_unrolled_tape_bytes(const cs_batch *batch, int32_t K);

/* Forward solve (Sec. III-B): from a_init (a0 when NULL) take Newton steps
 * p = -H^{-1} F with F = M (a - a0) + J^T (D o A o r) (eq. 6) and
 * H = M + J^T diag(D o A) J (eq. 9), A = 1[r < 0], each scaled by the exact
 * minimiser of L along p (eq. 10).  Iterate a_k is converged when
 * ||F(a_k)||_2 <= tol tr(M), or (k >= 1) the step into it was small,
 * ||a_k - a_{k-1}||_inf <= tol (1 + ||a_k||_inf), and left the active set
 * unchanged, A(a_k) = A(a_{k-1}); at most max_iter steps are taken.  M is
 * read as symmetric (the SMALL family reads its lower triangle only).
 * params->flags = CS_FORWARD_CG selects the conjugate-gradient solver instead.
 * Writes a_out [n per instance], state (factor of H at the returned iterate and
 * its active set), status [B] (CS_ST_* bits) and, if non-NULL, iters [B]
 * (steps taken).  a_init, iters may be NULL. */
int cs_forward(const cs_batch *batch, const cs_solver_params *params,
               const void *M, const void *J, const void *a0, const void *aref, const void *D,
               const void *a_init, void *a_out, void *state, size_t state_bytes,
               int32_t *status, int32_t *iters, void *stream);

/* IFT vector-Jacobian product (Sec. III-C, eq. 17) at the solution `a` that
 * cs_forward returned, using the saved factor of H(A*) and A* from `state`:
 *   H lambda = abar,  sigma = J lambda,  w = D o A* o r*,
 *   a0bar = M^T lambda,  arefbar = D o A* o sigma,  Dbar = -A* o r* o sigma,
 *   Jbar = -(w lambda^T + arefbar a^T),  Mbar = -lambda (a - a0)^T.
 * Each of the five outputs may be NULL (not computed).  Inputs must be the
 * ones given to the cs_forward call that wrote `state`.  If that call stopped
 * at max_iter the product linearises at the returned iterate. */
int cs_ift_vjp(const cs_batch *batch, const void *state, size_t state_bytes,
               const void *M, const void *J, const void *a0, const void *aref, const void *D,
               const void *a, const void *abar,
               void *a0bar, void *arefbar, void *Jbar, void *Dbar, void *Mbar, void *stream);

/* IFT Jacobian-vector products (Sec. III-C, eq. 15, forward mode): for k
 * tangent directions (da0_j, daref_j) of a0 and aref per instance, the
 * directional derivatives of the solution cs_forward returned,
 *   da_j = -F_a^{-1} F_theta (da0_j, daref_j) = H^{-1} (M da0_j + J^T (D o A* o daref_j)),
 * with the saved factor of H(A*) and A* from `state` (the same inputs as that
 * cs_forward call).  These are the columns of the linearised contact dynamics
 * an iLQR step needs: a direction of the actuation enters through a0, a
 * direction of the velocity through aref.  Layout, direction-major: instance
 * i's k directions of a0 at element k * off_n[i] of da0 (k x n), of aref at
 * k * off_m[i] of daref (k x m), results at k * off_n[i] of da (k x n); uniform
 * batches use off_n[i] = i n, off_m[i] = i m.  da0 or daref may be NULL (zero
 * tangent); da is required when k > 0.  k >= 0.  n <= 96 per instance (else
 * CS_EUNSUPPORTED).  Arithmetic in FP64 for both dtypes (two steps of
 * iterative refinement with the saved factor). */
int cs_ift_jvp(const cs_batch *batch, const void *state, size_t state_bytes,
               const void *M, const void *J, const void *D, int32_t k,
               const void *da0, const void *daref, void *da, void *stream);

/* Unrolled-trace VJP (the baseline gradient): runs exactly K = params->max_iter
 * steps of the same solver from a0 (steps after the stopping rule fires are the
 * identity), records each step on `tape`, then differentiates abar . a_K
 * through the recorded trace in reverse with the active sets and line-search
 * pieces held fixed.  Writes a_out, the five gradients (each non-NULL),
 * status [B] and, if non-NULL, iters [B].  tape_bytes must be at least
 * cs_unrolled_tape_bytes(batch, K). */
int cs_unrolled_vjp(const cs_batch *batch, const cs_solver_params *params,
                    const void *M, const void *J, const void *a0, const void *aref, const void *D,
                    const void *abar, void *a_out,
                    void *a0bar, void *arefbar, void *Jbar, void *Dbar, void *Mbar,
                    void *tape, size_t tape_bytes, int32_t *status, int32_t *iters,
                    void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as cs_unrolled_vjp with flags 0 (record and reverse sweep in
 * one call), with the tape in a library-owned static device array of
 * CS_STATIC_TAPE_BYTES bytes instead of a caller buffer.  Each GPU the
 * library runs on holds its own array until the process ends; every call on
 * a GPU uses that GPU's array (on the device current at the call), so calls
 * that overlap on one GPU (different streams, no ordering between them) race
 * and give undefined results.  The tape is written before it is read within
 * a call: nothing carries over from the previous call.  Returns CS_ENOSPC
 * when cs_unrolled_tape_bytes(batch, params->max_iter) exceeds
 * CS_STATIC_TAPE_BYTES, CS_EINVAL for params->flags != 0 and otherwise the
 * errors of cs_unrolled_vjp.  Allocates nothing. */
#define CS_STATIC_TAPE_BYTES ((size_t)64 << 20)
int cs_unrolled_vjp_static(const cs_batch *batch, const cs_solver_params *params,
                           const void *M, const void *J, const void *a0, const void *aref,
                           const void *D, const void *abar, void *a_out,
                           void *a0bar, void *arefbar, void *Jbar, void *Dbar, void *Mbar,
                           int32_t *status, int32_t *iters, void *stream);

/* Whole rollouts through the solve in one launch (Sec. IV-A: a
 * semi-implicit trajectory v_{t+1} = v_t + h a_t, a_t the contact solve's
 * solution; Sec. III-C, eq. 17: each solve's adjoint; Sec. IV-B: the forward's
 * states kept for, or recomputed in, the backward).  Per instance and step
 * t = 0 .. horizon-1, with M, J, D fixed over the horizon:
 *   a0_t = M^{-1} tau_t,   aref_t = -b_damp J v_t + c,   a_t = solve (as
 *   cs_forward: Newton, exact line search, the same stopping rule, starting
 *   at a0_t),   v_{t+1} = v_t + h a_t.
 * The backward, from v-bar_T (given, or 2 (v_T - v_goal), the gradient of
 * ||v_T - v_goal||^2), runs t = horizon-1 .. 0:
 *   lambda_t = H_t^{-1} (h v-bar_{t+1}),  tau-bar_t = lambda_t,
 *   v-bar_t = v-bar_{t+1} - b_damp J^T (D o A_t o J lambda_t),
 * and writes tau-bar and v-bar_0.  flags: CS_ROLLOUT_FORWARD and/or
 * CS_ROLLOUT_BACKWARD (both: one launch for the loss gradient), and
 * CS_ROLLOUT_RECOMPUTE to keep only each step's active set (m bytes) and
 * rebuild H_t = M + J^T diag(D o A_t) J in the backward instead of keeping
 * its factor.  A BACKWARD-only call reads the workspace and status a FORWARD
 * call with the same inputs and flags left, and needs vbar_T.  Layouts:
 * M [n x n], J [m x n] row-major, D and c [m], v0, v_goal, vbar_T, v_T,
 * v0_bar [n] at the batch's offsets; tau and tau_bar step-major,
 * [horizon][total_n].  c may be NULL (zero).  status [B] (required): the
 * CS_ST_* bits of every step OR-ed, CONVERGED only when every step
 * converged; iters [B] (may be NULL): Newton steps over the horizon.  n <= 32
 * per instance and J resident in LDS (m n + 3 n^2 + 5 m values within
 * 160 KiB), else CS_EUNSUPPORTED.  Workspace: cs_rollout_workspace_bytes. */
typedef struct cs_rollout_params {
    int32_t horizon;   /* steps T >= 1 */
    int32_t flags;     /* CS_ROLLOUT_FORWARD | CS_ROLLOUT_BACKWARD [| CS_ROLLOUT_RECOMPUTE] */
    int32_t max_iter;  /* Newton steps per solve (>= 0) */
    int32_t reserved;  /* 0 */
    double tol;        /* stopping tolerance of each solve (>= 0) */
    double h;          /* time step */
    double b_damp;     /* damping of the reference acceleration */
} cs_rollout_params;
#define CS_ROLLOUT_FORWARD 1
#define CS_ROLLOUT_BACKWARD 2
#define CS_ROLLOUT_RECOMPUTE 4

/* Workspace bytes for cs_rollout: per step, the factors of H_t (omitted with
 * CS_ROLLOUT_RECOMPUTE) and the active sets.  0 on invalid arguments. */
size_t cs_rollout_workspace_bytes(const cs_batch *batch, const cs_rollout_params *params);

int cs_rollout(const cs_batch *batch, const cs_rollout_params *params, const void *M,
               const void *J, const void *D, const void *c, const void *v0, const void *tau,
               const void *v_goal, const void *vbar_T, void *v_T, void *tau_bar, void *v0_bar,
               void *workspace, size_t workspace_bytes, int32_t *status, int32_t *iters,
               void *stream);

/* Round (elliptic) Coulomb cone (Sec. III-A, eqs. 2, 3, 5): contact c of an
 * instance owns rows 3c (normal) and 3c+1, 3c+2 (tangential) of J and aref, so
 * every instance's row count is a multiple of 3 (a packed instance that is
 * not gets CS_ST_BADDESC; a uniform batch, CS_EINVAL); dn, dt and mu hold one
 * value per contact, instance i's at off_m[i] / 3 (uniform: i m / 3):
 * R^{-1} = diag(dn, dt, dt) > 0 and mu >= 0.  The contact's regulariser is the
 * R^{-1}-weighted squared distance of u_c = J_c a - aref_c to the dual cone
 * {z_N >= mu |z_T|}; with x = (sqrt(dn) u_N, sqrt(dt) u_T), mh = mu sqrt(dn/dt),
 * nn = x_N, t = |x_T| it is 0 where nn >= mh t (zone 0), (nn^2 + t^2) / 2
 * where mh nn + t <= 0 (zone 2), (mh t - nn)^2 / (2 (1 + mh^2)) otherwise
 * (zone 1), with closed-form gradient w_c and 3 x 3 Hessian block G_c.
 * cs_forward_ell: Newton steps with H = M + sum_c J_c^T G_c J_c and the exact
 * line search (the root of phi', found by safeguarded Newton steps), the
 * stopping rule of cs_forward with the zone pattern in place of the active set;
 * params->flags must be 0.  The state layout is cs_forward's: the factor of H
 * at the returned iterate, then per row one byte, the contact's zone in its
 * normal row's byte (0 in the tangential rows').  Arithmetic in FP64 for both
 * dtypes.  n <= 32 and J resident in LDS (within 160 KiB), else
 * CS_EUNSUPPORTED. */
int cs_forward_ell(const cs_batch *batch, const cs_solver_params *params, const void *M,
                   const void *J, const void *a0, const void *aref, const void *dn, const void *dt,
                   const void *mu, const void *a_init, void *a_out, void *state,
                   size_t state_bytes, int32_t *status, int32_t *iters, void *stream);

/* IFT VJP with the round cone (eq. 17) at the solution cs_forward_ell returned,
 * with its zones and factor: H lambda = abar, sigma = J lambda,
 *   a0bar = M^T lambda, arefbar_c = G_c sigma_c, Jbar = -(w lambda^T + arefbar a^T),
 *   Mbar = -lambda (a - a0)^T,  (dn, dt, mu)bar_c = -sigma_c . dw_c/d(dn, dt, mu)
 * (at fixed u_c).  Every output may be NULL.  Layouts as cs_forward_ell. */
int cs_ift_vjp_ell(const cs_batch *batch, const void *state, size_t state_bytes,
                   const void *M, const void *J, const void *a0, const void *aref, const void *dn,
                   const void *dt, const void *mu, const void *a, const void *abar, void *a0bar,
                   void *arefbar, void *Jbar, void *dnbar, void *dtbar, void *mubar, void *Mbar,
                   void *stream);

/* Mixed regularised rows (Sec. III-A's other constraint rows): row i has a
 * kind (one byte): 0 one-sided (a pyramid edge or a limit), s = D min(r, 0)^2 / 2;
 * 1 equality, s = D r^2 / 2; 2 friction loss with bound floss_i >= 0 (its force
 * saturates at +-floss), s = D r^2 / 2 for |r| <= floss / D and
 * floss |r| - floss^2 / (2 D) beyond (floss is read for kind 2 only; D > 0).
 * cs_forward_rows: Newton steps with H = M + J^T diag(g) J (g_i = D_i where the
 * row is in its quadratic zone, else 0), the exact line search (phi' is
 * piecewise linear), the stopping rule of cs_forward with the zone pattern in
 * place of the active set; params->flags must be 0.  The state layout is
 * cs_forward's, each row's byte holding its zone: 0 no force, 1 quadratic,
 * 2 / 3 saturated at +floss / -floss.  kind [total_m] and floss [total_m] at
 * off_m.  Arithmetic in FP64 for both dtypes.  n <= 32 and J resident in LDS
 * (within 160 KiB), else CS_EUNSUPPORTED; a bad kind or D <= 0 gives
 * CS_ST_NONFINITE. */
int cs_forward_rows(const cs_batch *batch, const cs_solver_params *params, const void *M,
                    const void *J, const void *a0, const void *aref, const void *D,
                    const uint8_t *kind, const void *floss, const void *a_init, void *a_out,
                    void *state, size_t state_bytes, int32_t *status, int32_t *iters,
                    void *stream);

/* IFT VJP with mixed rows (eq. 17) at the solution cs_forward_rows returned,
 * with its zones and factor: H lambda = abar, sigma = J lambda,
 *   a0bar = M^T lambda, arefbar_i = g_i sigma_i, Dbar_i = -r_i sigma_i (zone 1,
 *   else 0), flossbar_i = -sigma_i (zone 2), +sigma_i (zone 3), else 0,
 *   Jbar = -(w lambda^T + arefbar a^T), Mbar = -lambda (a - a0)^T.
 * Every output may be NULL.  Layouts as cs_forward_rows. */
int cs_ift_vjp_rows(const cs_batch *batch, const void *state, size_t state_bytes,
                    const void *M, const void *J, const void *a0, const void *aref, const void *D,
                    const uint8_t *kind, const void *floss, const void *a, const void *abar,
                    void *a0bar, void *arefbar, void *Jbar, void *Dbar, void *flossbar, void *Mbar,
                    void *stream);

/* Name of an error code. */
const char *cs_strerror(int code);

/* Library ABI version (bumped on incompatible changes). */
int cs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CS_H */
