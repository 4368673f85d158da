// cs_generic.hpp -- team-per-instance kernels (any n <= 128, m <= 32 NT).
//
// One workgroup of NT threads solves one instance at a time (grid-stride over
// the batch in `order`).  The Newton matrix and its Cholesky factor live in
// LDS; rows of J are distributed over the threads (row i -> thread i mod NT)
// and read from global memory; columns and matrix entries are distributed the
// same way.  This path covers every supported shape; the small-instance
// kernels in cs_small.hpp are the fast path for small n.
#pragma once

#include "cs_device.hpp"

namespace cs {

// LDS carve-up shared by the generic kernels.
template <typename T>
struct GenLds {
    T *H, *diag, *a, *a0, *F, *p, *y, *v, *u, *pb, *ab, *red, *wk;
    T *r, *q, *Dv, *c1, *c2;
    uint8_t *A, *Ap;
};

// Row stride of H in LDS: odd, so that rows handled by consecutive threads
// sit in distinct LDS banks.
__host__ __device__ inline int gen_ld(int n) { return n | 1; }

__host__ __device__ inline size_t gen_lds_bytes(int nmax, int mmax, int NT, size_t s) {
    size_t nT = (size_t)nmax * (nmax + 1) + 11 * (size_t)nmax + 16 * (size_t)(NT / 64) + 16 * 17 +
                5 * (size_t)mmax;
    return nT * s + 2 * (size_t)mmax + 64;
}

template <typename T>
__device__ inline GenLds<T> gen_carve(unsigned char *smem, int nmax, int mmax, int NT) {
    GenLds<T> L;
    T *p = reinterpret_cast<T *>(smem);
    L.H = p; p += (size_t)nmax * (nmax + 1);   // row stride gen_ld(n) <= nmax + 1
    L.diag = p; p += nmax;
    L.a = p; p += nmax;
    L.a0 = p; p += nmax;
    L.F = p; p += nmax;
    L.p = p; p += nmax;
    L.y = p; p += nmax;
    L.v = p; p += nmax;
    L.u = p; p += nmax;
    L.pb = p; p += nmax;
    L.ab = p; p += nmax;
    L.red = p; p += 16 * (NT / 64);
    L.wk = p; p += 16 * 17;
    L.r = p; p += mmax;
    L.q = p; p += mmax;
    L.Dv = p; p += mmax;
    L.c1 = p; p += mmax;
    L.c2 = p; p += mmax;
    unsigned char *b = reinterpret_cast<unsigned char *>(p);
    L.A = b; b += mmax;
    L.Ap = b;
    return L;
}

// Shared per-iteration pieces --------------------------------------------

// r = J a - aref, A = 1[r < 0] for this thread's rows.  Returns whether any
// of this thread's rows changed activity.
template <int NT, typename T>
__device__ inline bool gen_residual(int n, int m, const T *__restrict__ J, const T *__restrict__ aref,
                                    const GenLds<T> &L) {
    bool changed = false;
    for (int i = threadIdx.x; i < m; i += NT) {
        const T *Ji = J + (size_t)i * n;
        T s = T(0);
        for (int j = 0; j < n; ++j) s += Ji[j] * L.a[j];
        const T r = s - aref[i];
        L.r[i] = r;
        const uint8_t an = r < T(0);
        changed |= an != L.A[i];
        L.A[i] = an;
    }
    return changed;
}

// F = M (a - a0) + J^T (D o A o r)  (eq. 6), threads over columns.
template <int NT, typename T>
__device__ inline void gen_gradient(int n, int m, const T *__restrict__ M, const T *__restrict__ J,
                                    const GenLds<T> &L) {
    for (int j = threadIdx.x; j < n; j += NT) {
        T f = T(0);
#pragma unroll 16
        for (int l = 0; l < n; ++l) f += M[(size_t)l * n + j] * (L.a[l] - L.a0[l]);
        for (int i = 0; i < m; ++i)
            if (L.A[i]) f += J[(size_t)i * n + j] * (L.Dv[i] * L.r[i]);
        L.F[j] = f;
    }
}

// H = M + J^T diag(D o A) J  (eq. 9), lower triangle, threads over entries.
template <int NT, typename T>
__device__ inline void gen_hessian(int n, int m, const T *__restrict__ M, const T *__restrict__ J,
                                   const GenLds<T> &L) {
    const int ne = n * (n + 1) / 2;
    for (int e = threadIdx.x; e < ne; e += NT) {
        int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        while (j * (j + 1) / 2 > e) --j;
        while ((j + 1) * (j + 2) / 2 <= e) ++j;
        const int l = e - j * (j + 1) / 2;
        T h = M[(size_t)j * n + l];
        for (int i = 0; i < m; ++i)
            if (L.A[i]) h += L.Dv[i] * J[(size_t)i * n + j] * J[(size_t)i * n + l];
        L.H[j * gen_ld(n) + l] = h;
    }
}

// Forward solve ------------------------------------------------------------

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_forward_generic(
    BatchView bv, int max_iter, T tol, int nmax, int mmax, const T *__restrict__ gM,
    const T *__restrict__ gJ, const T *__restrict__ ga0, const T *__restrict__ garef,
    const T *__restrict__ gD, const T *__restrict__ gainit, T *__restrict__ gaout,
    T *__restrict__ gfac, uint8_t *__restrict__ gmask, int32_t *__restrict__ gstatus,
    int32_t *__restrict__ giters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const GenLds<T> L = gen_carve<T>(smem, nmax, mmax, NT);
    const int tid = threadIdx.x;
    for (int w = blockIdx.x; w < bv.B; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) {   // team-uniform
            mark_bad(I, gstatus, giters, tid == 0);
            continue;
        }
        const int n = I.n, m = I.m, ldh = gen_ld(n);
        const T *M = gM + I.onn, *J = gJ + I.omn, *a0 = ga0 + I.on, *aref = garef + I.om,
                *D = gD + I.om;
        bool bad = false;
        for (int j = tid; j < n; j += NT) {
            const T x = a0[j];
            const T y = gainit ? gainit[I.on + j] : x;
            L.a0[j] = x;
            L.a[j] = y;
            bad |= !finite_val(x) || !finite_val(y);
        }
        for (int i = tid; i < m; i += NT) {
            const T d = D[i];
            L.Dv[i] = d;
            bad |= !finite_val(d) || !finite_val(aref[i]);
        }
        for (int e = tid; e < n * n; e += NT) {
            const T x = M[e];
            L.H[(e / n) * ldh + e % n] = x;
            bad |= !finite_val(x);
        }
        for (int e = tid; e < m * n; e += NT) bad |= !finite_val(J[e]);
        const int anybad = __syncthreads_or(bad);
        int st = 0, k = 0;
        if (anybad) {
            st = ST_NONFINITE;
        } else if (!team_cholesky<NT>(L.H, L.diag, n, ldh, L.wk)) {
            st = ST_NOTSPD;
        }
        if (st == 0) {
            T trM = T(0);
            for (int j = 0; j < n; ++j) trM += M[(size_t)j * n + j];
            T step_inf = T(-1);
            int lsfail = 0;
            for (k = 0;; ++k) {
                const bool same = !__syncthreads_or(gen_residual<NT>(n, m, J, aref, L));
                gen_gradient<NT>(n, m, M, J, L);
                __syncthreads();
                T g2 = T(0), anorm = T(0);
                for (int j = 0; j < n; ++j) {
                    g2 += L.F[j] * L.F[j];
                    anorm = fmax(anorm, fabs(L.a[j]));
                }
                if (sqrt(g2) <= tol * trM ||
                    (step_inf >= T(0) && same && step_inf <= tol * (T(1) + anorm))) {
                    st = ST_CONVERGED;
                    break;
                }
                if (k == max_iter) { st = ST_MAXITER; break; }
                gen_hessian<NT>(n, m, M, J, L);
                for (int j = tid; j < n; j += NT) L.y[j] = -L.F[j];
                __syncthreads();
                if (!team_cholesky<NT>(L.H, L.diag, n, ldh, L.wk)) { st = ST_NOTSPD; break; }
                team_chol_solve<NT>(L.H, L.diag, L.y, L.p, n, ldh);
                // q = J p; M p and M (a - a0) for the line search coefficients
                for (int i = tid; i < m; i += NT) {
                    const T *Ji = J + (size_t)i * n;
                    T s = T(0);
                    for (int j = 0; j < n; ++j) s += Ji[j] * L.p[j];
                    L.q[i] = s;
                }
                for (int j = tid; j < n; j += NT) {
                    T mp = T(0), md = T(0);
#pragma unroll 16
                    for (int l = 0; l < n; ++l) {
                        const T mlj = M[(size_t)l * n + j];   // = M[j][l]: M is symmetric
                        mp += mlj * L.p[l];
                        md += mlj * (L.a[l] - L.a0[l]);
                    }
                    L.v[j] = mp;
                    L.u[j] = md;
                }
                __syncthreads();
                T c0 = T(0), b0 = T(0);
                for (int j = 0; j < n; ++j) {
                    c0 += L.p[j] * L.v[j];
                    b0 += L.p[j] * L.u[j];
                }
                uint32_t bits;
                T cpiece;
                int fl;
                const T alpha = team_line_search<NT>(m, L.r, L.q, L.Dv, c0, b0, L.red, bits,
                                                     cpiece, fl);
                lsfail |= fl;
                step_inf = T(0);
                for (int j = 0; j < n; ++j) step_inf = fmax(step_inf, fabs(alpha * L.p[j]));
                __syncthreads();
                for (int j = tid; j < n; j += NT) L.a[j] += alpha * L.p[j];
                __syncthreads();
            }
            if (lsfail) st |= ST_LSFAIL;
            if (st & (ST_CONVERGED | ST_MAXITER)) {
                // factor of H at the returned iterate (A from its residual)
                gen_hessian<NT>(n, m, M, J, L);
                __syncthreads();
                if (!team_cholesky<NT>(L.H, L.diag, n, ldh, L.wk)) st = ST_NOTSPD;
            }
        }
        const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
        const T nanv = T(__builtin_nan(""));
        for (int j = tid; j < n; j += NT) gaout[I.on + j] = ok ? L.a[j] : nanv;
        T *fac = gfac + fac_offset(I);
        for (int e = tid; e < n * n; e += NT) {
            const int j = e / n, l = e - (e / n) * n;
            if (l < j) fac[j * (j + 1) / 2 + l] = ok ? L.H[j * ldh + l] : nanv;
            else if (l == j) fac[j * (j + 1) / 2 + l] = ok ? L.diag[j] : nanv;
        }
        for (int i = tid; i < m; i += NT) gmask[I.om + i] = ok ? L.A[i] : 0;
        if (tid == 0) {
            gstatus[I.b] = st;
            if (giters) giters[I.b] = k;
        }
        __syncthreads();
    }
}

// IFT VJP -------------------------------------------------------------------

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_ift_vjp_generic(
    BatchView bv, int nmax, int mmax, const T *__restrict__ gfac, const uint8_t *__restrict__ gmask,
    const T *__restrict__ gM, const T *__restrict__ gJ, const T *__restrict__ ga0,
    const T *__restrict__ garef, const T *__restrict__ gD, const T *__restrict__ ga,
    const T *__restrict__ gabar, T *__restrict__ ga0bar, T *__restrict__ garefbar,
    T *__restrict__ gJbar, T *__restrict__ gDbar, T *__restrict__ gMbar) {
    extern __shared__ __align__(16) unsigned char smem[];
    const GenLds<T> L = gen_carve<T>(smem, nmax, mmax, NT);
    const int tid = threadIdx.x;
    for (int w = blockIdx.x; w < bv.B; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) continue;   // team-uniform: outputs untouched
        const int n = I.n, m = I.m, ldh = gen_ld(n);
        const T *M = gM + I.onn, *J = gJ + I.omn, *aref = garef + I.om, *D = gD + I.om;
        const T *fac = gfac + fac_offset(I);
        for (int e = tid; e < n * n; e += NT) {
            const int j = e / n, l = e - (e / n) * n;
            if (l < j) L.H[j * ldh + l] = fac[j * (j + 1) / 2 + l];
            else if (l == j) L.diag[j] = fac[j * (j + 1) / 2 + l];
        }
        for (int j = tid; j < n; j += NT) {
            L.a[j] = ga[I.on + j];
            L.a0[j] = ga0[I.on + j];
            L.y[j] = gabar[I.on + j];
        }
        __syncthreads();
        // lambda = H^{-1} abar (H symmetric, so H^T lambda = abar is the same system),
        // then one step of iterative refinement with H v = M v + J^T (D o A* o J v)
        team_chol_solve<NT>(L.H, L.diag, L.y, L.u, n, ldh);
        for (int i = tid; i < m; i += NT) {
            const T *Ji = J + (size_t)i * n;
            T s = T(0);
            for (int j = 0; j < n; ++j) s += Ji[j] * L.u[j];
            L.q[i] = gmask[I.om + i] ? D[i] * s : T(0);
        }
        __syncthreads();
        for (int j = tid; j < n; j += NT) {
            T s = gabar[I.on + j];
#pragma unroll 16
            for (int l = 0; l < n; ++l) s -= M[(size_t)l * n + j] * L.u[l];
            for (int i = 0; i < m; ++i) s -= J[(size_t)i * n + j] * L.q[i];
            L.y[j] = s;
        }
        __syncthreads();
        team_chol_solve<NT>(L.H, L.diag, L.y, L.p, n, ldh);
        for (int j = tid; j < n; j += NT) L.u[j] += L.p[j];
        __syncthreads();
        for (int i = tid; i < m; i += NT) {
            const T *Ji = J + (size_t)i * n;
            T ja = T(0), sig = T(0);
            for (int j = 0; j < n; ++j) {
                ja += Ji[j] * L.a[j];
                sig += Ji[j] * L.u[j];
            }
            const T r = ja - aref[i];
            const bool act = gmask[I.om + i] != 0;
            const T d = D[i];
            const T wv = act ? d * r : T(0);
            const T ar = act ? d * sig : T(0);
            if (garefbar) garefbar[I.om + i] = ar;
            if (gDbar) gDbar[I.om + i] = act ? -r * sig : T(0);
            L.c1[i] = wv;
            L.c2[i] = ar;
        }
        __syncthreads();
        if (gJbar) {
            for (int e = tid; e < m * n; e += NT) {
                const int i = e / n, j = e - (e / n) * n;
                gJbar[I.omn + e] = -(L.c1[i] * L.u[j] + L.c2[i] * L.a[j]);
            }
        }
        if (ga0bar) {
            for (int j = tid; j < n; j += NT) {
                T s = T(0);
                for (int l = 0; l < n; ++l) s += M[(size_t)l * n + j] * L.u[l];
                ga0bar[I.on + j] = s;
            }
        }
        if (gMbar) {
            for (int e = tid; e < n * n; e += NT) {
                const int j = e / n, l = e - (e / n) * n;
                gMbar[I.onn + e] = -L.u[j] * (L.a[l] - L.a0[l]);
            }
        }
        __syncthreads();
    }
}

// Unrolled VJP ----------------------------------------------------------------
//
// Tape layout: see the comment above rec_T_elems in cs_device.hpp.

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_unrolled_generic(
    BatchView bv, int K, int mode, T tol, int nmax, int mmax, const T *__restrict__ gM,
    const T *__restrict__ gJ, const T *__restrict__ ga0, const T *__restrict__ garef,
    const T *__restrict__ gD, const T *__restrict__ gabar, T *__restrict__ gaout,
    T *__restrict__ ga0bar, T *__restrict__ garefbar, T *__restrict__ gJbar,
    T *__restrict__ gDbar, T *__restrict__ gMbar, T *__restrict__ tapeT,
    uint8_t *__restrict__ tapeB, int32_t *__restrict__ gstatus, int32_t *__restrict__ giters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const GenLds<T> L = gen_carve<T>(smem, nmax, mmax, NT);
    const int tid = threadIdx.x;
    for (int w = blockIdx.x; w < bv.B; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) {   // team-uniform
            if (mode != ST_REP) mark_bad(I, gstatus, giters, tid == 0);
            continue;
        }
        const int n = I.n, m = I.m, ldh = gen_ld(n);
        const T *M = gM + I.onn, *J = gJ + I.omn, *a0 = ga0 + I.on, *aref = garef + I.om,
                *D = gD + I.om;
        T *a0bar = ga0bar + I.on, *arefbar = garefbar + I.om, *Jbar = gJbar + I.omn,
          *Dbar = gDbar + I.om, *Mbar = gMbar + I.onn;
        const int ne = n * (n + 1) / 2;
        const size_t recT = (size_t)rec_T_elems(n, m);
        T *tT = tapeT + tape_T_offset(I, K);
        uint8_t *tB = tapeB + tape_B_offset(I, K);

        const bool do_fwd = mode != ST_REP, do_rev = mode != ST_REC;
        // zero the accumulated gradients
        if (do_rev) {
            for (int j = tid; j < n; j += NT) a0bar[j] = T(0);
            for (int i = tid; i < m; i += NT) { arefbar[i] = T(0); Dbar[i] = T(0); }
            for (int e = tid; e < m * n; e += NT) Jbar[e] = T(0);
            for (int e = tid; e < n * n; e += NT) Mbar[e] = T(0);
        }

        bool bad = false;
        for (int j = tid; j < n; j += NT) {
            const T x = a0[j];
            L.a0[j] = x;
            L.a[j] = x;
            bad |= !finite_val(x) || (do_rev && !finite_val(gabar[I.on + j]));
        }
        for (int i = tid; i < m; i += NT) {
            const T d = D[i];
            L.Dv[i] = d;
            bad |= !finite_val(d) || !finite_val(aref[i]);
        }
        for (int e = tid; e < n * n; e += NT) {
            const T x = M[e];
            L.H[(e / n) * ldh + e % n] = x;
            bad |= !finite_val(x);
        }
        for (int e = tid; e < m * n; e += NT) bad |= !finite_val(J[e]);
        const int anybad = __syncthreads_or(bad);
        int st = 0, steps = 0;
        if (!do_fwd) {
            st = gstatus[I.b] | (anybad ? ST_NONFINITE : 0);
            steps = giters[I.b];
        } else if (anybad) {
            st = ST_NONFINITE;
        } else if (!team_cholesky<NT>(L.H, L.diag, n, ldh, L.wk)) {
            st = ST_NOTSPD;
        }

        if (do_fwd && st == 0) {
            // ---- forward K steps with the tape
            T trM = T(0);
            for (int j = 0; j < n; ++j) trM += M[(size_t)j * n + j];
            T step_inf = T(-1);
            int lsfail = 0;
            bool conv = false;
            for (int k = 0; k < K; ++k) {
                const bool same = !__syncthreads_or(gen_residual<NT>(n, m, J, aref, L));
                gen_gradient<NT>(n, m, M, J, L);
                __syncthreads();
                T g2 = T(0), anorm = T(0);
                for (int j = 0; j < n; ++j) {
                    g2 += L.F[j] * L.F[j];
                    anorm = fmax(anorm, fabs(L.a[j]));
                }
                if (sqrt(g2) <= tol * trM ||
                    (step_inf >= T(0) && same && step_inf <= tol * (T(1) + anorm))) {
                    conv = true;
                    break;
                }
                gen_hessian<NT>(n, m, M, J, L);
                for (int j = tid; j < n; j += NT) L.y[j] = -L.F[j];
                __syncthreads();
                if (!team_cholesky<NT>(L.H, L.diag, n, ldh, L.wk)) { st = ST_NOTSPD; break; }
                team_chol_solve<NT>(L.H, L.diag, L.y, L.p, n, ldh);
                for (int i = tid; i < m; i += NT) {
                    const T *Ji = J + (size_t)i * n;
                    T s = T(0);
                    for (int j = 0; j < n; ++j) s += Ji[j] * L.p[j];
                    L.q[i] = s;
                }
                for (int j = tid; j < n; j += NT) {
                    T mp = T(0), md = T(0);
#pragma unroll 16
                    for (int l = 0; l < n; ++l) {
                        const T mlj = M[(size_t)l * n + j];   // = M[j][l]: M is symmetric
                        mp += mlj * L.p[l];
                        md += mlj * (L.a[l] - L.a0[l]);
                    }
                    L.v[j] = mp;
                    L.u[j] = md;
                }
                __syncthreads();
                T c0 = T(0), b0 = T(0);
                for (int j = 0; j < n; ++j) {
                    c0 += L.p[j] * L.v[j];
                    b0 += L.p[j] * L.u[j];
                }
                uint32_t bits;
                T cpiece;
                int fl;
                const T alpha = team_line_search<NT>(m, L.r, L.q, L.Dv, c0, b0, L.red, bits,
                                                     cpiece, fl);
                lsfail |= fl;
                // record step k
                T *rec = tT + (size_t)k * recT;
                uint8_t *recB = tB + (size_t)k * 2 * m;
                for (int j = tid; j < n; j += NT) {
                    rec[j] = L.a[j];
                    rec[n + j] = L.p[j];
                }
                for (int e = tid; e < n * n; e += NT) {
                    const int j = e / n, l = e - (e / n) * n;
                    if (l < j) rec[2 * n + j * (j + 1) / 2 + l] = L.H[j * ldh + l];
                    else if (l == j) rec[2 * n + j * (j + 1) / 2 + l] = L.diag[j];
                }
                for (int i = tid, jj = 0; i < m; i += NT, ++jj) {
                    rec[2 * n + ne + i] = L.r[i];
                    rec[2 * n + ne + m + i] = L.q[i];
                    recB[i] = L.A[i];
                    recB[m + i] = (bits >> jj) & 1u;
                }
                if (tid == 0) {
                    rec[2 * n + ne + 2 * m] = alpha;
                    rec[2 * n + ne + 2 * m + 1] = cpiece;
                }
                step_inf = T(0);
                for (int j = 0; j < n; ++j) step_inf = fmax(step_inf, fabs(alpha * L.p[j]));
                __syncthreads();
                for (int j = tid; j < n; j += NT) L.a[j] += alpha * L.p[j];
                __syncthreads();
                steps = k + 1;
            }
            if (st == 0) {
                if (!conv) {
                    const bool same = !__syncthreads_or(gen_residual<NT>(n, m, J, aref, L));
                    gen_gradient<NT>(n, m, M, J, L);
                    __syncthreads();
                    T g2 = T(0), anorm = T(0);
                    for (int j = 0; j < n; ++j) {
                        g2 += L.F[j] * L.F[j];
                        anorm = fmax(anorm, fabs(L.a[j]));
                    }
                    conv = sqrt(g2) <= tol * trM ||
                           (step_inf >= T(0) && same && step_inf <= tol * (T(1) + anorm));
                }
                st = conv ? ST_CONVERGED : ST_MAXITER;
                if (lsfail) st |= ST_LSFAIL;
            }
        }
        const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
        const T nanv = T(__builtin_nan(""));
        for (int j = tid; j < n; j += NT) {
            if (do_fwd) gaout[I.on + j] = ok ? L.a[j] : nanv;
            L.ab[j] = do_rev ? gabar[I.on + j] : T(0);
        }
        if (do_fwd && tid == 0) {
            gstatus[I.b] = st;
            if (giters) giters[I.b] = steps;
        }
        __syncthreads();

        // ---- reverse sweep over the recorded steps
        for (int k = (ok && do_rev ? steps : 0) - 1; k >= 0; --k) {
            const T *rec = tT + (size_t)k * recT;
            const uint8_t *recB = tB + (size_t)k * 2 * m;
            const T *rr = rec + 2 * n + ne, *rq = rr + m;
            const T alpha = rec[2 * n + ne + 2 * m], c = rec[2 * n + ne + 2 * m + 1];
            for (int j = tid; j < n; j += NT) {
                L.a[j] = rec[j];
                L.p[j] = rec[n + j];
            }
            for (int e = tid; e < n * n; e += NT) {
                const int j = e / n, l = e - (e / n) * n;
                if (l < j) L.H[j * ldh + l] = rec[2 * n + j * (j + 1) / 2 + l];
                else if (l == j) L.diag[j] = rec[2 * n + j * (j + 1) / 2 + l];
            }
            for (int i = tid; i < m; i += NT) {
                L.r[i] = rr[i];
                L.q[i] = rq[i];
                L.A[i] = recB[i];
                L.Ap[i] = recB[m + i];
            }
            __syncthreads();
            // a_{k+1} = a_k + alpha p ; alpha = -b / c
            T alphab = T(0);
            for (int j = 0; j < n; ++j) alphab += L.ab[j] * L.p[j];
            const T bb = -alphab / c;
            const T cb = -alphab * alpha / c;
            // per-row adjoints from c = p^T M p + sum_{A'} D q^2 and b = p^T M d + sum_{A'} D q r
            for (int i = tid; i < m; i += NT) {
                const T d = L.Dv[i], qi = L.q[i], ri = L.r[i];
                T qb = T(0), rb = T(0), db = T(0);
                if (L.Ap[i]) {
                    qb = T(2) * cb * d * qi + bb * d * ri;
                    rb = bb * d * qi;
                    db = cb * qi * qi + bb * qi * ri;
                }
                L.c1[i] = qb;   // q-bar
                L.c2[i] = rb;   // r-bar (partial)
                Dbar[i] += db;
            }
            __syncthreads();
            // p-bar = alpha abar + cb (M + M^T) p + bb M d + J^T qbar ; also M^T p for a-bar
            for (int j = tid; j < n; j += NT) {
                T mp = T(0), mtp = T(0), md = T(0);
                for (int l = 0; l < n; ++l) {
                    const T mjl = M[(size_t)j * n + l], mlj = M[(size_t)l * n + j];
                    mp += mjl * L.p[l];
                    mtp += mlj * L.p[l];
                    md += mjl * (L.a[l] - L.a0[l]);
                }
                T jq = T(0);
                for (int i = 0; i < m; ++i) jq += J[(size_t)i * n + j] * L.c1[i];
                L.pb[j] = alpha * L.ab[j] + cb * (mp + mtp) + bb * md + jq;
                L.v[j] = mtp;
                L.y[j] = L.pb[j];
            }
            __syncthreads();
            // u = H^{-1} pbar ; gbar = -u
            team_chol_solve<NT>(L.H, L.diag, L.y, L.u, n, ldh);
            // rows: Ju; D-bar, r-bar updates; J-bar row coefficients
            for (int i = tid; i < m; i += NT) {
                const T *Ji = J + (size_t)i * n;
                T ju = T(0);
                for (int j = 0; j < n; ++j) ju += Ji[j] * L.u[j];
                const T d = L.Dv[i], qi = L.q[i], ri = L.r[i];
                T rb = L.c2[i];
                T cu = T(0);
                T cp = L.c1[i];
                if (L.A[i]) {
                    Dbar[i] += -ju * (qi + ri);
                    rb += -d * ju;
                    cu = -d * (qi + ri);
                    cp += -d * ju;
                }
                L.c2[i] = rb;
                L.c1[i] = cp;
                L.q[i] = cu;   // reuse: coefficient of u in the J-bar row
                arefbar[i] -= rb;
            }
            __syncthreads();
            // J-bar += cp p^T + cu u^T + rb a_k^T
            for (int e = tid; e < m * n; e += NT) {
                const int i = e / n, j = e - (e / n) * n;
                Jbar[e] += L.c1[i] * L.p[j] + L.q[i] * L.u[j] + L.c2[i] * L.a[j];
            }
            // M-bar += p (cb p + bb d)^T - u (p + d)^T
            for (int e = tid; e < n * n; e += NT) {
                const int j = e / n, l = e - (e / n) * n;
                const T dl = L.a[l] - L.a0[l];
                Mbar[e] += L.p[j] * (cb * L.p[l] + bb * dl) - L.u[j] * (L.p[l] + dl);
            }
            // a_k-bar = abar + bb M^T p - M^T u + J^T rbar ; a0-bar -= bb M^T p - M^T u
            for (int j = tid; j < n; j += NT) {
                T mtu = T(0);
                for (int l = 0; l < n; ++l) mtu += M[(size_t)l * n + j] * L.u[l];
                T jr = T(0);
                for (int i = 0; i < m; ++i) jr += J[(size_t)i * n + j] * L.c2[i];
                const T through_m = bb * L.v[j] - mtu;
                L.pb[j] = L.ab[j] + through_m + jr;
                a0bar[j] -= through_m;
            }
            __syncthreads();
            for (int j = tid; j < n; j += NT) L.ab[j] = L.pb[j];
            __syncthreads();
        }
        // the first iterate is a0
        if (do_rev)
            for (int j = tid; j < n; j += NT) a0bar[j] += ok ? L.ab[j] : nanv;
        __syncthreads();
    }
}

}  // namespace cs
