// cs_rollout.hpp -- a whole semi-implicit rollout through the contact solve,
// forward and backward, in one launch (Sec. IV-A: trajectories through the
// solve, v_{t+1} = v_t + h a_t; Sec. III-C, eq. 17: the adjoint of each solve;
// Sec. IV-B: checkpointing of the forward for the backward).
//
// Per step t the solve takes a0_t = M^{-1} tau_t and aref_t = -b J v_t + c
// (c a per-row constant, the spring term of the reference acceleration), with
// M, J, D fixed over the horizon.  Its adjoint, for a-bar_t = h v-bar_{t+1}:
//   lambda_t = H_t^{-1} a-bar_t            (H_t = M + J^T diag(D o A_t) J),
//   tau-bar_t = M^{-T} (M^T lambda_t) = lambda_t,
//   v-bar_t = v-bar_{t+1} - b J^T (D o A_t o J lambda_t).
//
// One workgroup of one wave per instance (grid-stride over the batch).  J,
// M and the Cholesky factor of M are loaded into LDS once and serve every
// Newton step of every time step and the whole backward sweep: the layered
// rollout reads J from HBM in each of its 2T launches.  Newton steps follow
// the SMALL / team solvers (eqs. 6, 9, 10, the same stopping rule); the
// Newton matrix is assembled over a list of the active rows and kept while
// the active set is unchanged.  The forward saves each step's active set
// (and, unless recomputing, the factor of H_t) in a workspace; the backward
// reads them back in reverse order, or rebuilds H_t from J and A_t, which
// gives the forward's factor bit for bit.
#pragma once

#include "cs_device.hpp"

namespace cs {

constexpr int RO_NT = 64;
constexpr int RO_NMAX = 32;   // the one-wave team Cholesky's limit

struct RoLayout {
    int ldj;
    uint32_t J, M, Lm, dm, H, dh, vec, red, wk, rows, list, A, bytes;
};

__host__ __device__ inline RoLayout ro_layout(int nmax, int mmax, int s) {
    RoLayout L;
    L.ldj = nmax | 1;   // odd row stride: row-parallel reads of one column spread over banks
    uint32_t o = 0;
    auto take = [&o](uint64_t bytes) {
        const uint32_t r = o;
        o += (uint32_t)((bytes + 15) & ~uint64_t(15));
        return r;
    };
    const uint64_t mm = mmax > 0 ? (uint64_t)mmax : 1;
    const uint64_t nn = (uint64_t)nmax * nmax;
    L.J = take((uint64_t)s * mm * L.ldj);
    L.M = take((uint64_t)s * nn);
    L.Lm = take((uint64_t)s * nn);
    L.dm = take((uint64_t)s * nmax);
    L.H = take((uint64_t)s * nn);
    L.dh = take((uint64_t)s * nmax);
    L.vec = take((uint64_t)s * 10 * nmax);
    L.red = take((uint64_t)s * 16);
    L.wk = take((uint64_t)s * 16 * 17);
    L.rows = take((uint64_t)s * 5 * mm);
    L.list = take(4 * mm);
    L.A = take(mm);
    L.bytes = o;
    return L;
}

template <typename T>
struct RolloutArgs {
    const T *M, *J, *D, *cref, *v0, *tau, *vgoal, *vbarT;
    T *vT, *taubar, *v0bar;
    uint8_t *ws;        // workspace: per step, the factors (unless recomputing) then the masks
    int64_t ws_step;    // bytes per step
    int64_t mask_off;   // byte offset of the masks within a step
    int32_t *status, *iters;
    int64_t tot_n;
    int horizon, max_iter;
    bool fwd, bwd, recompute;
    T tol, h, bdamp;
};

// (j, l), l <= j, of packed lower-triangle entry e
__device__ inline void ro_tri(int e, int &j, int &l) {
    j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while (j * (j + 1) / 2 > e) --j;
    while ((j + 1) * (j + 2) / 2 <= e) ++j;
    l = e - j * (j + 1) / 2;
}

// H's lower triangle (row stride n) = M + sum over the listed rows of
// D_i J_ij J_il: thread tid owns entries tid + RO_NT k, k < E, and walks the
// rows once for all of them (independent accumulators, every load of a row
// issued together).
template <int E, typename T>
__device__ inline void ro_assemble(int n, int ne, int ldj, int cnt, const int *list, const T *Dv,
                                   const T *Js, const T *Ms, T *H) {
    const int tid = threadIdx.x;
    int jo[E], lo[E];
    T s[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int e = min(tid + RO_NT * k, ne - 1);   // clamped: every read in bounds
        int j, l;
        ro_tri(e, j, l);
        jo[k] = j;
        lo[k] = l;
        s[k] = T(0);
    }
#pragma unroll 2
    for (int c = 0; c < cnt; ++c) {
        const int i = list[c];
        const T d = Dv[i];
        const T *Jr = Js + i * ldj;
        T x[E], y[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            x[k] = Jr[jo[k]];
            y[k] = Jr[lo[k]];
        }
#pragma unroll
        for (int k = 0; k < E; ++k) s[k] += (d * x[k]) * y[k];
    }
#pragma unroll
    for (int k = 0; k < E; ++k)
        if (tid + RO_NT * k < ne) H[jo[k] * n + lo[k]] = Ms[jo[k] * n + lo[k]] + s[k];
}

template <typename T>
__global__ __launch_bounds__(RO_NT) void k_rollout(BatchView bv, int count, int nmax, int mmax,
                                                   RolloutArgs<T> g) {
    constexpr int NT = RO_NT;
    extern __shared__ __align__(16) unsigned char smem[];
    const RoLayout Lo = ro_layout(nmax, mmax, (int)sizeof(T));
    T *Js = reinterpret_cast<T *>(smem + Lo.J);
    T *Ms = reinterpret_cast<T *>(smem + Lo.M);
    T *Lm = reinterpret_cast<T *>(smem + Lo.Lm);
    T *dm = reinterpret_cast<T *>(smem + Lo.dm);
    T *H = reinterpret_cast<T *>(smem + Lo.H);
    T *dh = reinterpret_cast<T *>(smem + Lo.dh);
    T *vec = reinterpret_cast<T *>(smem + Lo.vec);
    T *red = reinterpret_cast<T *>(smem + Lo.red);
    T *wk = reinterpret_cast<T *>(smem + Lo.wk);
    T *rows = reinterpret_cast<T *>(smem + Lo.rows);
    int *list = reinterpret_cast<int *>(smem + Lo.list);
    uint8_t *A = smem + Lo.A;
    T *a = vec, *a0 = vec + nmax, *F = vec + 2 * nmax, *p = vec + 3 * nmax, *y = vec + 4 * nmax,
      *Mp = vec + 5 * nmax, *u = vec + 6 * nmax, *vel = vec + 7 * nmax, *vb = vec + 8 * nmax,
      *lam = vec + 9 * nmax;
    T *r = rows, *q = rows + mmax, *Dv = rows + 2 * mmax, *cr = rows + 3 * mmax,
      *ar = rows + 4 * mmax;
    const int tid = threadIdx.x;
    const int ldj = Lo.ldj;
    const T nanv = T(__builtin_nan(""));

    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) {   // team-uniform
            mark_bad(I, g.status, g.iters, tid == 0);
            continue;
        }
        const int n = I.n, m = I.m, ne = n * (n + 1) / 2;
        bool bad = false;
        for (int e = tid; e < m * n; e += NT) {
            const int i = e / n, j = e - i * n;
            const T x = g.J[I.omn + e];
            Js[i * ldj + j] = x;
            bad |= !finite_val(x);
        }
        for (int e = tid; e < n * n; e += NT) {
            const T x = g.M[I.onn + e];
            Ms[e] = x;
            Lm[e] = x;
            bad |= !finite_val(x);
        }
        for (int i = tid; i < m; i += NT) {
            const T d = g.D[I.om + i], c = g.cref ? g.cref[I.om + i] : T(0);
            Dv[i] = d;
            cr[i] = c;
            bad |= !finite_val(d) || !finite_val(c);
        }
        if (g.fwd)
            for (int j = tid; j < n; j += NT) {
                const T x = g.v0[I.on + j];
                vel[j] = x;
                bad |= !finite_val(x);
            }
        int st_all = __syncthreads_or(bad) ? ST_NONFINITE : 0;
        T trM = T(0);
        for (int j = 0; j < n; ++j) trM += Ms[j * n + j];

        // Active-row list of A (row order) by ballot; returns the count.
        auto make_list = [&]() {
            int cnt = 0;
            for (int base = 0; base < m; base += NT) {
                const int i = base + tid;
                const bool an = i < m && A[i] != 0;
                const uint64_t bal = __builtin_amdgcn_ballot_w64(an);
                if (an)
                    list[cnt + (int)__builtin_amdgcn_mbcnt_hi(
                                   (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] = i;
                cnt += (int)__builtin_popcountll(bal);
            }
            return cnt;
        };
        // H = M + J^T diag(D o A) J over the listed rows (eq. 9), lower triangle
        auto assemble = [&](int cnt) {
            switch ((ne + NT - 1) / NT) {   // entries per thread, 1 .. 9 for n <= 32
                case 1: ro_assemble<1>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
                case 2: ro_assemble<2>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
                case 3: ro_assemble<3>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
                case 4: ro_assemble<4>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
                case 5: ro_assemble<5>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
                case 6: ro_assemble<6>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
                case 7: ro_assemble<7>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
                case 8: ro_assemble<8>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
                default: ro_assemble<9>(n, ne, ldj, cnt, list, Dv, Js, Ms, H); break;
            }
            __syncthreads();
        };
        // out_j = sum over the listed rows of J_ij x_i (x per row), the two
        // half-waves taking alternate rows
        auto jt_rows = [&](int cnt, const T *x, int j) {
            const int half = tid >> 5;
            T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
            if (j < n) {
                // four rows per round with their own sums: their list and
                // row loads are in flight together
                int c = half;
                for (; c + 6 < cnt; c += 8) {
                    const int i0 = list[c], i1 = list[c + 2], i2 = list[c + 4], i3 = list[c + 6];
                    s0 += Js[i0 * ldj + j] * x[i0];
                    s1 += Js[i1 * ldj + j] * x[i1];
                    s2 += Js[i2 * ldj + j] * x[i2];
                    s3 += Js[i3 * ldj + j] * x[i3];
                }
                for (; c < cnt; c += 2) {
                    const int i = list[c];
                    s0 += Js[i * ldj + j] * x[i];
                }
            }
            const T s = (s0 + s1) + (s2 + s3);
            return s + __shfl_xor(s, 32, 64);
        };

        if (g.fwd) {
            int conv_all = 1, it_all = 0;
            if (st_all == 0 && !team_cholesky<NT>(Lm, dm, n, n, wk)) st_all = ST_NOTSPD;
            for (int t = 0; t < g.horizon && st_all == 0; ++t) {
                // a0 = M^{-1} tau_t; aref = -b J v_t + c
                bool tb = false;
                for (int j = tid; j < n; j += NT) {
                    const T x = g.tau[(int64_t)t * g.tot_n + I.on + j];
                    y[j] = x;
                    tb |= !finite_val(x);
                }
                if (__syncthreads_or(tb)) { st_all = ST_NONFINITE; break; }
                team_chol_solve<NT>(Lm, dm, y, a0, n, n);
                for (int i = tid; i < m; i += NT) {
                    T s = T(0);
                    for (int j = 0; j < n; ++j) s += Js[i * ldj + j] * vel[j];
                    ar[i] = -g.bdamp * s + cr[i];
                    A[i] = 0;
                }
                for (int j = tid; j < n; j += NT) a[j] = a0[j];
                __syncthreads();
                int st = 0, k, lsfail = 0;
                T step_inf = T(-1), alpha_prev = T(0);
                for (k = 0;; ++k) {
                    // residual and active set (eq. 6); after the first step
                    // r = J a - aref is carried, r <- r + alpha J p, with the
                    // previous step's q = J p
                    bool changed = false;
                    for (int i = tid; i < m; i += NT) {
                        T ri;
                        if (k == 0) {
                            T s = T(0);
#pragma unroll 8
                            for (int j = 0; j < n; ++j) s += Js[i * ldj + j] * a[j];
                            ri = s - ar[i];
                        } else {
                            ri = r[i] + alpha_prev * q[i];
                        }
                        r[i] = ri;
                        q[i] = Dv[i] * ri;   // w before the line search needs q
                        const uint8_t an = ri < T(0);
                        changed |= an != A[i];
                        A[i] = an;
                    }
                    const bool same = !__syncthreads_or(changed) && k > 0;
                    const int cnt = make_list();
                    __syncthreads();
                    // F = M (a - a0) + J^T (D o A o r); ||F||^2 and ||a||_inf by
                    // wave reductions of the lanes' entries
                    T fj = T(0), aj = T(0);
                    {
                        const int j = tid & 31;
                        const T s = jt_rows(cnt, q, j);
                        if (tid < 32 && j < n) {
                            // u = M (a - a0): formed at the first step, then
                            // carried, u <- u + alpha M p
                            T md = u[j];
                            if (k == 0) {
                                md = T(0);
                                for (int l = 0; l < n; ++l) md += Ms[j * n + l] * (a[l] - a0[l]);
                            }
                            u[j] = md;
                            fj = md + s;
                            F[j] = fj;
                            aj = fabs(a[j]);
                        }
                    }
                    const T g2 = wave_sum(fj * fj);
                    const T anorm = wave_max(aj);
                    __syncthreads();
                    // Newton matrix (kept while the active set is unchanged)
                    if (!same) {
                        assemble(cnt);
                        if (!team_cholesky<NT>(H, dh, n, n, wk)) { st = ST_NOTSPD; break; }
                    }
                    if (sqrt(g2) <= g.tol * trM ||
                        (same && step_inf >= T(0) && step_inf <= g.tol * (T(1) + anorm))) {
                        st = ST_CONVERGED;
                        break;
                    }
                    if (k == g.max_iter) { st = ST_MAXITER; break; }
                    for (int j = tid; j < n; j += NT) y[j] = -F[j];
                    __syncthreads();
                    team_chol_solve<NT>(H, dh, y, p, n, n);
                    for (int i = tid; i < m; i += NT) {
                        T s = T(0);
#pragma unroll 8
                        for (int j = 0; j < n; ++j) s += Js[i * ldj + j] * p[j];
                        q[i] = s;
                    }
                    // c0 = p^T M p, b0 = p^T M (a - a0) by wave reductions
                    T pm = T(0), pu = T(0);
                    if (tid < n) {
                        T s = T(0);
                        for (int l = 0; l < n; ++l) s += Ms[tid * n + l] * p[l];
                        Mp[tid] = s;
                        pm = p[tid] * s;
                        pu = p[tid] * u[tid];
                    }
                    const T c0 = wave_sum(pm), b0 = wave_sum(pu);
                    __syncthreads();
                    uint32_t bits;
                    T cpiece;
                    int fl;
                    const T alpha = team_line_search<NT>(m, r, q, Dv, c0, b0, red, bits, cpiece, fl);
                    lsfail |= fl;
                    step_inf = wave_max(tid < n ? fabs(alpha * p[tid]) : T(0));
                    __syncthreads();
                    for (int j = tid; j < n; j += NT) {
                        a[j] += alpha * p[j];
                        u[j] += alpha * Mp[j];
                    }
                    alpha_prev = alpha;
                    __syncthreads();
                }
                if (lsfail) st |= ST_LSFAIL;
                it_all += k;
                conv_all &= (st & ST_CONVERGED) != 0;
                st_all |= st & ~ST_CONVERGED;
                if (st & ST_NOTSPD) break;
                // the step's state for the backward sweep
                uint8_t *wst = g.ws + (int64_t)t * g.ws_step;
                for (int i = tid; i < m; i += NT) wst[g.mask_off + I.om + i] = A[i];
                if (!g.recompute) {
                    T *fac = reinterpret_cast<T *>(wst) + fac_offset(I);
                    for (int e = tid; e < ne; e += NT) {
                        int j, l;
                        ro_tri(e, j, l);
                        fac[e] = l < j ? H[j * n + l] : dh[j];
                    }
                }
                for (int j = tid; j < n; j += NT) vel[j] += g.h * a[j];
                __syncthreads();
            }
            const bool ok = !(st_all & (ST_NONFINITE | ST_NOTSPD));
            for (int j = tid; j < n; j += NT) g.vT[I.on + j] = ok ? vel[j] : nanv;
            if (tid == 0) {
                g.status[I.b] = st_all | (ok && conv_all ? ST_CONVERGED : 0);
                if (g.iters) g.iters[I.b] = it_all;
            }
        } else {
            // backward only: the forward call's status decides
            st_all |= g.status[I.b] & (ST_NONFINITE | ST_NOTSPD);
        }

        if (g.bwd) {
            const bool ok = !(st_all & (ST_NONFINITE | ST_NOTSPD));
            // v-bar_T: given, or the gradient of ||v_T - v_goal||^2
            for (int j = tid; j < n; j += NT)
                vb[j] = g.vbarT ? g.vbarT[I.on + j] : T(2) * (vel[j] - g.vgoal[I.on + j]);
            __syncthreads();
            for (int t = g.horizon - 1; t >= 0 && ok; --t) {
                const uint8_t *wst = g.ws + (int64_t)t * g.ws_step;
                for (int i = tid; i < m; i += NT) A[i] = wst[g.mask_off + I.om + i];
                __syncthreads();
                if (g.recompute) {
                    const int cnt = make_list();
                    __syncthreads();
                    assemble(cnt);
                    team_cholesky<NT>(H, dh, n, n, wk);   // SPD: it was factored in the forward
                } else {
                    const T *fac = reinterpret_cast<const T *>(wst) + fac_offset(I);
                    for (int e = tid; e < ne; e += NT) {
                        int j, l;
                        ro_tri(e, j, l);
                        if (l < j) H[j * n + l] = fac[e];
                        else dh[j] = fac[e];
                    }
                }
                for (int j = tid; j < n; j += NT) y[j] = g.h * vb[j];
                __syncthreads();
                team_chol_solve<NT>(H, dh, y, lam, n, n);
                for (int j = tid; j < n; j += NT)
                    g.taubar[(int64_t)t * g.tot_n + I.on + j] = lam[j];
                // s_i = D_i A_i (J lambda)_i
                for (int i = tid; i < m; i += NT) {
                    T s = T(0);
                    for (int j = 0; j < n; ++j) s += Js[i * ldj + j] * lam[j];
                    q[i] = A[i] ? Dv[i] * s : T(0);
                }
                const int cnt = make_list();
                __syncthreads();
                {
                    const int j = tid & 31;
                    const T s = jt_rows(cnt, q, j);
                    if (tid < 32 && j < n) vb[j] -= g.bdamp * s;
                }
                __syncthreads();
            }
            if (!ok)
                for (int t = tid; t < g.horizon * n; t += NT) {
                    const int tt = t / n, j = t - tt * n;
                    g.taubar[(int64_t)tt * g.tot_n + I.on + j] = nanv;
                }
            for (int j = tid; j < n; j += NT) g.v0bar[I.on + j] = ok ? vb[j] : nanv;
        }
        __syncthreads();
    }
}

inline bool rollout_supported(int nmax, int mmax, int s) {
    return nmax >= 1 && nmax <= RO_NMAX && ro_layout(nmax, mmax, s).bytes <= 160 * 1024 &&
           mmax <= 32 * RO_NT;
}

template <typename T>
int launch_rollout(const BatchView &bv, int count, int nmax, int mmax, const RolloutArgs<T> &g,
                   hipStream_t stream) {
    const size_t lds = ro_layout(nmax, mmax, (int)sizeof(T)).bytes;
    auto kern = k_rollout<T>;
    if (!ensure_lds(reinterpret_cast<const void *>(kern), lds)) return -3;
    const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(RO_NT), lds, stream, bv, count, nmax, mmax, g);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cs
