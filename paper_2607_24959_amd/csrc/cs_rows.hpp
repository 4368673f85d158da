// cs_rows.hpp -- contact solves with mixed regularised rows (Sec. III-A: the
// frictional block and the other regularised constraint rows; Sec. III-B;
// Sec. III-C, eq. 17).
//
// Row i has a kind: 0 one-sided (a pyramid edge or a limit), s = D min(r, 0)^2 / 2;
// 1 equality, s = D r^2 / 2; 2 friction loss with bound f >= 0, s = D r^2 / 2 for
// |r| <= f / D and f |r| - f^2 / (2 D) beyond (the force saturates at +-f).
// Each s_i is C^1 and piecewise quadratic, so phi'(alpha) is piecewise linear
// and the exact line search is the safeguarded piece Newton of the pyramid
// solvers with generalised piece sums.  Zone codes: 0 no force, 1 quadratic
// (w = D r, curvature D), 2 / 3 saturated at +f / -f (w = +-f, curvature 0).
//
// One wave per instance (grid-stride over the batch): J in LDS in the storage
// type, everything else in FP64.  Rows over lanes; the Newton matrix is
// M + sum over the zone-1 rows of D_i J_i^T J_i (rows listed by ballot, each
// thread's lower-triangle entries in one pass), kept while the zones are
// unchanged; J^T w over the rows with a force.  The state is the factor of H
// at the returned iterate and each row's zone code.
#pragma once

#include "cs_device.hpp"

namespace cs {

constexpr int RW_NT = 64;
constexpr int RW_NMAX = 32;

struct RwLayout {
    int ldj;
    uint32_t J, M, H, dh, vec, rows, kind, list, list2, zone, red, wk, bytes;
};

__host__ __device__ inline RwLayout rw_layout(int nmax, int mmax, int s) {
    RwLayout L;
    L.ldj = nmax | 1;
    uint32_t o = 0;
    auto take = [&o](uint64_t bytes) {
        const uint32_t r = o;
        o += (uint32_t)((bytes + 15) & ~uint64_t(15));
        return r;
    };
    const uint64_t mm = mmax > 0 ? (uint64_t)mmax : 1;
    L.J = take((uint64_t)s * mm * L.ldj);
    L.M = take(8ull * nmax * nmax);
    L.H = take(8ull * nmax * nmax);
    L.dh = take(8ull * nmax);
    L.vec = take(8ull * 8 * nmax);
    L.rows = take(8ull * 7 * mm);
    L.kind = take(mm);
    L.list = take(4ull * mm);
    L.list2 = take(4ull * mm);
    L.zone = take(mm);
    L.red = take(8ull * 16);
    L.wk = take(8ull * 16 * 17);
    L.bytes = o;
    return L;
}

__device__ inline int rw_zone(int kind, double r, double D, double f) {
    if (kind == 0) return r < 0.0 ? 1 : 0;
    if (kind == 1) return 1;
    const double d = f / D;
    return r > d ? 2 : (r < -d ? 3 : 1);
}

template <typename T>
struct RwArgs {
    const T *M, *J, *a0, *aref, *D, *fl, *ainit, *a, *abar;
    const uint8_t *kind;
    T *aout, *fac, *a0bar, *arefbar, *Jbar, *Dbar, *flbar, *Mbar;
    uint8_t *mask;
    int32_t *status, *iters;
    int max_iter;
    double tol;
};

template <typename T>
struct RwCtx {
    T *Js;
    double *Ms, *H, *dh, *vec, *r, *q, *w, *Dv, *fv, *ar, *g, *red, *wk;
    uint8_t *kind, *zone;
    int *list, *list2;
    int ldj, n, m;
};

template <typename T>
__device__ inline RwCtx<T> rw_carve(unsigned char *smem, int nmax, int mmax) {
    const RwLayout Lo = rw_layout(nmax, mmax, (int)sizeof(T));
    RwCtx<T> c;
    c.Js = reinterpret_cast<T *>(smem + Lo.J);
    c.Ms = reinterpret_cast<double *>(smem + Lo.M);
    c.H = reinterpret_cast<double *>(smem + Lo.H);
    c.dh = reinterpret_cast<double *>(smem + Lo.dh);
    c.vec = reinterpret_cast<double *>(smem + Lo.vec);
    double *rows = reinterpret_cast<double *>(smem + Lo.rows);
    const int mm = mmax > 0 ? mmax : 1;
    c.r = rows;
    c.q = rows + mm;
    c.w = rows + 2 * mm;
    c.Dv = rows + 3 * mm;
    c.fv = rows + 4 * mm;
    c.ar = rows + 5 * mm;
    c.g = rows + 6 * mm;
    c.kind = smem + Lo.kind;
    c.list = reinterpret_cast<int *>(smem + Lo.list);
    c.list2 = reinterpret_cast<int *>(smem + Lo.list2);
    c.zone = smem + Lo.zone;
    c.red = reinterpret_cast<double *>(smem + Lo.red);
    c.wk = reinterpret_cast<double *>(smem + Lo.wk);
    c.ldj = Lo.ldj;
    return c;
}

// Rows whose zone satisfies `pred`, in row order; returns their count.
template <typename T, typename P>
__device__ inline int rw_list(const RwCtx<T> &X, int *out, P pred) {
    int cnt = 0;
    for (int base = 0; base < X.m; base += RW_NT) {
        const int i = base + (int)threadIdx.x;
        const bool on = i < X.m && pred(X.zone[i]);
        const uint64_t bal = __builtin_amdgcn_ballot_w64(on);
        if (on)
            out[cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] = i;
        cnt += (int)__builtin_popcountll(bal);
    }
    return cnt;
}

// H = M + sum over the listed rows of g_i J_i^T J_i (lower triangle).
template <typename T>
__device__ inline void rw_assemble(const RwCtx<T> &X, int cnt) {
    const int n = X.n, ne = n * (n + 1) / 2, ldj = X.ldj;
    for (int e = threadIdx.x; e < ne; e += RW_NT) {
        int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        while (j * (j + 1) / 2 > e) --j;
        while ((j + 1) * (j + 2) / 2 <= e) ++j;
        const int l = e - j * (j + 1) / 2;
        double s = 0.0;
        for (int c = 0; c < cnt; ++c) {
            const int i = X.list[c];
            s += (X.g[i] * double(X.Js[i * ldj + j])) * double(X.Js[i * ldj + l]);
        }
        X.H[j * n + l] = X.Ms[j * n + l] + s;
    }
    __syncthreads();
}

// out_j = sum over the rows in `lst` (cnt of them) of J_ij x_i, the two
// half-waves taking alternate rows; valid in lanes < 32 with j < n.
template <typename T>
__device__ inline double rw_jt(const RwCtx<T> &X, const int *lst, int cnt, const double *x, int j) {
    const int half = threadIdx.x >> 5;
    double s = 0.0;
    if (j < X.n)
        for (int c = half; c < cnt; c += 2) {
            const int i = lst[c];
            s += double(X.Js[i * X.ldj + j]) * x[i];
        }
    return s + __shfl_xor(s, 32, 64);
}

template <typename T>
__device__ inline bool rw_load(const RwCtx<T> &X, const Inst &I, const RwArgs<T> &g) {
    const int n = X.n, m = X.m, tid = threadIdx.x;
    bool bad = false;
    for (int e = tid; e < m * n; e += RW_NT) {
        const int i = e / n, j = e - i * n;
        const T x = g.J[I.omn + e];
        X.Js[i * X.ldj + j] = x;
        bad |= !finite_val(x);
    }
    for (int e = tid; e < n * n; e += RW_NT) {
        const T x = g.M[I.onn + e];
        X.Ms[e] = double(x);
        bad |= !finite_val(x);
    }
    for (int i = tid; i < m; i += RW_NT) {
        const T d = g.D[I.om + i], f = g.fl[I.om + i], ar = g.aref[I.om + i];
        const uint8_t k = g.kind[I.om + i];
        X.Dv[i] = double(d);
        X.fv[i] = double(f);
        X.ar[i] = double(ar);
        X.kind[i] = k;
        bad |= !finite_val(d) || !finite_val(f) || !finite_val(ar) || k > 2 || !(d > T(0)) ||
               (k == 2 && f < T(0));
    }
    return bad;
}

template <typename T>
__global__ __launch_bounds__(RW_NT) void k_forward_rows(BatchView bv, int count, int nmax, int mmax,
                                                        RwArgs<T> g) {
    extern __shared__ __align__(16) unsigned char smem[];
    RwCtx<T> X = rw_carve<T>(smem, nmax, mmax);
    const int tid = threadIdx.x;
    double *a = X.vec, *a0 = X.vec + nmax, *F = X.vec + 2 * nmax, *p = X.vec + 3 * nmax,
           *y = X.vec + 4 * nmax, *Mp = X.vec + 5 * nmax, *md = X.vec + 6 * nmax;
    for (int wi = blockIdx.x; wi < count; wi += gridDim.x) {
        const Inst I = inst_at(bv, wi);
        if (!I.ok) {   // team-uniform
            mark_bad(I, g.status, g.iters, tid == 0);
            continue;
        }
        X.n = I.n;
        X.m = I.m;
        const int n = X.n, m = X.m, ldj = X.ldj;
        bool bad = rw_load(X, I, g);
        for (int j = tid; j < n; j += RW_NT) {
            const T x0 = g.a0[I.on + j], xi = g.ainit ? g.ainit[I.on + j] : x0;
            a0[j] = double(x0);
            a[j] = double(xi);
            bad |= !finite_val(x0) || !finite_val(xi);
        }
        for (int i = tid; i < m; i += RW_NT) X.zone[i] = 0;
        int st = __syncthreads_or(bad) ? ST_NONFINITE : 0;
        int k = 0;
        if (st == 0) {
            for (int e = tid; e < n * n; e += RW_NT) X.H[e] = X.Ms[e];
            __syncthreads();
            if (!team_cholesky<RW_NT>(X.H, X.dh, n, n, X.wk)) st = ST_NOTSPD;
        }
        if (st == 0) {
            double trM = 0.0;
            for (int j = 0; j < n; ++j) trM += X.Ms[j * n + j];
            double step_inf = -1.0;
            int lsfail = 0;
            for (k = 0;; ++k) {
                // residual, zones, w and g (eq. 6)
                bool changed = false;
                for (int i = tid; i < m; i += RW_NT) {
                    double s = 0.0;
                    for (int j = 0; j < n; ++j) s += double(X.Js[i * ldj + j]) * a[j];
                    const double ri = s - X.ar[i];
                    const int z = rw_zone(X.kind[i], ri, X.Dv[i], X.fv[i]);
                    X.r[i] = ri;
                    X.w[i] = z == 1 ? X.Dv[i] * ri : (z == 2 ? X.fv[i] : (z == 3 ? -X.fv[i] : 0.0));
                    X.g[i] = z == 1 ? X.Dv[i] : 0.0;
                    changed |= z != X.zone[i];
                    X.zone[i] = (uint8_t)z;
                }
                const bool same = !__syncthreads_or(changed) && k > 0;
                const int cq = rw_list(X, X.list, [](uint8_t z) { return z == 1; });
                const int cf = rw_list(X, X.list2, [](uint8_t z) { return z != 0; });
                __syncthreads();
                double fj = 0.0, aj = 0.0;
                {
                    const int j = tid & 31;
                    const double s = rw_jt(X, X.list2, cf, X.w, j);
                    if (tid < 32 && j < n) {
                        double d = 0.0;
                        for (int l = 0; l < n; ++l) d += X.Ms[j * n + l] * (a[l] - a0[l]);
                        md[j] = d;
                        fj = d + s;
                        F[j] = fj;
                        aj = fabs(a[j]);
                    }
                }
                // ||F||^2 and ||a||_inf by wave reductions of the lanes' entries
                const double g2 = wave_sum(fj * fj);
                const double anorm = wave_max(aj);
                __syncthreads();
                if (!same) {   // H depends on the zone-1 rows only
                    rw_assemble(X, cq);
                    if (!team_cholesky<RW_NT>(X.H, X.dh, n, n, X.wk)) { st = ST_NOTSPD; break; }
                }
                if (sqrt(g2) <= g.tol * trM ||
                    (same && step_inf >= 0.0 && step_inf <= g.tol * (1.0 + anorm))) {
                    st = ST_CONVERGED;
                    break;
                }
                if (k == g.max_iter) { st = ST_MAXITER; break; }
                for (int j = tid; j < n; j += RW_NT) y[j] = -F[j];
                __syncthreads();
                team_chol_solve<RW_NT>(X.H, X.dh, y, p, n, n);
                for (int i = tid; i < m; i += RW_NT) {
                    double s = 0.0;
                    for (int j = 0; j < n; ++j) s += double(X.Js[i * ldj + j]) * p[j];
                    X.q[i] = s;
                }
                // c0 = p^T M p, b0 = p^T M (a - a0) by wave reductions
                double pm = 0.0, pu = 0.0;
                if (tid < n) {
                    double s = 0.0;
                    for (int l = 0; l < n; ++l) s += X.Ms[tid * n + l] * p[l];
                    Mp[tid] = s;
                    pm = p[tid] * s;
                    pu = p[tid] * md[tid];
                }
                const double c0 = wave_sum(pm), b0 = wave_sum(pu);
                __syncthreads();
                // exact line search (eq. 10): phi' = c t + b on the piece of
                // trial t; a Newton point -b/c is accepted when its own piece
                // sums come out the same (equal zone sets give bitwise equal
                // sums; a different set with equal sums has the same line)
                auto piece = [&](double t, double &c, double &b) {
                    double v2[2] = {0.0, 0.0};
                    for (int i = tid; i < m; i += RW_NT) {
                        const double qi = X.q[i], ri = X.r[i];
                        const int z = rw_zone(X.kind[i], ri + t * qi, X.Dv[i], X.fv[i]);
                        if (z == 1) {
                            const double dq = X.Dv[i] * qi;
                            v2[0] += dq * qi;
                            v2[1] += dq * ri;
                        } else if (z == 2) {
                            v2[1] += X.fv[i] * qi;
                        } else if (z == 3) {
                            v2[1] -= X.fv[i] * qi;
                        }
                    }
                    team_sum<RW_NT>(v2, X.red);
                    c = c0 + v2[0];
                    b = b0 + v2[1];
                };
                double t = 1.0, c, b;
                piece(t, c, b);
                double lo = 0.0, hi = inf_val<double>();
                int fl = 1;
                for (int it = 0; it < 96; ++it) {
                    const double gp = c * t + b;
                    if (gp == 0.0) { fl = 0; break; }
                    if (gp < 0.0) lo = t; else hi = t;
                    if (hi < inf_val<double>() && hi - lo <= 32.0 * 2.220446049250313e-16 * hi) {
                        fl = 0;
                        break;
                    }
                    double cand = -b / c;
                    const bool newton = cand > lo && cand < hi;
                    if (!newton) cand = hi < inf_val<double>() ? 0.5 * (lo + hi) : 2.0 * lo + 1.0;
                    double nc, nb;
                    piece(cand, nc, nb);
                    const bool same_piece = nc == c && nb == b;
                    c = nc;
                    b = nb;
                    t = cand;
                    if (newton && same_piece) { fl = 0; break; }
                }
                lsfail |= fl;
                step_inf = wave_max(tid < n ? fabs(t * p[tid]) : 0.0);
                __syncthreads();
                for (int j = tid; j < n; j += RW_NT) a[j] += t * p[j];
                __syncthreads();
            }
            if (lsfail) st |= ST_LSFAIL;
        }
        const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
        const T nanv = T(__builtin_nan(""));
        for (int j = tid; j < n; j += RW_NT) g.aout[I.on + j] = ok ? T(a[j]) : nanv;
        T *fac = g.fac + fac_offset(I);
        for (int e = tid; e < n * (n + 1) / 2; e += RW_NT) {
            int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            while (j * (j + 1) / 2 > e) --j;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int l = e - j * (j + 1) / 2;
            fac[e] = ok ? T(l < j ? X.H[j * n + l] : X.dh[j]) : nanv;
        }
        for (int i = tid; i < m; i += RW_NT) g.mask[I.om + i] = ok ? X.zone[i] : 0;
        if (tid == 0) {
            g.status[I.b] = st;
            if (g.iters) g.iters[I.b] = k;
        }
        __syncthreads();
    }
}

// IFT VJP with mixed rows (eq. 17) at the solution the forward returned, with
// its zones and factor: lambda = H^{-1} abar (the saved factor, then two steps
// of refinement with H v = M v + J^T (g o J v) in FP64), sigma = J lambda,
//   a0bar = M^T lambda, arefbar_i = g_i sigma_i, Dbar_i = -r_i sigma_i (zone 1),
//   fbar_i = -+sigma_i (zones 2 / 3), Jbar = -(w lambda^T + arefbar a^T),
//   Mbar = -lambda (a - a0)^T.
template <typename T>
__global__ __launch_bounds__(RW_NT) void k_ift_vjp_rows(BatchView bv, int count, int nmax, int mmax,
                                                        RwArgs<T> g) {
    extern __shared__ __align__(16) unsigned char smem[];
    RwCtx<T> X = rw_carve<T>(smem, nmax, mmax);
    const int tid = threadIdx.x;
    double *a = X.vec, *a0 = X.vec + nmax, *lam = X.vec + 2 * nmax, *y = X.vec + 3 * nmax,
           *x = X.vec + 4 * nmax, *v = X.vec + 5 * nmax;
    for (int wi = blockIdx.x; wi < count; wi += gridDim.x) {
        const Inst I = inst_at(bv, wi);
        if (!I.ok) continue;   // team-uniform: outputs untouched
        X.n = I.n;
        X.m = I.m;
        const int n = X.n, m = X.m, ldj = X.ldj;
        rw_load(X, I, g);
        for (int j = tid; j < n; j += RW_NT) {
            a[j] = double(g.a[I.on + j]);
            a0[j] = double(g.a0[I.on + j]);
        }
        const T *fac = g.fac + fac_offset(I);
        for (int e = tid; e < n * (n + 1) / 2; e += RW_NT) {
            int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            while (j * (j + 1) / 2 > e) --j;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int l = e - j * (j + 1) / 2;
            if (l < j) X.H[j * n + l] = double(fac[e]);
            else X.dh[j] = double(fac[e]);
        }
        __syncthreads();
        for (int i = tid; i < m; i += RW_NT) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += double(X.Js[i * ldj + j]) * a[j];
            const double ri = s - X.ar[i];
            const int z = g.mask[I.om + i];
            X.zone[i] = (uint8_t)z;
            X.r[i] = ri;
            X.w[i] = z == 1 ? X.Dv[i] * ri : (z == 2 ? X.fv[i] : (z == 3 ? -X.fv[i] : 0.0));
            X.g[i] = z == 1 ? X.Dv[i] : 0.0;
        }
        __syncthreads();
        const int cq = rw_list(X, X.list, [](uint8_t z) { return z == 1; });
        __syncthreads();
        // out = H v = M v + J^T (g o J v); leaves J v in q and g o J v in ar (aref
        // is not needed past the residual above)
        auto hv = [&](const double *vin, double *out) {
            for (int i = tid; i < m; i += RW_NT) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += double(X.Js[i * ldj + j]) * vin[j];
                X.q[i] = s;
            }
            __syncthreads();
            for (int i = tid; i < m; i += RW_NT) X.ar[i] = X.g[i] * X.q[i];
            __syncthreads();
            const int j = tid & 31;
            const double s = rw_jt(X, X.list, cq, X.ar, j);
            if (tid < 32 && j < n) {
                double d = 0.0;
                for (int l = 0; l < n; ++l) d += X.Ms[j * n + l] * vin[l];
                out[j] = d + s;
            }
            __syncthreads();
        };
        for (int j = tid; j < n; j += RW_NT) y[j] = double(g.abar[I.on + j]);
        __syncthreads();
        team_chol_solve<RW_NT>(X.H, X.dh, y, lam, n, n);
        for (int it = 0; it < 2; ++it) {
            hv(lam, v);
            for (int j = tid; j < n; j += RW_NT) y[j] = double(g.abar[I.on + j]) - v[j];
            __syncthreads();
            team_chol_solve<RW_NT>(X.H, X.dh, y, x, n, n);
            for (int j = tid; j < n; j += RW_NT) lam[j] += x[j];
            __syncthreads();
        }
        hv(lam, v);   // q = sigma = J lambda, ar = g o sigma = arefbar
        if (g.a0bar)
            for (int j = tid; j < n; j += RW_NT) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += X.Ms[l * n + j] * lam[l];
                g.a0bar[I.on + j] = T(s);
            }
        for (int i = tid; i < m; i += RW_NT) {
            const int z = X.zone[i];
            if (g.arefbar) g.arefbar[I.om + i] = T(X.ar[i]);
            if (g.Dbar) g.Dbar[I.om + i] = T(z == 1 ? -X.r[i] * X.q[i] : 0.0);
            if (g.flbar) g.flbar[I.om + i] = T(z == 2 ? -X.q[i] : (z == 3 ? X.q[i] : 0.0));
        }
        if (g.Jbar)
            for (int e = tid; e < m * n; e += RW_NT) {
                const int i = e / n, j = e - i * n;
                g.Jbar[I.omn + e] = T(-(X.w[i] * lam[j] + X.ar[i] * a[j]));
            }
        if (g.Mbar)
            for (int e = tid; e < n * n; e += RW_NT) {
                const int j = e / n, l = e - j * n;
                g.Mbar[I.onn + e] = T(-lam[j] * (a[l] - a0[l]));
            }
        __syncthreads();
    }
}

inline bool rows_supported(int nmax, int mmax, int s) {
    return nmax >= 1 && nmax <= RW_NMAX && mmax <= 32 * RW_NT &&
           rw_layout(nmax, mmax, s).bytes <= 160 * 1024;
}

template <typename T>
int launch_rows(bool vjp, const BatchView &bv, int count, int nmax, int mmax, const RwArgs<T> &g,
                hipStream_t stream) {
    const size_t lds = rw_layout(nmax, mmax, (int)sizeof(T)).bytes;
    auto kern = vjp ? k_ift_vjp_rows<T> : k_forward_rows<T>;
    if (!ensure_lds(reinterpret_cast<const void *>(kern), lds)) return -3;
    const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(RW_NT), lds, stream, bv, count, nmax, mmax, g);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cs
