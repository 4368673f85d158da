// cs_ell.hpp -- contact solves with the round (elliptic) Coulomb cone
// (Sec. III-A, eqs. 2, 3, 5; Sec. III-B; Sec. III-C, eq. 17).
//
// Contact c owns rows 3c (normal) and 3c+1, 3c+2 (tangential) of J and aref,
// regularisation weights R^{-1} = diag(dn_c, dt_c, dt_c) and friction mu_c.
// Its share of the reduced objective is the weighted squared distance of
// u_c = J_c a - aref_c to the dual cone K* = {z_N >= mu |z_T|}.  In the scaled
// coordinates x = (sqrt(dn) u_N, sqrt(dt) u_T) that is the Euclidean distance
// to the second-order cone {x_N >= mh |x_T|}, mh = mu sqrt(dn / dt), with three
// zones (nn = x_N, t = |x_T|):
//   0: nn >= mh t (inside)       s = 0
//   2: mh nn + t <= 0 (polar)     s = (nn^2 + t^2) / 2
//   1: otherwise                  s = (mh t - nn)^2 / (2 (1 + mh^2)).
// The gradient w_c = ds/du_c and the 3 x 3 Hessian block G_c follow in closed
// form; F = M (a - a0) + J^T w (eq. 6) and H = M + sum_c J_c^T G_c J_c (eq. 9).
// phi(alpha) = L(a + alpha p) is convex and C^1 but not piecewise quadratic, so
// the exact line search finds the root of phi' by Newton steps kept inside a
// bracket.
//
// One wave per instance (grid-stride over the batch): J in LDS in the storage
// type, every other quantity and every sum in FP64 (FP32 storage changes only
// what is read and written).  Contacts are distributed over the lanes; the
// Newton matrix is M + J_A^T K with K = G J formed for the contacts off zone
// 0 (listed by ballot), then the one-wave team Cholesky and solves.  The
// state is the packed factor of H at the returned iterate and each contact's
// zone (in the byte of its normal row; the tangential rows' bytes are 0).
#pragma once

#include "cs_device.hpp"

namespace cs {

constexpr int EL_NT = 64;
constexpr int EL_NMAX = 32;

struct ElLayout {
    int ldj;
    uint32_t J, M, H, dh, vec, rows, K, con, pre, G, list, zone, red, wk, bytes;
};

__host__ __device__ inline ElLayout el_layout(int nmax, int mmax, int s) {
    ElLayout L;
    L.ldj = nmax | 1;
    uint32_t o = 0;
    auto take = [&o](uint64_t bytes) {
        const uint32_t r = o;
        o += (uint32_t)((bytes + 15) & ~uint64_t(15));
        return r;
    };
    const uint64_t mm = mmax > 0 ? (uint64_t)mmax : 3, nc = mm / 3 > 0 ? mm / 3 : 1;
    L.J = take((uint64_t)s * mm * L.ldj);
    L.M = take(8ull * nmax * nmax);
    L.H = take(8ull * nmax * nmax);
    L.dh = take(8ull * nmax);
    L.vec = take(8ull * 8 * nmax);
    L.rows = take(8ull * 4 * mm);
    L.K = take(8ull * mm * nmax);
    L.con = take(8ull * 3 * nc);
    L.pre = take(8ull * 4 * nc);
    L.G = take(8ull * 6 * nc);
    L.list = take(4ull * nc);
    L.zone = take(nc);
    L.red = take(8ull * 16);
    L.wk = take(8ull * 16 * 17);
    L.bytes = o;
    return L;
}

// A contact's constants: sqrt(dn), sqrt(dt), mh = mu sqrt(dn / dt) and
// 1 / (1 + mh^2), formed once per solve.
struct ElCon {
    double sn, st, mh, ik;
};

__device__ inline ElCon el_con(double dn, double dt, double mu) {
    ElCon k;
    k.sn = sqrt(dn);
    k.st = sqrt(dt);
    k.mh = mu * k.sn / k.st;
    k.ik = 1.0 / (1.0 + k.mh * k.mh);
    return k;
}

// One contact: zone, w = ds/du (3) and G (upper triangle 00 01 02 11 12 22).
// `force_zone` >= 0 evaluates that zone's formulas instead of classifying.
__device__ inline int el_block(const double (&u)[3], const ElCon &K, double (&w)[3],
                               double (&G)[6], int force_zone = -1) {
    const double sn = K.sn, st = K.st, mh = K.mh;
    const double nn = sn * u[0], x1 = st * u[1], x2 = st * u[2];
    const double t = sqrt(x1 * x1 + x2 * x2);
    int zone = force_zone;
    if (zone < 0) zone = nn >= mh * t ? 0 : (mh * nn + t <= 0.0 ? 2 : 1);
    double g0 = 0, g1 = 0, g2 = 0, h00 = 0, h01 = 0, h02 = 0, h11 = 0, h12 = 0, h22 = 0;
    if (zone == 2) {
        g0 = nn;
        g1 = x1;
        g2 = x2;
        h00 = h11 = h22 = 1.0;
    } else if (zone == 1 && t > 0.0) {
        const double ik = K.ik, h = mh * t - nn, it = 1.0 / t;
        const double t1 = x1 * it, t2 = x2 * it;
        const double e0 = -1.0, e1 = mh * t1, e2 = mh * t2;
        g0 = h * ik * e0;
        g1 = h * ik * e1;
        g2 = h * ik * e2;
        const double c = h * mh * ik * it;
        h00 = e0 * e0 * ik;
        h01 = e0 * e1 * ik;
        h02 = e0 * e2 * ik;
        h11 = e1 * e1 * ik + c * (1.0 - t1 * t1);
        h12 = e1 * e2 * ik - c * t1 * t2;
        h22 = e2 * e2 * ik + c * (1.0 - t2 * t2);
    }
    w[0] = sn * g0;
    w[1] = st * g1;
    w[2] = st * g2;
    G[0] = sn * h00 * sn;
    G[1] = sn * h01 * st;
    G[2] = sn * h02 * st;
    G[3] = st * h11 * st;
    G[4] = st * h12 * st;
    G[5] = st * h22 * st;
    return zone;
}

// Entry (r, q) of a block stored as its upper triangle 00 01 02 11 12 22.
__device__ inline double el_g(const double *G6, int r, int q) {
    const int i = r < q ? r : q, j = r < q ? q : r;
    return G6[i == 0 ? j : (i == 1 ? j + 2 : 5)];
}

template <typename T>
struct ElArgs {
    const T *M, *J, *a0, *aref, *dn, *dt, *mu, *ainit, *a, *abar;
    T *aout, *fac, *a0bar, *arefbar, *Jbar, *dnbar, *dtbar, *mubar, *Mbar;
    uint8_t *mask;
    int32_t *status, *iters;
    int max_iter;
    double tol;
};

// Shared per-instance context of the two kernels.
template <typename T>
struct ElCtx {
    T *Js;
    double *Ms, *H, *dh, *vec, *rows, *K, *con, *G, *red, *wk;
    ElCon *pre;
    int *list;
    uint8_t *zone;
    int ldj, n, m, nc;
};

template <typename T>
__device__ inline ElCtx<T> el_carve(unsigned char *smem, int nmax, int mmax) {
    const ElLayout Lo = el_layout(nmax, mmax, (int)sizeof(T));
    ElCtx<T> c;
    c.Js = reinterpret_cast<T *>(smem + Lo.J);
    c.Ms = reinterpret_cast<double *>(smem + Lo.M);
    c.H = reinterpret_cast<double *>(smem + Lo.H);
    c.dh = reinterpret_cast<double *>(smem + Lo.dh);
    c.vec = reinterpret_cast<double *>(smem + Lo.vec);
    c.rows = reinterpret_cast<double *>(smem + Lo.rows);
    c.K = reinterpret_cast<double *>(smem + Lo.K);
    c.con = reinterpret_cast<double *>(smem + Lo.con);
    c.pre = reinterpret_cast<ElCon *>(smem + Lo.pre);
    c.G = reinterpret_cast<double *>(smem + Lo.G);
    c.list = reinterpret_cast<int *>(smem + Lo.list);
    c.zone = smem + Lo.zone;
    c.red = reinterpret_cast<double *>(smem + Lo.red);
    c.wk = reinterpret_cast<double *>(smem + Lo.wk);
    c.ldj = Lo.ldj;
    return c;
}

// Contacts off zone 0, in contact order; returns their count.
template <typename T>
__device__ inline int el_list(const ElCtx<T> &X) {
    int cnt = 0;
    for (int base = 0; base < X.nc; base += EL_NT) {
        const int c = base + (int)threadIdx.x;
        const bool on = c < X.nc && X.zone[c] != 0;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(on);
        if (on)
            X.list[cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] = c;
        cnt += (int)__builtin_popcountll(bal);
    }
    return cnt;
}

// H = M + sum over the listed contacts of J_c^T G_c J_c: K = G J first (rows
// of the listed contacts), then each thread's lower-triangle entries.
template <typename T>
__device__ inline void el_assemble(const ElCtx<T> &X, int cnt) {
    const int n = X.n, tid = threadIdx.x, ldj = X.ldj;
    for (int e = tid; e < 3 * cnt * n; e += EL_NT) {
        const int ci = e / (3 * n), rem = e - ci * 3 * n, r = rem / n, l = rem - r * n;
        const int c = X.list[ci];
        const double *G6 = X.G + 6 * c;
        const T *Jc = X.Js + 3 * c * ldj;
        X.K[(3 * c + r) * n + l] = el_g(G6, r, 0) * double(Jc[l]) + el_g(G6, r, 1) * double(Jc[ldj + l]) +
                                   el_g(G6, r, 2) * double(Jc[2 * ldj + l]);
    }
    __syncthreads();
    const int ne = n * (n + 1) / 2;
    for (int e = tid; e < ne; e += EL_NT) {
        int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        while (j * (j + 1) / 2 > e) --j;
        while ((j + 1) * (j + 2) / 2 <= e) ++j;
        const int l = e - j * (j + 1) / 2;
        double s = 0.0;
        for (int ci = 0; ci < cnt; ++ci) {
            const int c = X.list[ci];
#pragma unroll
            for (int r = 0; r < 3; ++r)
                s += double(X.Js[(3 * c + r) * ldj + j]) * X.K[(3 * c + r) * n + l];
        }
        X.H[j * n + l] = X.Ms[j * n + l] + s;
    }
    __syncthreads();
}

// Load J (storage type), M (FP64 copy), and the contact parameters; returns
// whether any of them is not finite.
template <typename T>
__device__ inline bool el_load(const ElCtx<T> &X, const Inst &I, const T *gM, const T *gJ,
                               const T *gdn, const T *gdt, const T *gmu) {
    const int n = X.n, m = X.m, tid = threadIdx.x;
    bool bad = false;
    for (int e = tid; e < m * n; e += EL_NT) {
        const int i = e / n, j = e - i * n;
        const T x = gJ[I.omn + e];
        X.Js[i * X.ldj + j] = x;
        bad |= !finite_val(x);
    }
    for (int e = tid; e < n * n; e += EL_NT) {
        const T x = gM[I.onn + e];
        X.Ms[e] = double(x);
        bad |= !finite_val(x);
    }
    const int64_t oc = I.om / 3;
    for (int c = tid; c < X.nc; c += EL_NT) {
        const T d1 = gdn[oc + c], d2 = gdt[oc + c], f = gmu[oc + c];
        X.con[3 * c] = double(d1);
        X.con[3 * c + 1] = double(d2);
        X.con[3 * c + 2] = double(f);
        X.pre[c] = el_con(double(d1), double(d2), double(f));
        bad |= !finite_val(d1) || !finite_val(d2) || !finite_val(f) || !(d1 > T(0)) ||
               !(d2 > T(0)) || f < T(0);
    }
    return bad;
}

template <typename T>
__global__ __launch_bounds__(EL_NT) void k_forward_ell(BatchView bv, int count, int nmax, int mmax,
                                                       ElArgs<T> g) {
    extern __shared__ __align__(16) unsigned char smem[];
    ElCtx<T> X = el_carve<T>(smem, nmax, mmax);
    const int tid = threadIdx.x;
    double *a = X.vec, *a0 = X.vec + nmax, *F = X.vec + 2 * nmax, *p = X.vec + 3 * nmax,
           *y = X.vec + 4 * nmax, *Mp = X.vec + 5 * nmax, *md = X.vec + 6 * nmax;
    double *u = X.rows, *q = X.rows + mmax, *w = X.rows + 2 * mmax, *ar = X.rows + 3 * mmax;
    for (int wi = blockIdx.x; wi < count; wi += gridDim.x) {
        const Inst I = inst_at(bv, wi);
        const bool shape_ok = I.ok && I.m % 3 == 0;
        if (!shape_ok) {   // team-uniform
            mark_bad(I, g.status, g.iters, tid == 0);
            continue;
        }
        X.n = I.n;
        X.m = I.m;
        X.nc = I.m / 3;
        const int n = X.n, m = X.m, nc = X.nc, ldj = X.ldj;
        bool bad = el_load(X, I, g.M, g.J, g.dn, g.dt, g.mu);
        for (int j = tid; j < n; j += EL_NT) {
            const T x0 = g.a0[I.on + j], xi = g.ainit ? g.ainit[I.on + j] : x0;
            a0[j] = double(x0);
            a[j] = double(xi);
            bad |= !finite_val(x0) || !finite_val(xi);
        }
        for (int i = tid; i < m; i += EL_NT) {
            const T x = g.aref[I.om + i];
            ar[i] = double(x);
            bad |= !finite_val(x);
        }
        for (int c = tid; c < nc; c += EL_NT) X.zone[c] = 0;
        int st = __syncthreads_or(bad) ? ST_NONFINITE : 0;
        int k = 0;
        if (st == 0) {
            // M must be positive definite: factor a copy
            for (int e = tid; e < n * n; e += EL_NT) X.H[e] = X.Ms[e];
            __syncthreads();
            if (!team_cholesky<EL_NT>(X.H, X.dh, n, n, X.wk)) st = ST_NOTSPD;
        }
        if (st == 0) {
            double trM = 0.0;
            for (int j = 0; j < n; ++j) trM += X.Ms[j * n + j];
            double step_inf = -1.0, step_prev = 0.0;
            int lsfail = 0;
            for (k = 0;; ++k) {
                // u = J a - aref (formed at the first step, then carried,
                // u <- u + t J p with the previous step's q = J p); per
                // contact: zone, w, G
                for (int i = tid; i < m; i += EL_NT) {
                    if (k == 0) {
                        double s = 0.0;
                        for (int j = 0; j < n; ++j) s += double(X.Js[i * ldj + j]) * a[j];
                        u[i] = s - ar[i];
                    } else {
                        u[i] += step_prev * q[i];
                    }
                }
                __syncthreads();
                bool changed = false;
                for (int c = tid; c < nc; c += EL_NT) {
                    const double uc[3] = {u[3 * c], u[3 * c + 1], u[3 * c + 2]};
                    double wc[3], Gc[6];
                    const int z = el_block(uc, X.pre[c], wc, Gc);
                    changed |= z != X.zone[c];
                    X.zone[c] = (uint8_t)z;
                    w[3 * c] = wc[0];
                    w[3 * c + 1] = wc[1];
                    w[3 * c + 2] = wc[2];
#pragma unroll
                    for (int e = 0; e < 6; ++e) X.G[6 * c + e] = Gc[e];
                }
                const bool same = !__syncthreads_or(changed) && k > 0;
                const int cnt = el_list(X);
                __syncthreads();
                // F = M (a - a0) + J^T w over the listed contacts' rows
                double fj = 0.0, aj = 0.0;
                {
                    const int j = tid & 31, half = tid >> 5;
                    double s = 0.0;
                    if (j < n)
                        for (int ci = half; ci < cnt; ci += 2) {
                            const int c = X.list[ci];
#pragma unroll
                            for (int r = 0; r < 3; ++r) s += double(X.Js[(3 * c + r) * ldj + j]) * w[3 * c + r];
                        }
                    s += __shfl_xor(s, 32, 64);
                    if (tid < 32 && j < n) {
                        // M (a - a0): formed at the first step, then carried
                        double d = md[j];
                        if (k == 0) {
                            d = 0.0;
                            for (int l = 0; l < n; ++l) d += X.Ms[j * n + l] * (a[l] - a0[l]);
                        }
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
                if (!same) {   // H depends on the zones' blocks: rebuild unless unchanged
                    el_assemble(X, cnt);
                    if (!team_cholesky<EL_NT>(X.H, X.dh, n, n, X.wk)) { st = ST_NOTSPD; break; }
                } else {
                    // same zones but G depends on u within zone 1: rebuild when any
                    // listed contact is in zone 1
                    bool z1 = false;
                    for (int ci = 0; ci < cnt; ++ci) z1 |= X.zone[X.list[ci]] == 1;
                    if (z1) {
                        el_assemble(X, cnt);
                        if (!team_cholesky<EL_NT>(X.H, X.dh, n, n, X.wk)) { st = ST_NOTSPD; break; }
                    }
                }
                if (sqrt(g2) <= g.tol * trM ||
                    (same && step_inf >= 0.0 && step_inf <= g.tol * (1.0 + anorm))) {
                    st = ST_CONVERGED;
                    break;
                }
                if (k == g.max_iter) { st = ST_MAXITER; break; }
                for (int j = tid; j < n; j += EL_NT) y[j] = -F[j];
                __syncthreads();
                team_chol_solve<EL_NT>(X.H, X.dh, y, p, n, n);
                for (int i = tid; i < m; i += EL_NT) {
                    double s = 0.0;
                    for (int j = 0; j < n; ++j) s += double(X.Js[i * ldj + j]) * p[j];
                    q[i] = s;
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
                // exact line search: the root of phi' (the rule of the oracle's
                // line search): Newton steps while no upper end is known, then
                // Newton steps inside the bracket that at least halve the step
                // before last, else a secant step on the bracket, else (the
                // bracket not halved in two evaluations, or the secant point
                // outside) bisection
                double glo;
                {
                    double v1[1] = {0.0};
                    for (int i = tid; i < m; i += EL_NT) v1[0] += w[i] * q[i];
                    team_sum<EL_NT>(v1, X.red);
                    glo = b0 + v1[0];
                }
                double lo = 0.0, hi = -1.0, ghi = 0.0, al = 1.0, best = 1.0,
                       dxold = inf_val<double>(), dx = inf_val<double>(),
                       wid1 = inf_val<double>(), wid2 = inf_val<double>();
                int fl = 1;
                for (int it = 0; it < 100; ++it) {
                    double v3[3] = {0.0, 0.0, 0.0};
                    for (int c = tid; c < nc; c += EL_NT) {
                        const double uc[3] = {u[3 * c] + al * q[3 * c], u[3 * c + 1] + al * q[3 * c + 1],
                                              u[3 * c + 2] + al * q[3 * c + 2]};
                        double wc[3], Gc[6];
                        el_block(uc, X.pre[c], wc, Gc);
                        const double q0 = q[3 * c], q1 = q[3 * c + 1], q2 = q[3 * c + 2];
                        const double wq = wc[0] * q0 + wc[1] * q1 + wc[2] * q2;
                        v3[0] += wq;
                        v3[1] += q0 * (Gc[0] * q0 + Gc[1] * q1 + Gc[2] * q2) +
                                 q1 * (Gc[1] * q0 + Gc[3] * q1 + Gc[4] * q2) +
                                 q2 * (Gc[2] * q0 + Gc[4] * q1 + Gc[5] * q2);
                        v3[2] += fabs(wq);
                    }
                    team_sum<EL_NT>(v3, X.red);
                    const double gv = c0 * al + b0 + v3[0], hv = c0 + v3[1];
                    const double sabs = fabs(c0 * al) + fabs(b0) + v3[2];
                    best = al;
                    if (gv == 0.0) { fl = 0; break; }
                    if (gv < 0.0) { lo = al; glo = gv; } else { hi = al; ghi = gv; }
                    if (fabs(gv) <= 1e-13 * sabs) { fl = 0; break; }
                    double nx = al - gv / hv;
                    if (hi < 0.0) {
                        if (!(nx > al)) nx = 2.0 * al;
                    } else {
                        const double wid = hi - lo;
                        if (wid <= 4e-16 * hi) { fl = 0; break; }
                        const bool slow = wid > 0.5 * wid2;
                        wid2 = wid1;
                        wid1 = wid;
                        if (!(nx > lo && nx < hi && fabs(nx - al) < 0.5 * fabs(dxold))) {
                            nx = lo - glo * (hi - lo) / (ghi - glo);
                            if (slow || !(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
                        }
                    }
                    dxold = dx;
                    dx = nx - al;
                    if (nx == al) { fl = 0; break; }
                    al = nx;
                }
                lsfail |= fl;
                step_inf = wave_max(tid < n ? fabs(best * p[tid]) : 0.0);
                __syncthreads();
                for (int j = tid; j < n; j += EL_NT) {
                    a[j] += best * p[j];
                    md[j] += best * Mp[j];
                }
                step_prev = best;
                __syncthreads();
            }
            if (lsfail) st |= ST_LSFAIL;
        }
        const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
        const T nanv = T(__builtin_nan(""));
        for (int j = tid; j < n; j += EL_NT) g.aout[I.on + j] = ok ? T(a[j]) : nanv;
        T *fac = g.fac + fac_offset(I);
        for (int e = tid; e < n * (n + 1) / 2; e += EL_NT) {
            int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            while (j * (j + 1) / 2 > e) --j;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int l = e - j * (j + 1) / 2;
            fac[e] = ok ? T(l < j ? X.H[j * n + l] : X.dh[j]) : nanv;
        }
        for (int i = tid; i < m; i += EL_NT)
            g.mask[I.om + i] = (ok && i % 3 == 0) ? X.zone[i / 3] : 0;
        if (tid == 0) {
            g.status[I.b] = st;
            if (g.iters) g.iters[I.b] = k;
        }
        __syncthreads();
    }
}

// IFT VJP with the round cone (eq. 17) at the solution the forward returned,
// with its zones and factor: lambda = H^{-1} abar (the saved factor, then two
// steps of refinement with H v = M v + J^T (G (J v)) in FP64), sigma = J lambda,
//   a0bar = M^T lambda, arefbar_c = G_c sigma_c, Jbar = -(w lambda^T + arefbar a^T),
//   Mbar = -lambda (a - a0)^T, and per contact (dn, dt, mu)bar = -sigma_c . dw_c/dtheta
// at fixed u_c (w_c = S g(S u_c, mh), S = diag(sqrt dn, sqrt dt, sqrt dt),
// mh = mu sqrt(dn / dt)).
template <typename T>
__global__ __launch_bounds__(EL_NT) void k_ift_vjp_ell(BatchView bv, int count, int nmax, int mmax,
                                                       ElArgs<T> g) {
    extern __shared__ __align__(16) unsigned char smem[];
    ElCtx<T> X = el_carve<T>(smem, nmax, mmax);
    const int tid = threadIdx.x;
    double *a = X.vec, *a0 = X.vec + nmax, *lam = X.vec + 2 * nmax, *y = X.vec + 3 * nmax,
           *x = X.vec + 4 * nmax, *v = X.vec + 5 * nmax;
    double *u = X.rows, *sg = X.rows + mmax, *w = X.rows + 2 * mmax, *ab = X.rows + 3 * mmax;
    for (int wi = blockIdx.x; wi < count; wi += gridDim.x) {
        const Inst I = inst_at(bv, wi);
        if (!I.ok || I.m % 3 != 0) continue;   // team-uniform: outputs untouched
        X.n = I.n;
        X.m = I.m;
        X.nc = I.m / 3;
        const int n = X.n, m = X.m, nc = X.nc, ldj = X.ldj;
        el_load(X, I, g.M, g.J, g.dn, g.dt, g.mu);
        for (int j = tid; j < n; j += EL_NT) {
            a[j] = double(g.a[I.on + j]);
            a0[j] = double(g.a0[I.on + j]);
        }
        const T *fac = g.fac + fac_offset(I);
        for (int e = tid; e < n * (n + 1) / 2; e += EL_NT) {
            int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            while (j * (j + 1) / 2 > e) --j;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int l = e - j * (j + 1) / 2;
            if (l < j) X.H[j * n + l] = double(fac[e]);
            else X.dh[j] = double(fac[e]);
        }
        for (int c = tid; c < nc; c += EL_NT) X.zone[c] = g.mask[I.om + 3 * c];
        __syncthreads();
        for (int i = tid; i < m; i += EL_NT) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += double(X.Js[i * ldj + j]) * a[j];
            u[i] = s - double(g.aref[I.om + i]);
        }
        __syncthreads();
        for (int c = tid; c < nc; c += EL_NT) {
            const double uc[3] = {u[3 * c], u[3 * c + 1], u[3 * c + 2]};
            double wc[3], Gc[6];
            el_block(uc, X.pre[c], wc, Gc, X.zone[c]);
            w[3 * c] = wc[0];
            w[3 * c + 1] = wc[1];
            w[3 * c + 2] = wc[2];
#pragma unroll
            for (int e = 0; e < 6; ++e) X.G[6 * c + e] = Gc[e];
        }
        const int cnt = el_list(X);
        __syncthreads();
        // H v = M v + J^T (G (J v)) over the listed contacts, into `out`
        auto hv = [&](const double *vin, double *out) {
            for (int i = tid; i < m; i += EL_NT) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += double(X.Js[i * ldj + j]) * vin[j];
                sg[i] = s;
            }
            __syncthreads();
            for (int c = tid; c < nc; c += EL_NT) {
                const double *G6 = X.G + 6 * c;
                const double s0 = sg[3 * c], s1 = sg[3 * c + 1], s2 = sg[3 * c + 2];
                ab[3 * c] = G6[0] * s0 + G6[1] * s1 + G6[2] * s2;
                ab[3 * c + 1] = G6[1] * s0 + G6[3] * s1 + G6[4] * s2;
                ab[3 * c + 2] = G6[2] * s0 + G6[4] * s1 + G6[5] * s2;
            }
            __syncthreads();
            const int j = tid & 31, half = tid >> 5;
            double s = 0.0;
            if (j < n)
                for (int ci = half; ci < cnt; ci += 2) {
                    const int c = X.list[ci];
#pragma unroll
                    for (int r = 0; r < 3; ++r) s += double(X.Js[(3 * c + r) * ldj + j]) * ab[3 * c + r];
                }
            s += __shfl_xor(s, 32, 64);
            if (tid < 32 && j < n) {
                double d = 0.0;
                for (int l = 0; l < n; ++l) d += X.Ms[j * n + l] * vin[l];
                out[j] = d + s;
            }
            __syncthreads();
        };
        for (int j = tid; j < n; j += EL_NT) y[j] = double(g.abar[I.on + j]);
        __syncthreads();
        team_chol_solve<EL_NT>(X.H, X.dh, y, lam, n, n);
        for (int it = 0; it < 2; ++it) {
            hv(lam, v);
            for (int j = tid; j < n; j += EL_NT) y[j] = double(g.abar[I.on + j]) - v[j];
            __syncthreads();
            team_chol_solve<EL_NT>(X.H, X.dh, y, x, n, n);
            for (int j = tid; j < n; j += EL_NT) lam[j] += x[j];
            __syncthreads();
        }
        // sigma = J lambda and arefbar = G sigma (left in sg and ab by hv)
        hv(lam, v);
        if (g.a0bar)
            for (int j = tid; j < n; j += EL_NT) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += X.Ms[l * n + j] * lam[l];
                g.a0bar[I.on + j] = T(s);
            }
        if (g.arefbar)
            for (int i = tid; i < m; i += EL_NT) g.arefbar[I.om + i] = T(ab[i]);
        if (g.Jbar)
            for (int e = tid; e < m * n; e += EL_NT) {
                const int i = e / n, j = e - i * n;
                g.Jbar[I.omn + e] = T(-(w[i] * lam[j] + ab[i] * a[j]));
            }
        if (g.Mbar)
            for (int e = tid; e < n * n; e += EL_NT) {
                const int j = e / n, l = e - j * n;
                g.Mbar[I.onn + e] = T(-lam[j] * (a[l] - a0[l]));
            }
        const int64_t oc = I.om / 3;
        for (int c = tid; c < nc; c += EL_NT) {
            const double dn = X.con[3 * c], dt = X.con[3 * c + 1], mu = X.con[3 * c + 2];
            const double sn = sqrt(dn), st = sqrt(dt), mh = mu * sn / st;
            const double uc[3] = {u[3 * c], u[3 * c + 1], u[3 * c + 2]};
            const double S[3] = {sn, st, st};
            const double xs[3] = {sn * uc[0], st * uc[1], st * uc[2]};
            const double *G6 = X.G + 6 * c;
            double gh[3], dgm[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < 3; ++i) gh[i] = w[3 * c + i] / S[i];
            if (X.zone[c] == 1) {
                const double t = sqrt(xs[1] * xs[1] + xs[2] * xs[2]);
                if (t > 0.0) {
                    const double k = 1.0 + mh * mh, h = mh * t - xs[0];
                    const double e[3] = {-1.0, mh * xs[1] / t, mh * xs[2] / t};
                    const double f = t / k - 2.0 * mh * h / (k * k);
                    dgm[0] = f * e[0];
                    dgm[1] = f * e[1] + h / k * xs[1] / t;
                    dgm[2] = f * e[2] + h / k * xs[2] / t;
                }
            }
            const double dS[3][3] = {{0.5 / sn, 0.0, 0.0}, {0.0, 0.5 / st, 0.5 / st}, {0.0, 0.0, 0.0}};
            const double dmh[3] = {mu / (2.0 * sn * st), -mu * sn / (2.0 * st * st * st), sn / st};
            double outv[3];
            for (int th = 0; th < 3; ++th) {
                double dx[3], dw[3];
                for (int i = 0; i < 3; ++i) dx[i] = dS[th][i] * uc[i];
                for (int i = 0; i < 3; ++i) {
                    // Ghat = S^{-1} G S^{-1}
                    double s = 0.0;
                    for (int j = 0; j < 3; ++j) s += el_g(G6, i, j) / (S[i] * S[j]) * dx[j];
                    dw[i] = dS[th][i] * gh[i] + S[i] * (s + dgm[i] * dmh[th]);
                }
                outv[th] = -(sg[3 * c] * dw[0] + sg[3 * c + 1] * dw[1] + sg[3 * c + 2] * dw[2]);
            }
            if (g.dnbar) g.dnbar[oc + c] = T(outv[0]);
            if (g.dtbar) g.dtbar[oc + c] = T(outv[1]);
            if (g.mubar) g.mubar[oc + c] = T(outv[2]);
        }
        __syncthreads();
    }
}

inline bool ell_supported(int nmax, int mmax, int s) {
    return nmax >= 1 && nmax <= EL_NMAX && el_layout(nmax, mmax, s).bytes <= 160 * 1024;
}

template <typename T>
int launch_ell(bool vjp, const BatchView &bv, int count, int nmax, int mmax, const ElArgs<T> &g,
               hipStream_t stream) {
    const size_t lds = el_layout(nmax, mmax, (int)sizeof(T)).bytes;
    auto kern = vjp ? k_ift_vjp_ell<T> : k_forward_ell<T>;
    if (!ensure_lds(reinterpret_cast<const void *>(kern), lds)) return -3;
    const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(EL_NT), lds, stream, bv, count, nmax, mmax, g);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cs
