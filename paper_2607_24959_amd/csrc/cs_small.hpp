// cs_small.hpp -- register-resident kernels for small instances.
//
// Mapping: a group of 16 lanes (one DPP row) owns one instance, so a wave
// solves four instances and a 256-thread workgroup sixteen.  Lane g of a group
// keeps rows i = g + 16 jj (jj < R) of J, aref, D, r, q in registers.  Every
// lane also keeps the whole lower triangle of M and of the Newton matrix
// (NP (NP + 1) / 2 values) and factors/solves it redundantly, so the only
// cross-lane traffic is the 16-lane all-reduce of row sums (four DPP adds per
// value).  n <= NP is handled by padding: padded coordinates have zero J
// columns, unit mass and a0 = a = 0, so they stay exactly zero.
//
// The all-reduce gives every lane of a group bit-identical totals (each DPP
// step adds the same two partials, only commuted), so every branch below is
// uniform within a group.
#pragma once

#include "cs_device.hpp"

namespace cs {

constexpr int SG = 16;   // lanes per instance

template <typename T> __device__ inline T gsum16(T v);

template <> __device__ inline float gsum16<float>(float v) {
    // quad xor 1, quad xor 2, half-row mirror, row mirror
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
    return v;
}

template <> __device__ inline double gsum16<double>(double v) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 16);
    return v;
}

template <int NP> struct Tri {
    static constexpr int NE = NP * (NP + 1) / 2;
    __host__ __device__ static constexpr int idx(int j, int l) { return j * (j + 1) / 2 + l; }  // l <= j
};

// Cholesky of the packed lower triangle in registers; returns false when a
// pivot is not positive.  inv[] receives 1 / L_jj.
template <typename T, int NP>
__device__ inline bool reg_cholesky(T (&H)[Tri<NP>::NE], T (&inv)[NP]) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        T s = H[Tri<NP>::idx(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= H[Tri<NP>::idx(j, k)] * H[Tri<NP>::idx(j, k)];
        ok = ok && (s > T(0));
        const T d = sqrt(s);
        H[Tri<NP>::idx(j, j)] = d;
        const T iv = T(1) / d;
        inv[j] = iv;
#pragma unroll
        for (int i = j + 1; i < NP; ++i) {
            T t = H[Tri<NP>::idx(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= H[Tri<NP>::idx(i, k)] * H[Tri<NP>::idx(j, k)];
            H[Tri<NP>::idx(i, j)] = t * iv;
        }
    }
    return ok;
}

// x = (L L^T)^{-1} b
template <typename T, int NP>
__device__ inline void reg_chol_solve(const T (&L)[Tri<NP>::NE], const T (&inv)[NP], const T (&b)[NP],
                                      T (&x)[NP]) {
    T y[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        T s = b[j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[Tri<NP>::idx(j, k)] * y[k];
        y[j] = s * inv[j];
    }
#pragma unroll
    for (int j = NP - 1; j >= 0; --j) {
        T s = y[j];
#pragma unroll
        for (int k = j + 1; k < NP; ++k) s -= L[Tri<NP>::idx(k, j)] * x[k];
        x[j] = s * inv[j];
    }
}

// symmetric M (lower triangle) times v
template <typename T, int NP>
__device__ inline void sym_mv(const T (&Ml)[Tri<NP>::NE], const T (&v)[NP], T (&out)[NP]) {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        T s = T(0);
#pragma unroll
        for (int l = 0; l < NP; ++l) s += Ml[l <= j ? Tri<NP>::idx(j, l) : Tri<NP>::idx(l, j)] * v[l];
        out[j] = s;
    }
}

// Per-group instance context: loads of one instance into registers.
template <typename T, int NP, int R>
struct SmallInst {
    int n, m;
    T J[R][NP];
    T aref[R], D[R];
    T Ml[Tri<NP>::NE];
    T a0[NP];
    bool bad;

    __device__ inline void load(const Inst &I, int g, const T *__restrict__ gM, const T *__restrict__ gJ,
                                const T *__restrict__ ga0, const T *__restrict__ garef,
                                const T *__restrict__ gD) {
        n = I.n;
        m = I.m;
        bad = false;
        const T *Jb = gJ + I.omn;
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            const int i = g + SG * jj;
            const bool live = i < m;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                T x = (live && j < n) ? Jb[(size_t)i * n + j] : T(0);
                bad |= !finite_val(x);
                J[jj][j] = x;
            }
            aref[jj] = live ? garef[I.om + i] : T(0);
            D[jj] = live ? gD[I.om + i] : T(0);
            bad |= !finite_val(aref[jj]) || !finite_val(D[jj]);
        }
        const T *Mb = gM + I.onn;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
#pragma unroll
            for (int l = 0; l <= j; ++l) {
                T x = (j < n && l < n) ? Mb[j * n + l] : (j == l ? T(1) : T(0));
                bad |= !finite_val(x);
                Ml[Tri<NP>::idx(j, l)] = x;
            }
            a0[j] = j < n ? ga0[I.on + j] : T(0);
            bad |= !finite_val(a0[j]);
        }
        // every lane checked a different part of J; the group agrees on `bad`
        T flag = bad ? T(1) : T(0);
        bad = gsum16(flag) != T(0);
    }
};

// One Newton solve of the group's instance.  On return a holds the iterate,
// H/inv the Cholesky factor of H(A(a)) (valid when st has CONVERGED/MAXITER)
// and act the active rows of this lane.
template <typename T, int NP, int R>
__device__ inline int small_solve(SmallInst<T, NP, R> &S, int max_iter, T tol, T (&a)[NP],
                                  T (&H)[Tri<NP>::NE], T (&inv)[NP], bool (&act)[R], int &iters) {
    iters = 0;
    {   // M must be positive definite
        T Hc[Tri<NP>::NE];
#pragma unroll
        for (int e = 0; e < Tri<NP>::NE; ++e) Hc[e] = S.Ml[e];
        if (!reg_cholesky<T, NP>(Hc, inv)) return ST_NOTSPD;
    }
    T trM = T(0);
#pragma unroll
    for (int j = 0; j < NP; ++j) trM += S.Ml[Tri<NP>::idx(j, j)];
    trM -= T(NP - S.n);   // padded coordinates carry unit mass
    T step_inf = T(-1);
    int st = 0, lsfail = 0;
    T r[R];
#pragma unroll
    for (int jj = 0; jj < R; ++jj) act[jj] = false;
    for (int k = 0;; ++k) {
        // residual, active set, gradient (eq. 6)
        T d[NP], F[NP], w[R];
        bool changed = false;
#pragma unroll
        for (int j = 0; j < NP; ++j) d[j] = a[j] - S.a0[j];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) s += S.J[jj][j] * a[j];
            r[jj] = s - S.aref[jj];
            const bool live = (int)(threadIdx.x & (SG - 1)) + SG * jj < S.m;
            const bool an = live && r[jj] < T(0);
            changed |= an != act[jj];
            act[jj] = an;
            w[jj] = an ? S.D[jj] * r[jj] : T(0);
        }
        sym_mv<T, NP>(S.Ml, d, F);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T s = T(0);
#pragma unroll
            for (int jj = 0; jj < R; ++jj) s += S.J[jj][j] * w[jj];
            F[j] += gsum16(s);
        }
        const bool same = gsum16(changed ? T(1) : T(0)) == T(0);
        T g2 = T(0), anorm = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            g2 += F[j] * F[j];
            anorm = fmax(anorm, fabs(a[j]));
        }
        // Newton matrix (eq. 9) -- assembled every pass, also for the state
#pragma unroll
        for (int j = 0; j < NP; ++j) {
#pragma unroll
            for (int l = 0; l <= j; ++l) {
                T s = T(0);
#pragma unroll
                for (int jj = 0; jj < R; ++jj) s += (act[jj] ? S.D[jj] : T(0)) * S.J[jj][j] * S.J[jj][l];
                H[Tri<NP>::idx(j, l)] = S.Ml[Tri<NP>::idx(j, l)] + gsum16(s);
            }
        }
        if (!reg_cholesky<T, NP>(H, inv)) { st = ST_NOTSPD; break; }
        if (sqrt(g2) <= tol * trM ||
            (step_inf >= T(0) && same && step_inf <= tol * (T(1) + anorm))) {
            st = ST_CONVERGED;
            break;
        }
        if (k == max_iter) { st = ST_MAXITER; break; }
        T p[NP], nF[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) nF[j] = -F[j];
        reg_chol_solve<T, NP>(H, inv, nF, p);
        // exact line search (eq. 10)
        T q[R];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) s += S.J[jj][j] * p[j];
            q[jj] = s;
        }
        T Mp[NP];
        sym_mv<T, NP>(S.Ml, p, Mp);
        T c0 = T(0), b0 = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            c0 += p[j] * Mp[j];
            b0 += Mp[j] * d[j];
        }
        T alpha;
        {
            T t = T(1), c, b;
            uint32_t bits = 0;
            {
                T sc = T(0), sb = T(0);
#pragma unroll
                for (int jj = 0; jj < R; ++jj) {
                    const bool live = (int)(threadIdx.x & (SG - 1)) + SG * jj < S.m;
                    if (live && r[jj] + t * q[jj] < T(0)) {
                        const T dq = S.D[jj] * q[jj];
                        sc += dq * q[jj];
                        sb += dq * r[jj];
                        bits |= 1u << jj;
                    }
                }
                c = c0 + gsum16(sc);
                b = b0 + gsum16(sb);
            }
            T lo = T(0), hi = inf_val<T>();
            alpha = t;
            int fail = 1;
            const T eps = T(sizeof(T) == 4 ? 1.1920929e-7 : 2.220446049250313e-16);
            for (int it = 0; it < 96; ++it) {
                const T gp = c * t + b;
                if (gp == T(0)) { alpha = t; fail = 0; break; }
                if (gp < T(0)) lo = t; else hi = t;
                if (hi < inf_val<T>() && hi - lo <= T(32) * eps * hi) { alpha = t; fail = 0; break; }
                T cand = -b / c;
                const bool newton = (cand > lo) && (cand < hi);
                if (!newton) cand = (hi < inf_val<T>()) ? T(0.5) * (lo + hi) : T(2) * lo + T(1);
                uint32_t nb = 0;
                T sc = T(0), sb = T(0);
#pragma unroll
                for (int jj = 0; jj < R; ++jj) {
                    const bool live = (int)(threadIdx.x & (SG - 1)) + SG * jj < S.m;
                    if (live && r[jj] + cand * q[jj] < T(0)) {
                        const T dq = S.D[jj] * q[jj];
                        sc += dq * q[jj];
                        sb += dq * r[jj];
                        nb |= 1u << jj;
                    }
                }
                const T mism = gsum16(T(__builtin_popcount(nb ^ bits)));
                c = c0 + gsum16(sc);
                b = b0 + gsum16(sb);
                bits = nb;
                t = cand;
                alpha = cand;
                if (newton && mism == T(0)) { fail = 0; break; }
            }
            lsfail |= fail;
        }
        step_inf = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const T s = alpha * p[j];
            a[j] += s;
            step_inf = fmax(step_inf, fabs(s));
        }
        iters = k + 1;
    }
    if (lsfail) st |= ST_LSFAIL;
    return st;
}

template <typename T, int NP, int R>
__global__ __launch_bounds__(256) void k_forward_small(
    BatchView bv, int nb_inst, int max_iter, T tol, const T *__restrict__ gM,
    const T *__restrict__ gJ, const T *__restrict__ ga0, const T *__restrict__ garef,
    const T *__restrict__ gD, const T *__restrict__ gainit, T *__restrict__ gaout,
    T *__restrict__ gfac, uint8_t *__restrict__ gmask, int32_t *__restrict__ gstatus,
    int32_t *__restrict__ giters) {
    const int g = threadIdx.x & (SG - 1);
    const int w = blockIdx.x * (blockDim.x / SG) + threadIdx.x / SG;
    if (w >= nb_inst) return;   // whole groups only: no cross-group traffic follows
    const Inst I = inst_at(bv, w);
    SmallInst<T, NP, R> S;
    S.load(I, g, gM, gJ, ga0, garef, gD);
    T a[NP];
    bool bad = S.bad;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        a[j] = j < S.n ? (gainit ? gainit[I.on + j] : S.a0[j]) : T(0);
        bad |= !finite_val(a[j]);
    }
    bad = gsum16(bad ? T(1) : T(0)) != T(0);
    T H[Tri<NP>::NE], inv[NP];
    bool act[R];
    int iters = 0, st;
    if (bad) {
        st = ST_NONFINITE;
    } else {
        st = small_solve<T, NP, R>(S, max_iter, tol, a, H, inv, act, iters);
    }
    const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
    const T nanv = T(__builtin_nan(""));
    // outputs: lane j < n writes a_j; factor entries spread over the group
#pragma unroll
    for (int j = 0; j < NP; ++j)
        if (j == g && j < S.n) gaout[I.on + j] = ok ? a[j] : nanv;
    T *fac = gfac + I.onn;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
#pragma unroll
        for (int l = 0; l <= j; ++l) {
            const int e = Tri<NP>::idx(j, l);
            if ((e & (SG - 1)) == g && j < S.n) fac[j * S.n + l] = ok ? H[e] : nanv;
        }
    }
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        const int i = g + SG * jj;
        if (i < S.m) gmask[I.om + i] = (ok && act[jj]) ? 1 : 0;
    }
    if (g == 0) {
        gstatus[I.b] = st;
        if (giters) giters[I.b] = iters;
    }
}

template <typename T, int NP, int R>
__global__ __launch_bounds__(256) void k_ift_vjp_small(
    BatchView bv, int nb_inst, const T *__restrict__ gfac, const uint8_t *__restrict__ gmask,
    const T *__restrict__ gM, const T *__restrict__ gJ, const T *__restrict__ ga0,
    const T *__restrict__ garef, const T *__restrict__ gD, const T *__restrict__ ga,
    const T *__restrict__ gabar, T *__restrict__ ga0bar, T *__restrict__ garefbar,
    T *__restrict__ gJbar, T *__restrict__ gDbar, T *__restrict__ gMbar) {
    const int g = threadIdx.x & (SG - 1);
    const int w = blockIdx.x * (blockDim.x / SG) + threadIdx.x / SG;
    if (w >= nb_inst) return;
    const Inst I = inst_at(bv, w);
    const int n = I.n, m = I.m;
    SmallInst<T, NP, R> S;
    S.load(I, g, gM, gJ, ga0, garef, gD);
    T L[Tri<NP>::NE], inv[NP], a[NP], ab[NP];
    const T *fac = gfac + I.onn;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
#pragma unroll
        for (int l = 0; l <= j; ++l)
            L[Tri<NP>::idx(j, l)] = (j < n && l < n) ? fac[j * n + l] : (j == l ? T(1) : T(0));
        inv[j] = T(1) / L[Tri<NP>::idx(j, j)];
        a[j] = j < n ? ga[I.on + j] : T(0);
        ab[j] = j < n ? gabar[I.on + j] : T(0);
    }
    bool act[R];
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        const int i = g + SG * jj;
        act[jj] = i < m && gmask[I.om + i] != 0;
    }
    // lambda = H^{-1} abar, one step of iterative refinement with
    // H v = M v + J^T (D o A* o J v)
    T lam[NP];
    reg_chol_solve<T, NP>(L, inv, ab, lam);
    {
        T Ml_l[NP], res[NP], dl[NP];
        sym_mv<T, NP>(S.Ml, lam, Ml_l);
        T t[R];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) s += S.J[jj][j] * lam[j];
            t[jj] = act[jj] ? S.D[jj] * s : T(0);
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T s = T(0);
#pragma unroll
            for (int jj = 0; jj < R; ++jj) s += S.J[jj][j] * t[jj];
            res[j] = ab[j] - Ml_l[j] - gsum16(s);
        }
        reg_chol_solve<T, NP>(L, inv, res, dl);
#pragma unroll
        for (int j = 0; j < NP; ++j) lam[j] += dl[j];
    }
    T *Jbar = gJbar ? gJbar + I.omn : nullptr;
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        const int i = g + SG * jj;
        if (i >= m) continue;
        T ja = T(0), sig = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            ja += S.J[jj][j] * a[j];
            sig += S.J[jj][j] * lam[j];
        }
        const T r = ja - S.aref[jj];
        const T wv = act[jj] ? S.D[jj] * r : T(0);
        const T ar = act[jj] ? S.D[jj] * sig : T(0);
        if (garefbar) garefbar[I.om + i] = ar;
        if (gDbar) gDbar[I.om + i] = act[jj] ? -r * sig : T(0);
        if (Jbar) {
#pragma unroll
            for (int j = 0; j < NP; ++j)
                if (j < n) Jbar[(size_t)i * n + j] = -(wv * lam[j] + ar * a[j]);
        }
    }
    if (ga0bar) {
        T mt[NP];
        sym_mv<T, NP>(S.Ml, lam, mt);
#pragma unroll
        for (int j = 0; j < NP; ++j)
            if (j == g && j < n) ga0bar[I.on + j] = mt[j];
    }
    if (gMbar) {
        T *Mb = gMbar + I.onn;
        T d[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) d[j] = a[j] - S.a0[j];
#pragma unroll
        for (int j = 0; j < NP; ++j)
#pragma unroll
            for (int l = 0; l < NP; ++l)
                if (((j * NP + l) & (SG - 1)) == g && j < n && l < n) Mb[j * n + l] = -lam[j] * d[l];
    }
}

// Host-side dispatch ---------------------------------------------------------

// Padded sizes and row capacities the small kernels are built for.
inline int small_np(int n) {
    if (n <= 3) return 3;
    if (n <= 6) return 6;
    if (n <= 9) return 9;
    if (n <= 12) return 12;
    return 0;
}
inline int small_r(int m) {
    if (m <= 16) return 1;
    if (m <= 32) return 2;
    if (m <= 64) return 4;
    return 0;
}

// FP32: n <= 12; FP64 (twice the registers per value): n <= 6.
inline bool small_supported(int nmax, int mmax, bool packed, int s) {
    const int np = small_np(nmax);
    return !packed && np != 0 && small_r(mmax) != 0 && (s == 4 ? np <= 12 : np <= 6);
}

inline bool small_unrolled_supported(int, int, bool, int) { return false; }

#define CS_SMALL_DISPATCH(NPV, RV, CALL)                                                      \
    if (np == NPV && rr == RV) { CALL(NPV, RV); }

#define CS_SMALL_ALL(CALL)                                                                    \
    if constexpr (sizeof(T) == 4) {                                                           \
        CS_SMALL_DISPATCH(3, 1, CALL) else CS_SMALL_DISPATCH(3, 2, CALL) else CS_SMALL_DISPATCH(3, 4, CALL) \
        else CS_SMALL_DISPATCH(6, 1, CALL) else CS_SMALL_DISPATCH(6, 2, CALL) else CS_SMALL_DISPATCH(6, 4, CALL) \
        else CS_SMALL_DISPATCH(9, 1, CALL) else CS_SMALL_DISPATCH(9, 2, CALL) else CS_SMALL_DISPATCH(9, 4, CALL) \
        else CS_SMALL_DISPATCH(12, 1, CALL) else CS_SMALL_DISPATCH(12, 2, CALL) else CS_SMALL_DISPATCH(12, 4, CALL) \
        else { return -4; }                                                                   \
    } else {                                                                                  \
        CS_SMALL_DISPATCH(3, 1, CALL) else CS_SMALL_DISPATCH(3, 2, CALL) else CS_SMALL_DISPATCH(3, 4, CALL) \
        else CS_SMALL_DISPATCH(6, 1, CALL) else CS_SMALL_DISPATCH(6, 2, CALL) else CS_SMALL_DISPATCH(6, 4, CALL) \
        else { return -4; }                                                                   \
    }

template <typename T>
int launch_small_forward(const BatchView &bv, int nmax, int mmax, int max_iter, T tol, const T *M,
                         const T *J, const T *a0, const T *aref, const T *D, const T *a_init,
                         T *a_out, T *fac, uint8_t *mask, int32_t *status, int32_t *iters,
                         hipStream_t stream) {
    const int np = small_np(nmax), rr = small_r(mmax);
    const int nb = bv.B;
    const dim3 grid((nb + 15) / 16), block(256);
#define CS_CALL_FWD(NPV, RV)                                                                  \
    hipLaunchKernelGGL((k_forward_small<T, NPV, RV>), grid, block, 0, stream, bv, nb, max_iter, \
                       tol, M, J, a0, aref, D, a_init, a_out, fac, mask, status, iters);
    CS_SMALL_ALL(CS_CALL_FWD)
#undef CS_CALL_FWD
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <typename T>
int launch_small_vjp(const BatchView &bv, int nmax, int mmax, const T *fac, const uint8_t *mask,
                     const T *M, const T *J, const T *a0, const T *aref, const T *D, const T *a,
                     const T *abar, T *a0bar, T *arefbar, T *Jbar, T *Dbar, T *Mbar,
                     hipStream_t stream) {
    const int np = small_np(nmax), rr = small_r(mmax);
    const int nb = bv.B;
    const dim3 grid((nb + 15) / 16), block(256);
#define CS_CALL_VJP(NPV, RV)                                                                  \
    hipLaunchKernelGGL((k_ift_vjp_small<T, NPV, RV>), grid, block, 0, stream, bv, nb, fac, mask, \
                       M, J, a0, aref, D, a, abar, a0bar, arefbar, Jbar, Dbar, Mbar);
    CS_SMALL_ALL(CS_CALL_VJP)
#undef CS_CALL_VJP
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <typename T>
int launch_small_unrolled(const BatchView &, int, int, int, T, const T *, const T *, const T *,
                          const T *, const T *, const T *, T *, T *, T *, T *, T *, T *, T *,
                          uint8_t *, int32_t *, int32_t *, hipStream_t) {
    return -4;
}

}  // namespace cs
