// cs_small.hpp -- register-resident kernels for small instances.
//
// Mapping: a group of 16 lanes (one DPP row) owns one instance, so a wave
// solves four instances and a 256-thread workgroup sixteen.  Lane g of a group
// owns the contiguous block of rows g R .. g R + R - 1 of J, aref, D, r, q and
// keeps it in registers; a block of a J row-major matrix is contiguous, so it
// is read (and J-bar written) with 16-byte vector accesses.  Every lane also
// keeps the lower triangle of M and of the Newton matrix (NP (NP + 1) / 2
// values) and factors/solves it redundantly, so the only cross-lane traffic is
// the 16-lane all-reduce of row sums (four DPP adds per value).  n <= NP is
// handled by padding: padded coordinates have zero J columns, unit mass and
// a0 = a = 0, so they stay exactly zero.  Rows past m have J = D = aref = 0,
// so they are never active and contribute nothing.
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

// Whether `x` holds in any lane of this lane's 16-lane group: one ballot and a
// shift, instead of a four-step DPP reduction (every lane of a group shares
// the group's control flow, so the group's 16 bits are all live or all not).
__device__ inline bool group_any16(bool x) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(x);
    return ((m >> (threadIdx.x & 48)) & 0xFFFFull) != 0;
}

// Two independent 16-lane sums with their DPP steps interleaved, so that each
// step of one hides the other's wait states (the compiler keeps a loop body's
// DPP chains in source order).
__device__ inline void gsum16x2(float &a, float &b) {
#define CS_GS2(CTRL)                                                                               \
    {                                                                                              \
        const float ta = __builtin_bit_cast(                                                       \
            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, a), CTRL, 0xF, 0xF, false)); \
        const float tb = __builtin_bit_cast(                                                       \
            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, b), CTRL, 0xF, 0xF, false)); \
        a += ta;                                                                                   \
        b += tb;                                                                                   \
    }
    CS_GS2(0xB1)
    CS_GS2(0x4E)
    CS_GS2(0x141)
    CS_GS2(0x140)
#undef CS_GS2
}

// FP64: the same four DPP steps on the two halves of each value.
template <int CTRL> __device__ inline double dpp_f64(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <> __device__ inline double gsum16<double>(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return v;
}
__device__ inline void gsum16x2(double &a, double &b) {
    const double a1 = dpp_f64<0xB1>(a), b1 = dpp_f64<0xB1>(b);
    a += a1;
    b += b1;
    const double a2 = dpp_f64<0x4E>(a), b2 = dpp_f64<0x4E>(b);
    a += a2;
    b += b2;
    const double a3 = dpp_f64<0x141>(a), b3 = dpp_f64<0x141>(b);
    a += a3;
    b += b3;
    const double a4 = dpp_f64<0x140>(a), b4 = dpp_f64<0x140>(b);
    a += a4;
    b += b4;
}

template <typename T> __device__ inline T fast_rsq(T x);
template <> __device__ inline float fast_rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ inline double fast_rsq<double>(double x) { return 1.0 / sqrt(x); }
template <typename T> __device__ inline T fast_rcp(T x);
template <> __device__ inline float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double fast_rcp<double>(double x) { return 1.0 / x; }

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); static constexpr int V = 4; };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); static constexpr int V = 2; };

template <int NP> struct Tri {
    static constexpr int NE = NP * (NP + 1) / 2;
    __host__ __device__ static constexpr int idx(int j, int l) { return j * (j + 1) / 2 + l; }  // l <= j
};

// Cholesky of the packed lower triangle in registers; returns false when a
// pivot is not positive.  inv[] receives 1 / L_jj.  Right-looking: once
// column j is scaled, every trailing entry takes its update independently, so
// the dependency chain per column is pivot -> rsq -> scale -> next pivot.
template <typename T, int NP>
__device__ inline bool reg_cholesky(T (&H)[Tri<NP>::NE], T (&inv)[NP]) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const T s = H[Tri<NP>::idx(j, j)];
        ok = ok && (s > T(0));
        const T iv = fast_rsq(s);
        H[Tri<NP>::idx(j, j)] = s * iv;
        inv[j] = iv;
#pragma unroll
        for (int i = j + 1; i < NP; ++i) H[Tri<NP>::idx(i, j)] *= iv;
#pragma unroll
        for (int i = j + 1; i < NP; ++i)
#pragma unroll
            for (int k = j + 1; k <= i; ++k)
                H[Tri<NP>::idx(i, k)] -= H[Tri<NP>::idx(i, j)] * H[Tri<NP>::idx(k, j)];
    }
    return ok;
}

// x = (L L^T)^{-1} b, both substitutions column-oriented: after each solved
// component the remaining right-hand side entries update independently.
template <typename T, int NP>
__device__ inline void reg_chol_solve(const T (&L)[Tri<NP>::NE], const T (&inv)[NP], const T (&b)[NP],
                                      T (&x)[NP]) {
    T y[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) y[j] = b[j];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        y[j] *= inv[j];
#pragma unroll
        for (int i = j + 1; i < NP; ++i) y[i] -= L[Tri<NP>::idx(i, j)] * y[j];
    }
#pragma unroll
    for (int j = NP - 1; j >= 0; --j) {
        x[j] = y[j] * inv[j];
#pragma unroll
        for (int i = 0; i < j; ++i) y[i] -= L[Tri<NP>::idx(j, i)] * x[j];
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

// Load CNT contiguous values starting at p; 16-byte vectors when `vec`,
// otherwise element by element (elements past `live` read as 0).
template <typename T, int CNT>
__device__ inline void load_run(const T *__restrict__ p, bool vec, int live, T (&out)[CNT]) {
    constexpr int V = Vec16<T>::V;
    if constexpr (CNT % V == 0) {
        if (vec) {
            typedef typename Vec16<T>::type VT;
            const VT *pv = reinterpret_cast<const VT *>(p);
#pragma unroll
            for (int v = 0; v < CNT / V; ++v) {
                const VT x = pv[v];
#pragma unroll
                for (int e = 0; e < V; ++e) out[v * V + e] = x[e];
            }
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < CNT; ++e) out[e] = e < live ? p[e] : T(0);
}

template <typename T, int CNT>
__device__ inline void store_run(T *__restrict__ p, bool vec, int live, const T (&in)[CNT]) {
    constexpr int V = Vec16<T>::V;
    if constexpr (CNT % V == 0) {
        if (vec) {
            typedef typename Vec16<T>::type VT;
            VT *pv = reinterpret_cast<VT *>(p);
#pragma unroll
            for (int v = 0; v < CNT / V; ++v) {
                VT x;
#pragma unroll
                for (int e = 0; e < V; ++e) x[e] = in[v * V + e];
                pv[v] = x;
            }
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < CNT; ++e)
        if (e < live) p[e] = in[e];
}

__device__ inline bool aligned16(const void *p) {
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// The 16 lanes of a group share one wave: LDS written by one lane of the
// group is visible to the others after this (in-order LDS within a wave).
__device__ inline void group_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copy cnt contiguous values into the group's LDS area with coalesced loads
// (lane g takes elements g, g + 16, ...).
template <typename T>
__device__ inline void group_copy_in(const T *__restrict__ src, int cnt, T *dst, int g) {
    for (int e = g; e < cnt; e += SG) dst[e] = src[e];
}

// x in FP64, converted where it is used: the empty asm stops the compiler
// from hoisting the conversions of loop-invariant values out of a loop
// (which would hold an FP64 copy of every one of them in registers).
template <typename T> __device__ inline double as_f64_here(T x) {
    asm volatile("" : "+v"(x));
    return double(x);
}

// LDS per group for staged inputs/outputs of one instance: M (NP x NP
// values used n x n), the factor (NE), and two NP-vectors.
template <int NP> struct GroupShm {
    static constexpr int NE = NP * (NP + 1) / 2;
    static constexpr int M0 = 0, F0 = NP * NP, V0 = F0 + NE, W0 = V0 + NP, SIZE = W0 + NP;
};

// Per-group instance context: one instance's data in registers.
template <typename T, int NP, int R>
struct SmallInst {
    int n, m, i0;        // i0: first row of this lane's block
    bool full;           // this lane's block is R full rows of width NP
    T J[R][NP];
    T aref[R], D[R];
    T Ml[Tri<NP>::NE];
    T a0[NP];
    bool bad;

    // True for the whole wave when every lane's block is R full rows of
    // width NP at 16-byte aligned addresses (where vector loads are used):
    // then load_fast() issues every load of the instance before any use.
    __device__ static inline bool fast_ok(const Inst &I, int g, const T *__restrict__ gJ,
                                          const T *__restrict__ garef, const T *__restrict__ gD) {
        constexpr int V = Vec16<T>::V;
        const int i0 = g * R;
        const bool fl = (I.n == NP) && (i0 + R <= I.m);
        const bool vj = (R * NP) % V != 0 || aligned16(gJ + I.omn + (int64_t)i0 * NP);
        const bool vr = R % V != 0 || (aligned16(garef + I.om + i0) && aligned16(gD + I.om + i0));
        return __builtin_amdgcn_ballot_w64(!(fl && vj && vr)) == 0;
    }

    // Loads of a full block (fast_ok): no predicates, so the compiler keeps
    // every load in flight together.
    __device__ inline void load_fast(const Inst &I, int g, const T *__restrict__ gM,
                                     const T *__restrict__ gJ, const T *__restrict__ ga0,
                                     const T *__restrict__ garef, const T *__restrict__ gD) {
        n = NP;
        m = I.m;
        i0 = g * R;
        full = true;
        T flat[R * NP];
        load_run<T, R * NP>(gJ + I.omn + (int64_t)i0 * NP, true, R * NP, flat);
        load_run<T, R>(garef + I.om + i0, true, R, aref);
        load_run<T, R>(gD + I.om + i0, true, R, D);
        const T *Mb = gM + I.onn;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
#pragma unroll
            for (int l = 0; l <= j; ++l) Ml[Tri<NP>::idx(j, l)] = Mb[j * NP + l];
            a0[j] = ga0[I.on + j];
        }
#pragma unroll
        for (int jj = 0; jj < R; ++jj)
#pragma unroll
            for (int j = 0; j < NP; ++j) J[jj][j] = flat[jj * NP + j];
    }

    // General loads (ragged blocks, n < NP).  msh: the group's LDS area for
    // M (n x n), or null to read M from global memory in every lane.
    __device__ inline void load_general(const Inst &I, int g, const T *__restrict__ gM,
                                        const T *__restrict__ gJ, const T *__restrict__ ga0,
                                        const T *__restrict__ garef, const T *__restrict__ gD,
                                        T *msh) {
        n = I.n;
        m = I.m;
        i0 = g * R;
        full = (n == NP) && (i0 + R <= m);
        const T *Jb = gJ + I.omn + (int64_t)i0 * n;
        if (full) {
            T flat[R * NP];
            load_run<T, R * NP>(Jb, aligned16(Jb), R * NP, flat);
#pragma unroll
            for (int jj = 0; jj < R; ++jj)
#pragma unroll
                for (int j = 0; j < NP; ++j) J[jj][j] = flat[jj * NP + j];
        } else {
#pragma unroll
            for (int jj = 0; jj < R; ++jj)
#pragma unroll
                for (int j = 0; j < NP; ++j)
                    J[jj][j] = (i0 + jj < m && j < n) ? Jb[(int64_t)jj * n + j] : T(0);
        }
        const int live = m - i0;
        const T *ar = garef + I.om + i0, *dd = gD + I.om + i0;
        load_run<T, R>(ar, live >= R && aligned16(ar), live, aref);
        load_run<T, R>(dd, live >= R && aligned16(dd), live, D);
        const T *Mb = gM + I.onn;
        if (msh) {
            group_copy_in(Mb, n * n, msh, g);
            group_sync();
            Mb = msh;
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
#pragma unroll
            for (int l = 0; l <= j; ++l)
                Ml[Tri<NP>::idx(j, l)] = (j < n) ? Mb[j * n + l] : (j == l ? T(1) : T(0));
            a0[j] = j < n ? ga0[I.on + j] : T(0);
        }
    }

    // The instance has a non-finite input (group-uniform).
    __device__ inline void check() {
        bool b = false;
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            b |= !finite_val(aref[jj]) || !finite_val(D[jj]);
#pragma unroll
            for (int j = 0; j < NP; ++j) b |= !finite_val(J[jj][j]);
        }
#pragma unroll
        for (int e = 0; e < Tri<NP>::NE; ++e) b |= !finite_val(Ml[e]);
#pragma unroll
        for (int j = 0; j < NP; ++j) b |= !finite_val(a0[j]);
        bad = gsum16(b ? T(1) : T(0)) != T(0);
    }

    __device__ inline void load(const Inst &I, int g, const T *__restrict__ gM,
                                const T *__restrict__ gJ, const T *__restrict__ ga0,
                                const T *__restrict__ garef, const T *__restrict__ gD,
                                T *msh = nullptr) {
        if (fast_ok(I, g, gJ, garef, gD))
            load_fast(I, g, gM, gJ, ga0, garef, gD);
        else
            load_general(I, g, gM, gJ, ga0, garef, gD, msh);
        check();
    }
};

// Where one instance's unrolled-trace records go (unused when not taping).
template <typename T>
struct StepTape {
    T *tT;          // this instance's T records
    uint8_t *tB;    // this instance's byte records
    int n, m, recT;
};

// Exact line search along p in registers (Sec. III-B, eq. 10); the method is
// the safeguarded piece Newton of team_line_search in cs_device.hpp.  Returns
// alpha; when BITS, the accepted piece's rows (bits) and slope c are returned
// for the tape.
//
// A Newton point is accepted when it lies on the piece that produced it.
// With BITS that is checked row by row (one more group sum per round);
// without, by the piece sums (c, b) coming out bitwise equal: equal row sets
// give equal sums (same partials, same reduction order), and a different set
// with equal sums has the same linear phi' there, whose root is the point.
template <bool BITS, typename T, int R>
__device__ inline T small_line_search(const T (&r)[R], const T (&q)[R], const T (&D)[R], T c0, T b0,
                                      uint32_t &bits_out, T &c_out, int &fail) {
    T dqq[R], dqr[R];
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        const T dq = D[jj] * q[jj];
        dqq[jj] = dq * q[jj];
        dqr[jj] = dq * r[jj];
    }
    auto piece = [&](T t, uint32_t &bits, T &c, T &b) {
        T sc = T(0), sb = T(0);
        uint32_t bb = 0;
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            const bool pa = r[jj] + t * q[jj] < T(0);
            sc += pa ? dqq[jj] : T(0);
            sb += pa ? dqr[jj] : T(0);
            if constexpr (BITS) bb |= (pa ? 1u : 0u) << jj;
        }
        gsum16x2(sc, sb);
        c = c0 + sc;
        b = b0 + sb;
        bits = bb;
    };
    T t = T(1), c, b;
    uint32_t bits;
    piece(t, bits, c, b);
    T lo = T(0), hi = inf_val<T>();
    fail = 1;
    const T eps = T(sizeof(T) == 4 ? 1.1920929e-7 : 2.220446049250313e-16);
    for (int it = 0; it < 96; ++it) {
        const T gp = c * t + b;
        if (gp == T(0)) { fail = 0; break; }
        if (gp < T(0)) lo = t; else hi = t;
        if (hi < inf_val<T>() && hi - lo <= T(32) * eps * hi) { fail = 0; break; }
        T cand = -b * fast_rcp(c);
        const bool newton = (cand > lo) && (cand < hi);
        if (!newton) cand = (hi < inf_val<T>()) ? T(0.5) * (lo + hi) : T(2) * lo + T(1);
        uint32_t nb;
        T nc, nbv;
        piece(cand, nb, nc, nbv);
        bool same;
        if constexpr (BITS) same = gsum16(T(__builtin_popcount(nb ^ bits))) == T(0);
        else same = (nc == c) && (nbv == b);
        bits = nb;
        c = nc;
        b = nbv;
        t = cand;
        if (newton && same) { fail = 0; break; }
    }
    bits_out = bits;
    c_out = c;
    return t;
}

// One Newton solve of the group's instance.  On return a holds the iterate,
// H/inv the Cholesky factor of H(A(a)) (valid when st has CONVERGED/MAXITER)
// and act the active rows of this lane.  When TAPE, every step taken is
// recorded in tp (the unrolled VJP's K is max_iter).
template <bool TAPE, typename T, int NP, int R>
__device__ inline int small_solve(const SmallInst<T, NP, R> &S, int max_iter, T tol, T (&a)[NP],
                                  T (&H)[Tri<NP>::NE], T (&inv)[NP], bool (&act)[R], int &iters,
                                  const StepTape<T> &tp) {
    constexpr int NE = Tri<NP>::NE;
    const int g = threadIdx.x & (SG - 1);
    iters = 0;
#pragma unroll
    for (int jj = 0; jj < R; ++jj) act[jj] = false;
    {   // M must be positive definite
        T Hc[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) Hc[e] = S.Ml[e];
        if (!reg_cholesky<T, NP>(Hc, inv)) return ST_NOTSPD;
    }
    T trM = T(0);
#pragma unroll
    for (int j = 0; j < NP; ++j) trM += S.Ml[Tri<NP>::idx(j, j)];
    trM -= T(NP - S.n);   // padded coordinates carry unit mass
    T step_inf = T(-1);
    int st = 0, lsfail = 0;
    bool have_factor = false;
    // Md = M (a - a0), carried across steps (Md += alpha M p) so each step
    // takes one product with M
    T Md[NP];
    {
        T d0[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) d0[j] = a[j] - S.a0[j];
        sym_mv<T, NP>(S.Ml, d0, Md);
    }
    for (int k = 0;; ++k) {
        // residual, active set and gradient (eq. 6)
        T d[NP], F[NP], r[R], wD[R];
        bool changed = false;
#pragma unroll
        for (int j = 0; j < NP; ++j) d[j] = a[j] - S.a0[j];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) s += S.J[jj][j] * a[j];
            r[jj] = s - S.aref[jj];
            const bool an = r[jj] < T(0);
            changed |= an != act[jj];
            act[jj] = an;
            wD[jj] = an ? S.D[jj] : T(0);
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T s = T(0);
#pragma unroll
            for (int jj = 0; jj < R; ++jj) s += S.J[jj][j] * (wD[jj] * r[jj]);
            F[j] = Md[j] + gsum16(s);
        }
        const bool same = (k > 0) && !group_any16(changed);
        T g2 = T(0), anorm = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            g2 += F[j] * F[j];
            anorm = fmax(anorm, fabs(a[j]));
        }
        // Newton matrix (eq. 9); it depends on the active set only, so an
        // unchanged set keeps the previous factor
        if (!(same && have_factor)) {
            T tj[R][NP];
#pragma unroll
            for (int jj = 0; jj < R; ++jj)
#pragma unroll
                for (int j = 0; j < NP; ++j) tj[jj][j] = wD[jj] * S.J[jj][j];
#pragma unroll
            for (int j = 0; j < NP; ++j) {
#pragma unroll
                for (int l = 0; l <= j; ++l) {
                    T s = T(0);
#pragma unroll
                    for (int jj = 0; jj < R; ++jj) s += tj[jj][j] * S.J[jj][l];
                    H[Tri<NP>::idx(j, l)] = S.Ml[Tri<NP>::idx(j, l)] + gsum16(s);
                }
            }
            if (!reg_cholesky<T, NP>(H, inv)) { st = ST_NOTSPD; break; }
            have_factor = true;
        }
        const T gtol = tol * trM;
        if (g2 <= gtol * gtol ||
            (step_inf >= T(0) && same && step_inf <= tol * (T(1) + anorm))) {
            st = ST_CONVERGED;
            break;
        }
        if (k == max_iter) { st = ST_MAXITER; break; }
        T p[NP], nF[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) nF[j] = -F[j];
        reg_chol_solve<T, NP>(H, inv, nF, p);
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
        uint32_t bits;
        T cpiece;
        int fail;
        const T alpha = small_line_search<TAPE, T, R>(r, q, S.D, c0, b0, bits, cpiece, fail);
        lsfail |= fail;
        if constexpr (TAPE) {
            T *rec = tp.tT + (int64_t)k * tp.recT;
            uint8_t *recB = tp.tB + (int64_t)k * 2 * tp.m;
            const int n = tp.n, m = tp.m;
#pragma unroll
            for (int j = 0; j < NP; ++j)
                if (j == g && j < n) {
                    rec[j] = a[j];
                    rec[n + j] = p[j];
                }
            // factor: packed lower triangle of the n x n leading block
#pragma unroll
            for (int j = 0; j < NP; ++j)
#pragma unroll
                for (int l = 0; l <= j; ++l) {
                    const int e = Tri<NP>::idx(j, l);
                    if ((e & (SG - 1)) == g && j < n) rec[2 * n + e] = H[e];
                }
            const int ne = n * (n + 1) / 2;
            const int live = m - S.i0;
#pragma unroll
            for (int jj = 0; jj < R; ++jj)
                if (jj < live) {
                    rec[2 * n + ne + S.i0 + jj] = r[jj];
                    rec[2 * n + ne + m + S.i0 + jj] = q[jj];
                    recB[S.i0 + jj] = act[jj] ? 1 : 0;
                    recB[m + S.i0 + jj] = (bits >> jj) & 1u;
                }
            if (g == 0) {
                rec[2 * n + ne + 2 * m] = alpha;
                rec[2 * n + ne + 2 * m + 1] = cpiece;
            }
        }
        step_inf = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const T s = alpha * p[j];
            a[j] += s;
            Md[j] += alpha * Mp[j];
            step_inf = fmax(step_inf, fabs(s));
        }
        iters = k + 1;
    }
    if (lsfail) st |= ST_LSFAIL;
    return st;
}

// The same minimiser by preconditioned nonlinear conjugate gradients (Sec.
// III-B names it as the other solver; eqs. 11-14: the IFT derivative depends
// on the root only).  Directions p_k = -z_k + beta_k p_{k-1} with z = M^{-1} F
// (M is factored once) and Polak-Ribiere beta_k = max(0, F_k . (z_k -
// z_{k-1}) / (F_{k-1} . z_{k-1})), restarted (beta = 0) when the active set
// changed or p_k is not a descent direction; every step takes the exact line
// search of the Newton solve.  Each step costs two passes over J (r and q)
// instead of the Newton step's J^T D J assembly and Cholesky factorisation.
//
// The iterate, directions and every sum are FP64 whatever the storage type:
// CG takes hundreds to thousands of steps, each building on the last, and in
// FP32 the gradient's rounding (M (a - a0) and J^T w nearly cancel at the
// root) stalls it short of the FP32 Newton solve's accuracy.  The
// preconditioner solve z = M^{-1} F runs in the storage type (any fixed SPD
// preconditioner leaves the minimiser unchanged).
//
// Converged when ||F|| <= tol tr(M) (the Newton rule's gradient test) or
// F . M^{-1} F <= tol^2 tr(M) (1 + ||a||_inf)^2: L is M-strongly convex (its
// curvature H >= M everywhere), so ||a - a*||_M <= sqrt(F . M^{-1} F) and the
// second test bounds the distance to the minimiser.  The Newton rule's
// small-step test is not used: a short CG step says little about the distance
// to the root.  On return a holds the iterate rounded to T and H the factor of
// H(A) at it (the state the IFT VJP reads), assembled once.
template <typename T, int NP, int R>
__device__ inline int small_solve_cg(const SmallInst<T, NP, R> &S, int max_iter, T tol,
                                     T (&a)[NP], T (&H)[Tri<NP>::NE], T (&inv)[NP],
                                     bool (&act)[R], int &iters) {
    typedef double C;
    constexpr int NE = Tri<NP>::NE;
    iters = 0;
#pragma unroll
    for (int jj = 0; jj < R; ++jj) act[jj] = false;
    T Lm[NE], invm[NP];
#pragma unroll
    for (int e = 0; e < NE; ++e) Lm[e] = S.Ml[e];
    if (!reg_cholesky<T, NP>(Lm, invm)) return ST_NOTSPD;
    C trM = C(0);
#pragma unroll
    for (int j = 0; j < NP; ++j) trM += C(S.Ml[Tri<NP>::idx(j, j)]);
    trM -= C(NP - S.n);
    auto mv = [&](const C (&v)[NP], C (&out)[NP]) {   // M v, FP64 sums
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            C t = C(0);
#pragma unroll
            for (int l = 0; l < NP; ++l)
                t += as_f64_here(S.Ml[l <= j ? Tri<NP>::idx(j, l) : Tri<NP>::idx(l, j)]) * v[l];
            out[j] = t;
        }
    };
    C x[NP], p[NP], zprev[NP], Dc[R];
    C fz_prev = C(0);
    int st = 0, lsfail = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        x[j] = C(a[j]);
        p[j] = C(0);
        zprev[j] = C(0);
    }
#pragma unroll
    for (int jj = 0; jj < R; ++jj) Dc[jj] = C(S.D[jj]);
    for (int k = 0;; ++k) {
        C d[NP], Md[NP], F[NP], r[R], wr[R];
        bool changed = false;
#pragma unroll
        for (int j = 0; j < NP; ++j) d[j] = x[j] - C(S.a0[j]);
        mv(d, Md);
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            C t = C(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) t += as_f64_here(S.J[jj][j]) * x[j];
            r[jj] = t - C(S.aref[jj]);
            const bool an = r[jj] < C(0);
            changed |= an != act[jj];
            act[jj] = an;
            wr[jj] = an ? Dc[jj] * r[jj] : C(0);
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            C t = C(0);
#pragma unroll
            for (int jj = 0; jj < R; ++jj) t += as_f64_here(S.J[jj][j]) * wr[jj];
            F[j] = Md[j] + gsum16(t);
        }
        const bool same = (k > 0) && !group_any16(changed);
        C z[NP];
        {
            T Ft[NP], zt[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) Ft[j] = T(F[j]);
            reg_chol_solve<T, NP>(Lm, invm, Ft, zt);
#pragma unroll
            for (int j = 0; j < NP; ++j) z[j] = C(zt[j]);
        }
        C g2 = C(0), fz = C(0), xnorm = C(0), beta = C(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            g2 += F[j] * F[j];
            fz += F[j] * z[j];
            xnorm = fmax(xnorm, fabs(x[j]));
        }
        const C gtol = C(tol) * trM, dtol = C(tol) * (C(1) + xnorm);
        if (g2 <= gtol * gtol || fz <= dtol * dtol * trM) {
            st = ST_CONVERGED;
            break;
        }
        if (k == max_iter) { st = ST_MAXITER; break; }
        if (same && fz_prev > C(0)) {
            C num = C(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) num += F[j] * (z[j] - zprev[j]);
            beta = fmax(C(0), num / fz_prev);
        }
        C fp = C(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            p[j] = -z[j] + beta * p[j];
            fp += F[j] * p[j];
        }
        if (fp >= C(0)) {
#pragma unroll
            for (int j = 0; j < NP; ++j) p[j] = -z[j];
        }
        C q[R];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            C t = C(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) t += as_f64_here(S.J[jj][j]) * p[j];
            q[jj] = t;
        }
        C Mp[NP];
        mv(p, Mp);
        C c0 = C(0), b0 = C(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            c0 += p[j] * Mp[j];
            b0 += Mp[j] * d[j];
        }
        uint32_t bits;
        C cpiece;
        int fail;
        const C alpha = small_line_search<false, C, R>(r, q, Dc, c0, b0, bits, cpiece, fail);
        lsfail |= fail;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            x[j] += alpha * p[j];
            zprev[j] = z[j];
        }
        fz_prev = fz;
        iters = k + 1;
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) a[j] = T(x[j]);
    if (st & (ST_CONVERGED | ST_MAXITER)) {
        // H(A) at the returned iterate (eq. 9), factored for the saved state
        T tj[R][NP];
#pragma unroll
        for (int jj = 0; jj < R; ++jj)
#pragma unroll
            for (int j = 0; j < NP; ++j) tj[jj][j] = (act[jj] ? S.D[jj] : T(0)) * S.J[jj][j];
#pragma unroll
        for (int j = 0; j < NP; ++j)
#pragma unroll
            for (int l = 0; l <= j; ++l) {
                T t = T(0);
#pragma unroll
                for (int jj = 0; jj < R; ++jj) t += tj[jj][j] * S.J[jj][l];
                H[Tri<NP>::idx(j, l)] = S.Ml[Tri<NP>::idx(j, l)] + gsum16(t);
            }
        if (!reg_cholesky<T, NP>(H, inv)) st = ST_NOTSPD;
    }
    if (lsfail) st |= ST_LSFAIL;
    return st;
}

// Final refinement of an FP32 solve that met the stopping rule: one Newton
// step on the converged active set with the gradient F(a) = M (a - a0) +
// J^T (D o A o (J a - aref)) (eq. 6) formed in FP64 and the step solved with
// the factor of H(A) the solve ended with, a <- a - H^{-1} F(a).  The step is
// zero in exact arithmetic (a is the root of F on A); in FP32 it removes the
// iterate's rounding error, which the gradients of eq. 17 would inherit.
template <typename T, int NP, int R>
__device__ inline void small_refine(const SmallInst<T, NP, R> &S, T (&a)[NP],
                                    const T (&L)[Tri<NP>::NE], const T (&inv)[NP],
                                    const bool (&act)[R]) {
    typedef double C;
    C w[R];
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        C s = C(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) s += C(S.J[jj][j]) * C(a[j]);
        w[jj] = act[jj] ? C(S.D[jj]) * (s - C(S.aref[jj])) : C(0);
    }
    T rhs[NP], d[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        C s = C(0), md = C(0);
#pragma unroll
        for (int jj = 0; jj < R; ++jj) s += C(S.J[jj][j]) * w[jj];
#pragma unroll
        for (int l = 0; l < NP; ++l)
            md += C(S.Ml[l <= j ? Tri<NP>::idx(j, l) : Tri<NP>::idx(l, j)]) * (C(a[l]) - C(S.a0[l]));
        rhs[j] = T(-(md + gsum16(s)));
    }
    reg_chol_solve<T, NP>(L, inv, rhs, d);
#pragma unroll
    for (int j = 0; j < NP; ++j) a[j] = T(C(a[j]) + C(d[j]));
}

// Newton: two workgroups per CU (256 VGPRs a lane); the FP64-arithmetic CG
// solve keeps more live state and takes one (512).
template <typename T, int NP, int R, bool CG = false>
__global__ __launch_bounds__(256, CG ? 1 : 2) void k_forward_small(
    BatchView bv, int nb_inst, int max_iter, T tol, const T *__restrict__ gM,
    const T *__restrict__ gJ, const T *__restrict__ ga0, const T *__restrict__ garef,
    const T *__restrict__ gD, const T *__restrict__ gainit, T *__restrict__ gaout,
    T *__restrict__ gfac, uint8_t *__restrict__ gmask, int32_t *__restrict__ gstatus,
    int32_t *__restrict__ giters) {
    constexpr int NE = Tri<NP>::NE;
    const int g = threadIdx.x & (SG - 1);
    const int w = blockIdx.x * (blockDim.x / SG) + threadIdx.x / SG;
    if (w >= nb_inst) return;   // whole groups only: no cross-group traffic follows
    const Inst I = inst_at(bv, w);
    if (!I.ok) {   // group-uniform
        mark_bad(I, gstatus, giters, g == 0);
        return;
    }
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
    T H[NE], inv[NP];
    bool act[R];
    int iters = 0, st;
    if (bad) {
        st = ST_NONFINITE;
#pragma unroll
        for (int jj = 0; jj < R; ++jj) act[jj] = false;
    } else {
        if constexpr (CG)
            st = small_solve_cg<T, NP, R>(S, max_iter, tol, a, H, inv, act, iters);
        else
            st = small_solve<false, T, NP, R>(S, max_iter, tol, a, H, inv, act, iters,
                                              StepTape<T>{nullptr, nullptr, 0, 0, 0});
        if constexpr (sizeof(T) == 4) {
            if (st & ST_CONVERGED) small_refine<T, NP, R>(S, a, H, inv, act);
        }
    }
    const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
    const T nanv = T(__builtin_nan(""));
    {   // lane g < n writes a[g]
        T ag = a[0];
#pragma unroll
        for (int j = 1; j < NP; ++j) ag = (g == j) ? a[j] : ag;
        if (g < S.n) gaout[I.on + g] = ok ? ag : nanv;
    }
    T *fac = gfac + fac_offset(I);
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int l = 0; l <= j; ++l) {
            const int e = Tri<NP>::idx(j, l);
            if ((e & (SG - 1)) == g && j < S.n) fac[e] = ok ? H[e] : nanv;
        }
    const int live = S.m - S.i0;
    uint8_t *mk = gmask + I.om + S.i0;
    if constexpr (R == 4) {
        if (live >= 4 && (reinterpret_cast<uintptr_t>(mk) & 3u) == 0) {
            uint32_t word = 0;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) word |= (ok && act[jj] ? 1u : 0u) << (8 * jj);
            *reinterpret_cast<uint32_t *>(mk) = word;
        } else {
#pragma unroll
            for (int jj = 0; jj < R; ++jj)
                if (jj < live) mk[jj] = (ok && act[jj]) ? 1 : 0;
        }
    } else {
#pragma unroll
        for (int jj = 0; jj < R; ++jj)
            if (jj < live) mk[jj] = (ok && act[jj]) ? 1 : 0;
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
    constexpr int NE = Tri<NP>::NE;
    const int g = threadIdx.x & (SG - 1);
    const int w = blockIdx.x * (blockDim.x / SG) + threadIdx.x / SG;
    if (w >= nb_inst) return;
    const Inst I = inst_at(bv, w);
    if (!I.ok) return;   // group-uniform: outputs untouched
    const int n = I.n, m = I.m;
    __shared__ T sh[(256 / SG) * GroupShm<NP>::SIZE];
    T *gsh = sh + (threadIdx.x / SG) * GroupShm<NP>::SIZE;
    SmallInst<T, NP, R> S;
    T L[NE], inv[NP], a[NP], ab[NP];
    bool act[R];
    if (S.fast_ok(I, g, gJ, garef, gD)) {
        // every load of the instance issued before any use
        const T *fp = gfac + fac_offset(I);
#pragma unroll
        for (int e = 0; e < NE; ++e) L[e] = fp[e];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            a[j] = ga[I.on + j];
            ab[j] = gabar[I.on + j];
        }
        const uint8_t *mk = gmask + I.om + g * R;
        uint8_t mb[R];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) mb[jj] = mk[jj];
        S.load_fast(I, g, gM, gJ, ga0, garef, gD);
#pragma unroll
        for (int jj = 0; jj < R; ++jj) act[jj] = mb[jj] != 0;
    } else {
        S.load_general(I, g, gM, gJ, ga0, garef, gD, gsh + GroupShm<NP>::M0);
        // the factor arrives through LDS: coalesced loads, then group broadcasts
        const T *fac = gsh + GroupShm<NP>::F0;
        group_copy_in(gfac + fac_offset(I), n * (n + 1) / 2, gsh + GroupShm<NP>::F0, g);
        group_sync();
#pragma unroll
        for (int j = 0; j < NP; ++j) {
#pragma unroll
            for (int l = 0; l <= j; ++l)
                L[Tri<NP>::idx(j, l)] = (j < n) ? fac[Tri<NP>::idx(j, l)] : (j == l ? T(1) : T(0));
            a[j] = j < n ? ga[I.on + j] : T(0);
            ab[j] = j < n ? gabar[I.on + j] : T(0);
        }
        const int lv = m - S.i0;
        const uint8_t *mk = gmask + I.om + S.i0;
#pragma unroll
        for (int jj = 0; jj < R; ++jj) act[jj] = jj < lv && mk[jj] != 0;
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) inv[j] = fast_rcp(L[Tri<NP>::idx(j, j)]);
    const int live = m - S.i0;
    // Arithmetic in FP64 whatever the storage type (the FP64 rate equals the
    // unpacked FP32 rate, and this kernel waits on memory): lambda = H^{-1}
    // abar from the stored factor, then two steps of iterative refinement
    // whose residual abar - H lambda, H v = M v + J^T (D o A* o J v), is
    // formed in FP64 from the stored inputs; the corrections are solved with
    // the stored factor.  lambda then carries the accuracy of the inputs,
    // not the factor's condition-number-sized rounding.
    typedef double C;
    C lam[NP];
    {
        T l0[NP];
        reg_chol_solve<T, NP>(L, inv, ab, l0);
#pragma unroll
        for (int j = 0; j < NP; ++j) lam[j] = C(l0[j]);
    }
#pragma unroll 1
    for (int it = 0; it < 2; ++it) {
        C t[R];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            C s = C(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) s += as_f64_here(S.J[jj][j]) * lam[j];
            t[jj] = act[jj] ? as_f64_here(S.D[jj]) * s : C(0);
        }
        T rt[NP], dl[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            C s = C(0), mv = C(0);
#pragma unroll
            for (int jj = 0; jj < R; ++jj) s += as_f64_here(S.J[jj][j]) * t[jj];
#pragma unroll
            for (int l = 0; l < NP; ++l)
                mv += as_f64_here(S.Ml[l <= j ? Tri<NP>::idx(j, l) : Tri<NP>::idx(l, j)]) * lam[l];
            rt[j] = T(as_f64_here(ab[j]) - mv - gsum16(s));
        }
        reg_chol_solve<T, NP>(L, inv, rt, dl);
#pragma unroll
        for (int j = 0; j < NP; ++j) lam[j] += C(dl[j]);
    }
    // per-row cotangents: r* = J a* - aref and sigma = J lambda in FP64
    T arb[R], db[R], Jb[R * NP];
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        C ja = C(0), sig = C(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            ja += C(S.J[jj][j]) * C(a[j]);
            sig += C(S.J[jj][j]) * lam[j];
        }
        const C r = ja - C(S.aref[jj]);
        const C wv = act[jj] ? C(S.D[jj]) * r : C(0);
        const C ar = act[jj] ? C(S.D[jj]) * sig : C(0);
        arb[jj] = T(ar);
        db[jj] = act[jj] ? T(-r * sig) : T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) Jb[jj * NP + j] = T(-(wv * lam[j] + ar * C(a[j])));
    }
    if (garefbar) {
        T *p = garefbar + I.om + S.i0;
        store_run<T, R>(p, live >= R && aligned16(p), live, arb);
    }
    if (gDbar) {
        T *p = gDbar + I.om + S.i0;
        store_run<T, R>(p, live >= R && aligned16(p), live, db);
    }
    if (gJbar) {
        T *p = gJbar + I.omn + (int64_t)S.i0 * n;
        if (S.full) {
            store_run<T, R * NP>(p, aligned16(p), R * NP, Jb);
        } else {
#pragma unroll
            for (int jj = 0; jj < R; ++jj)
#pragma unroll
                for (int j = 0; j < NP; ++j)
                    if (jj < live && j < n) p[(int64_t)jj * n + j] = Jb[jj * NP + j];
        }
    }
    if (ga0bar) {
        C mg = C(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            C s = C(0);
#pragma unroll
            for (int l = 0; l < NP; ++l)
                s += C(S.Ml[l <= j ? Tri<NP>::idx(j, l) : Tri<NP>::idx(l, j)]) * lam[l];
            mg = (g == j) ? s : mg;
        }
        if (g < n) ga0bar[I.on + g] = T(mg);
    }
    if (gMbar) {
        // lambda and a - a0 through LDS; lane g writes entries g, g + 16, ...
        T *vl = gsh + GroupShm<NP>::V0, *vd = gsh + GroupShm<NP>::W0;
        if (g == 0) {
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                vl[j] = T(lam[j]);
                vd[j] = T(C(a[j]) - C(S.a0[j]));
            }
        }
        group_sync();
        T *Mb = gMbar + I.onn;
        int j = g / n, l = g - (g / n) * n;
        const int dj = SG / n, dl = SG - (SG / n) * n;
        for (int e = g; e < n * n; e += SG) {
            Mb[e] = -vl[j] * vd[l];
            j += dj;
            l += dl;
            if (l >= n) { l -= n; ++j; }
        }
    }
}

// Unrolled VJP: the K-step solve with its tape, then the reverse sweep with
// every cotangent accumulated in registers (J-bar rows, D-bar, aref-bar by the
// lane owning the row; M-bar entry f by lane f mod 16).
template <typename T, int NP, int R>
__global__ __launch_bounds__(256) void k_unrolled_small(
    BatchView bv, int nb_inst, int K, int mode, T tol, const T *__restrict__ gM, const T *__restrict__ gJ,
    const T *__restrict__ ga0, const T *__restrict__ garef, const T *__restrict__ gD,
    const T *__restrict__ gabar, T *__restrict__ gaout, T *__restrict__ ga0bar,
    T *__restrict__ garefbar, T *__restrict__ gJbar, T *__restrict__ gDbar, T *__restrict__ gMbar,
    T *__restrict__ tapeT, uint8_t *__restrict__ tapeB, int32_t *__restrict__ gstatus,
    int32_t *__restrict__ giters) {
    constexpr int NE = Tri<NP>::NE;
    constexpr int MBL = (NP * NP + SG - 1) / SG;   // M-bar entries per lane
    const int g = threadIdx.x & (SG - 1);
    const int w = blockIdx.x * (blockDim.x / SG) + threadIdx.x / SG;
    if (w >= nb_inst) return;
    const Inst I = inst_at(bv, w);
    if (!I.ok) {   // group-uniform
        if (mode != ST_REP) mark_bad(I, gstatus, giters, g == 0);
        return;
    }
    const int n = I.n, m = I.m;
    SmallInst<T, NP, R> S;
    S.load(I, g, gM, gJ, ga0, garef, gD);
    T a[NP], ab[NP];
    bool bad = S.bad;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        a[j] = S.a0[j];
        ab[j] = (mode != ST_REC && j < n) ? gabar[I.on + j] : T(0);
        bad |= !finite_val(ab[j]);
    }
    bad = gsum16(bad ? T(1) : T(0)) != T(0);
    const int ne = n * (n + 1) / 2;
    const int recT = 2 * n + ne + 2 * m + 2;
    const StepTape<T> tp{tapeT + tape_T_offset(I, K), tapeB + tape_B_offset(I, K), n, m, recT};
    const T nanv = T(__builtin_nan(""));
    int steps = 0, st;
    if (mode == ST_REP) {
        st = gstatus[I.b];
        steps = giters[I.b];
        if (bad) st |= ST_NONFINITE;
    } else {
        T H[NE], inv[NP];
        bool act[R];
        if (bad) {
            st = ST_NONFINITE;
        } else {
            st = small_solve<true, T, NP, R>(S, K, tol, a, H, inv, act, steps, tp);
        }
        const bool okf = !(st & (ST_NONFINITE | ST_NOTSPD));
#pragma unroll
        for (int j = 0; j < NP; ++j)
            if (j == g && j < n) gaout[I.on + j] = okf ? a[j] : nanv;
        if (g == 0) {
            gstatus[I.b] = st;
            if (giters) giters[I.b] = steps;
        }
        if (mode == ST_REC) return;
    }
    const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));

    // reverse sweep
    T Jb[R][NP], arb[R], db[R], Mb[MBL], a0b[NP];
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        arb[jj] = T(0);
        db[jj] = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) Jb[jj][j] = T(0);
    }
#pragma unroll
    for (int e = 0; e < MBL; ++e) Mb[e] = T(0);
#pragma unroll
    for (int j = 0; j < NP; ++j) a0b[j] = T(0);
    const int live = m - S.i0;
    for (int k = (ok ? steps : 0) - 1; k >= 0; --k) {
        const T *rec = tp.tT + (int64_t)k * recT;
        const uint8_t *recB = tp.tB + (int64_t)k * 2 * m;
        T ak[NP], p[NP], Lk[NE], iv[NP], r[R], q[R];
        bool A[R], Ap[R];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            ak[j] = j < n ? rec[j] : T(0);
            p[j] = j < n ? rec[n + j] : T(0);
#pragma unroll
            for (int l = 0; l <= j; ++l)
                Lk[Tri<NP>::idx(j, l)] = j < n ? rec[2 * n + Tri<NP>::idx(j, l)] : (j == l ? T(1) : T(0));
            iv[j] = fast_rcp(Lk[Tri<NP>::idx(j, j)]);
        }
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            const bool lv = jj < live;
            r[jj] = lv ? rec[2 * n + ne + S.i0 + jj] : T(0);
            q[jj] = lv ? rec[2 * n + ne + m + S.i0 + jj] : T(0);
            A[jj] = lv && recB[S.i0 + jj] != 0;
            Ap[jj] = lv && recB[m + S.i0 + jj] != 0;
        }
        const T alpha = rec[2 * n + ne + 2 * m], c = rec[2 * n + ne + 2 * m + 1];
        T d[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) d[j] = ak[j] - S.a0[j];
        // a_{k+1} = a_k + alpha p with alpha = -b / c
        T alphab = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) alphab += ab[j] * p[j];
        const T bb = -alphab / c;
        const T cb = -alphab * alpha / c;
        T qb[R], rb[R];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            const T dd = S.D[jj];
            qb[jj] = Ap[jj] ? T(2) * cb * dd * q[jj] + bb * dd * r[jj] : T(0);
            rb[jj] = Ap[jj] ? bb * dd * q[jj] : T(0);
            db[jj] += Ap[jj] ? cb * q[jj] * q[jj] + bb * q[jj] * r[jj] : T(0);
        }
        T Mp[NP], Md[NP], pb[NP];
        sym_mv<T, NP>(S.Ml, p, Mp);
        sym_mv<T, NP>(S.Ml, d, Md);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T s = T(0);
#pragma unroll
            for (int jj = 0; jj < R; ++jj) s += S.J[jj][j] * qb[jj];
            pb[j] = alpha * ab[j] + T(2) * cb * Mp[j] + bb * Md[j] + gsum16(s);
        }
        // p = -H^{-1} g: u = H^{-1} pbar, gbar = -u, Hbar = -u p^T
        T u[NP];
        reg_chol_solve<T, NP>(Lk, iv, pb, u);
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            T ju = T(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) ju += S.J[jj][j] * u[j];
            const T dd = S.D[jj];
            db[jj] += A[jj] ? -ju * (q[jj] + r[jj]) : T(0);
            rb[jj] += A[jj] ? -dd * ju : T(0);
            const T cp = qb[jj] - (A[jj] ? dd * ju : T(0));
            const T cu = A[jj] ? -dd * (q[jj] + r[jj]) : T(0);
            arb[jj] -= rb[jj];
#pragma unroll
            for (int j = 0; j < NP; ++j) Jb[jj][j] += cp * p[j] + cu * u[j] + rb[jj] * ak[j];
        }
        T Mu[NP];
        sym_mv<T, NP>(S.Ml, u, Mu);
#pragma unroll
        for (int e = 0; e < MBL; ++e) {
            const int f = g + SG * e;
            if (f < NP * NP) {
                const int j = f / NP, l = f % NP;
                Mb[e] += p[j] * (cb * p[l] + bb * d[l]) - u[j] * (p[l] + d[l]);
            }
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T s = T(0);
#pragma unroll
            for (int jj = 0; jj < R; ++jj) s += S.J[jj][j] * rb[jj];
            const T through_m = bb * Mp[j] - Mu[j];
            ab[j] = ab[j] + through_m + gsum16(s);
            a0b[j] -= through_m;
        }
    }
#pragma unroll
    for (int j = 0; j < NP; ++j)
        if (j == g && j < n) ga0bar[I.on + j] = ok ? a0b[j] + ab[j] : nanv;
    {
        T *p1 = garefbar + I.om + S.i0, *p2 = gDbar + I.om + S.i0;
        store_run<T, R>(p1, live >= R && aligned16(p1), live, arb);
        store_run<T, R>(p2, live >= R && aligned16(p2), live, db);
        T *pj = gJbar + I.omn + (int64_t)S.i0 * n;
        if (S.full) {
            T flat[R * NP];
#pragma unroll
            for (int jj = 0; jj < R; ++jj)
#pragma unroll
                for (int j = 0; j < NP; ++j) flat[jj * NP + j] = Jb[jj][j];
            store_run<T, R * NP>(pj, aligned16(pj), R * NP, flat);
        } else {
#pragma unroll
            for (int jj = 0; jj < R; ++jj)
#pragma unroll
                for (int j = 0; j < NP; ++j)
                    if (jj < live && j < n) pj[(int64_t)jj * n + j] = Jb[jj][j];
        }
        T *pm = gMbar + I.onn;
#pragma unroll
        for (int e = 0; e < MBL; ++e) {
            const int f = g + SG * e;
            if (f < NP * NP) {
                const int j = f / NP, l = f % NP;
                if (j < n && l < n) pm[j * n + l] = ok ? Mb[e] : nanv;
            }
        }
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
inline bool small_supported(int nmax, int mmax, int s) {
    const int np = small_np(nmax);
    return np != 0 && small_r(mmax) != 0 && (s == 4 ? np <= 12 : np <= 6);
}

// The unrolled kernel also keeps the J-bar rows and M-bar in registers.
inline bool small_unrolled_supported(int nmax, int mmax, int s) {
    const int np = small_np(nmax);
    return np != 0 && small_r(mmax) != 0 && (s == 4 ? np <= 9 : np <= 6);
}

#define CS_SMALL_DISPATCH(NPV, RV, CALL)                                                      \
    if (np == NPV && rr == RV) { CALL(NPV, RV); }

#define CS_SMALL_F64(CALL)                                                                    \
    CS_SMALL_DISPATCH(3, 1, CALL) else CS_SMALL_DISPATCH(3, 2, CALL) else CS_SMALL_DISPATCH(3, 4, CALL) \
    else CS_SMALL_DISPATCH(6, 1, CALL) else CS_SMALL_DISPATCH(6, 2, CALL) else CS_SMALL_DISPATCH(6, 4, CALL) \
    else { return -4; }

#define CS_SMALL_F32_9(CALL)                                                                  \
    CS_SMALL_DISPATCH(3, 1, CALL) else CS_SMALL_DISPATCH(3, 2, CALL) else CS_SMALL_DISPATCH(3, 4, CALL) \
    else CS_SMALL_DISPATCH(6, 1, CALL) else CS_SMALL_DISPATCH(6, 2, CALL) else CS_SMALL_DISPATCH(6, 4, CALL) \
    else CS_SMALL_DISPATCH(9, 1, CALL) else CS_SMALL_DISPATCH(9, 2, CALL) else CS_SMALL_DISPATCH(9, 4, CALL) \
    else { return -4; }

#define CS_SMALL_F32_12(CALL)                                                                 \
    CS_SMALL_DISPATCH(3, 1, CALL) else CS_SMALL_DISPATCH(3, 2, CALL) else CS_SMALL_DISPATCH(3, 4, CALL) \
    else CS_SMALL_DISPATCH(6, 1, CALL) else CS_SMALL_DISPATCH(6, 2, CALL) else CS_SMALL_DISPATCH(6, 4, CALL) \
    else CS_SMALL_DISPATCH(9, 1, CALL) else CS_SMALL_DISPATCH(9, 2, CALL) else CS_SMALL_DISPATCH(9, 4, CALL) \
    else CS_SMALL_DISPATCH(12, 1, CALL) else CS_SMALL_DISPATCH(12, 2, CALL) else CS_SMALL_DISPATCH(12, 4, CALL) \
    else { return -4; }

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
    if constexpr (sizeof(T) == 4) { CS_SMALL_F32_12(CS_CALL_FWD) } else { CS_SMALL_F64(CS_CALL_FWD) }
#undef CS_CALL_FWD
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// The conjugate-gradient forward (small_solve_cg) in the same kernel shell.
template <typename T>
int launch_small_forward_cg(const BatchView &bv, int nmax, int mmax, int max_iter, T tol,
                            const T *M, const T *J, const T *a0, const T *aref, const T *D,
                            const T *a_init, T *a_out, T *fac, uint8_t *mask, int32_t *status,
                            int32_t *iters, hipStream_t stream) {
    const int np = small_np(nmax), rr = small_r(mmax);
    const int nb = bv.B;
    const dim3 grid((nb + 15) / 16), block(256);
#define CS_CALL_FWD_CG(NPV, RV)                                                               \
    hipLaunchKernelGGL((k_forward_small<T, NPV, RV, true>), grid, block, 0, stream, bv, nb,    \
                       max_iter, tol, M, J, a0, aref, D, a_init, a_out, fac, mask, status, iters);
    if constexpr (sizeof(T) == 4) { CS_SMALL_F32_12(CS_CALL_FWD_CG) } else { CS_SMALL_F64(CS_CALL_FWD_CG) }
#undef CS_CALL_FWD_CG
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
    if constexpr (sizeof(T) == 4) { CS_SMALL_F32_12(CS_CALL_VJP) } else { CS_SMALL_F64(CS_CALL_VJP) }
#undef CS_CALL_VJP
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <typename T>
int launch_small_unrolled(const BatchView &bv, int nmax, int mmax, int K, int mode, T tol, const T *M,
                          const T *J, const T *a0, const T *aref, const T *D, const T *abar,
                          T *a_out, T *a0bar, T *arefbar, T *Jbar, T *Dbar, T *Mbar, T *tapeT,
                          uint8_t *tapeB, int32_t *status, int32_t *iters, hipStream_t stream) {
    const int np = small_np(nmax), rr = small_r(mmax);
    const int nb = bv.B;
    const dim3 grid((nb + 15) / 16), block(256);
#define CS_CALL_UNR(NPV, RV)                                                                  \
    hipLaunchKernelGGL((k_unrolled_small<T, NPV, RV>), grid, block, 0, stream, bv, nb, K, mode, tol, M, \
                       J, a0, aref, D, abar, a_out, a0bar, arefbar, Jbar, Dbar, Mbar, tapeT,      \
                       tapeB, status, iters);
    if constexpr (sizeof(T) == 4) { CS_SMALL_F32_9(CS_CALL_UNR) } else { CS_SMALL_F64(CS_CALL_UNR) }
#undef CS_CALL_UNR
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cs
