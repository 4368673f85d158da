// cs_device.hpp -- device building blocks shared by the contact-solve kernels.
//
// A "team" is the NT threads of one workgroup working on one instance at a
// time.  Team reductions are wave butterflies (fixed order, so results are
// bitwise reproducible) followed, for NT > 64, by a pass over per-wave
// partials in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace cs {

enum : int {
    ST_CONVERGED = 1,
    ST_MAXITER = 2,
    ST_NONFINITE = 4,
    ST_NOTSPD = 8,
    ST_LSFAIL = 16,
};

// cs_unrolled_vjp phases (cs_solver_params.flags)
enum : int { ST_BOTH = 0, ST_REC = 1, ST_REP = 2 };

// Device view of the batch descriptor.
struct BatchView {
    int B, nv_u, nr_u;
    const int32_t *nv, *nr;
    const int64_t *off_nn, *off_mn, *off_n, *off_m;
    const int32_t *order;
};

// One instance's shape and element offsets.
struct Inst {
    int b, n, m;
    int64_t onn, omn, on, om;
};

__device__ inline Inst inst_at(const BatchView &bv, int w) {
    Inst I;
    I.b = bv.order ? bv.order[w] : w;
    if (bv.nv) {
        I.n = bv.nv[I.b];
        I.m = bv.nr[I.b];
        I.onn = bv.off_nn[I.b];
        I.omn = bv.off_mn[I.b];
        I.on = bv.off_n[I.b];
        I.om = bv.off_m[I.b];
    } else {
        const int64_t b = I.b;
        I.n = bv.nv_u;
        I.m = bv.nr_u;
        I.onn = b * I.n * I.n;
        I.omn = b * I.m * I.n;
        I.on = b * I.n;
        I.om = b * I.m;
    }
    return I;
}

// Layouts shared by every kernel family.
//  state: factor region, instance i's Cholesky factor of H(A*) as a packed
//  lower triangle (entry (j, l), l <= j, at j (j + 1) / 2 + l) starting at
//  element (off_nn[i] + off_n[i]) / 2 = sum_{b < i} n_b (n_b + 1) / 2; then
//  (256-byte aligned) one byte of A* per row at off_m[i].
//  tape: T region, instance i's K records start at element
//  K (2 off_n + (off_nn + off_n) / 2 + 2 off_m + 2 i), each record being
//  [a_k (n) | p_k (n) | L_k (n (n + 1) / 2) | r_k (m) | q_k (m) | alpha_k | c_k];
//  byte region (256-byte aligned after it): K records [A_k (m) | A'_k (m)]
//  at K 2 off_m[i].
__host__ __device__ inline int64_t rec_T_elems(int n, int m) {
    return 2 * (int64_t)n + (int64_t)n * (n + 1) / 2 + 2 * (int64_t)m + 2;
}
__device__ inline int64_t fac_offset(const Inst &I) { return (I.onn + I.on) / 2; }
__device__ inline int64_t tape_T_offset(const Inst &I, int K) {
    return (int64_t)K * (2 * I.on + (I.onn + I.on) / 2 + 2 * I.om + 2 * (int64_t)I.b);
}
__device__ inline int64_t tape_B_offset(const Inst &I, int K) { return (int64_t)K * 2 * I.om; }

// Raise a kernel's dynamic-LDS limit once; later launches (for instance inside
// a captured HIP graph) make no runtime call.  Returns false on a HIP error.
inline bool ensure_lds(const void *kernel, size_t lds) {
    static std::mutex mu;
    static const void *keys[128];
    static size_t vals[128];
    static int nk = 0;
    std::lock_guard<std::mutex> lock(mu);
    int i = 0;
    while (i < nk && keys[i] != kernel) ++i;
    if (i < nk && vals[i] >= lds) return true;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
        return false;
    if (i == nk && nk < 128) keys[nk++] = kernel;
    if (i < 128) vals[i] = lds;
    return true;
}

template <typename T> __device__ inline T inf_val();
template <> __device__ inline float inf_val<float>() { return __builtin_huge_valf(); }
template <> __device__ inline double inf_val<double>() { return __builtin_huge_val(); }

template <typename T> __device__ inline bool finite_val(T x) { return __builtin_isfinite(x); }

template <typename T> __device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T> __device__ inline T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, 64);
        v = v > u ? v : u;
    }
    return v;
}

// Sum NV values over the team; every thread receives the totals.
// sred must hold NV * (NT / 64) elements.
template <int NT, typename T, int NV>
__device__ inline void team_sum(T (&v)[NV], T *sred) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if constexpr (NT > 64) {
        constexpr int NW = NT / 64;
        const int w = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k) sred[k * NW + w] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            T s = T(0);
#pragma unroll
            for (int i = 0; i < NW; ++i) s += sred[k * NW + i];
            v[k] = s;
        }
    }
}

// In-place Cholesky H = L L^T of the n x n row-major matrix in LDS (lower
// triangle read and overwritten strictly below the diagonal; the diagonal of
// L goes to diag[]).  Left-looking by columns, one barrier per column.
// Returns false (team-uniform) when a pivot is not positive.
// The matrix has row stride ld (ld = n for a dense n x n block).
template <int NT, typename T>
__device__ inline bool team_cholesky(T *H, T *diag, int n, int ld) {
    bool ok = true;
    for (int j = 0; j < n; ++j) {
        T s = H[j * ld + j];
        for (int k = 0; k < j; ++k) s -= H[j * ld + k] * H[j * ld + k];
        ok = ok && (s > T(0));
        const T ljj = sqrt(s);
        const T inv = T(1) / ljj;
        for (int i = j + 1 + (int)threadIdx.x; i < n; i += NT) {
            T t = H[i * ld + j];
            for (int k = 0; k < j; ++k) t -= H[i * ld + k] * H[j * ld + k];
            H[i * ld + j] = t * inv;
        }
        if ((int)threadIdx.x == (j % NT)) diag[j] = ljj;
        __syncthreads();
    }
    return ok;
}
template <int NT, typename T>
__device__ inline bool team_cholesky(T *H, T *diag, int n) { return team_cholesky<NT>(H, diag, n, n); }

// Solve L L^T x = b with the factor from team_cholesky.  b is overwritten;
// the solution is returned in x.  One barrier per column and direction.
template <int NT, typename T>
__device__ inline void team_chol_solve(const T *L, const T *diag, T *b, T *x, int n, int ld) {
    // forward: L y = b, y stored in x
    for (int j = 0; j < n; ++j) {
        const T yj = b[j] / diag[j];
        if ((int)threadIdx.x == (j % NT)) x[j] = yj;
        for (int i = j + 1 + (int)threadIdx.x; i < n; i += NT) b[i] -= L[i * ld + j] * yj;
        __syncthreads();
    }
    // backward: L^T x = y (in place in x)
    for (int j = n - 1; j >= 0; --j) {
        const T xj = x[j] / diag[j];
        __syncthreads();
        if ((int)threadIdx.x == (j % NT)) x[j] = xj;
        for (int i = (int)threadIdx.x; i < j; i += NT) x[i] -= L[j * ld + i] * xj;
        __syncthreads();
    }
}
template <int NT, typename T>
__device__ inline void team_chol_solve(const T *L, const T *diag, T *b, T *x, int n) {
    team_chol_solve<NT>(L, diag, b, x, n, n);
}

// Exact line search along p (Sec. III-B, eq. 10): the minimiser of
// phi(t) = L(a + t p), i.e. the root of the continuous, strictly increasing,
// piecewise-linear phi'(t) = c0 t + b0 + sum_i D_i q_i min(r_i + t q_i, 0)
// with c0 = p^T M p, b0 = p^T M (a - a0), q = J p.
//
// Safeguarded piece Newton: at a trial t the active rows {r + t q < 0} fix a
// line phi' = c t + b; its root -b/c is accepted when the active rows there
// are the same (it is then the exact root); otherwise the trial moves to the
// root (inside the bracket) or to the bracket midpoint; a bracket narrower
// than rounding ends the search at the current trial.  Rows belong to
// threads as i = tid + NT * jj (jj < 32, so m <= 32 NT).
// Returns alpha; bits_out gets this thread's rows of the accepted piece,
// c_out that piece's slope.  fail is set when the safeguard cap was hit.
template <int NT, typename T>
__device__ inline T team_line_search(int m, const T *r, const T *q, const T *D, T c0, T b0,
                                     T *sred, uint32_t &bits_out, T &c_out, int &fail) {
    const int tid = threadIdx.x;
    T t = T(1);
    uint32_t bits = 0;
    T c, b;
    {
        T v[2] = {T(0), T(0)};
        for (int i = tid, jj = 0; i < m; i += NT, ++jj) {
            const T qi = q[i], ri = r[i];
            if (ri + t * qi < T(0)) {
                const T dq = D[i] * qi;
                v[0] += dq * qi;
                v[1] += dq * ri;
                bits |= 1u << jj;
            }
        }
        team_sum<NT>(v, sred);
        c = c0 + v[0];
        b = b0 + v[1];
    }
    T lo = T(0), hi = inf_val<T>();
    T alpha = t;
    fail = 1;
    const T eps = T(sizeof(T) == 4 ? 1.1920929e-7 : 2.220446049250313e-16);
    for (int it = 0; it < 96; ++it) {
        const T g = c * t + b;
        if (g == T(0)) { alpha = t; fail = 0; break; }
        if (g < T(0)) lo = t; else hi = t;
        // the root lies within rounding of a breakpoint: the two adjacent pieces
        // disagree only by rounding, take the current trial
        if (hi < inf_val<T>() && hi - lo <= T(32) * eps * hi) { alpha = t; fail = 0; break; }
        T cand = -b / c;
        const bool newton = (cand > lo) && (cand < hi);
        if (!newton) cand = (hi < inf_val<T>()) ? T(0.5) * (lo + hi) : T(2) * lo + T(1);
        uint32_t nb = 0;
        T v[3] = {T(0), T(0), T(0)};
        for (int i = tid, jj = 0; i < m; i += NT, ++jj) {
            const T qi = q[i], ri = r[i];
            if (ri + cand * qi < T(0)) {
                const T dq = D[i] * qi;
                v[0] += dq * qi;
                v[1] += dq * ri;
                nb |= 1u << jj;
            }
        }
        v[2] = T(__builtin_popcount(nb ^ bits));
        team_sum<NT>(v, sred);
        bits = nb;
        c = c0 + v[0];
        b = b0 + v[1];
        t = cand;
        alpha = cand;
        if (newton && v[2] == T(0)) { fail = 0; break; }
    }
    bits_out = bits;
    c_out = c;
    return alpha;
}

}  // namespace cs
