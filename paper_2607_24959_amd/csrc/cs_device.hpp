// cs_device.hpp -- device building blocks shared by the contact-solve kernels.
//
// A "team" is the NT threads of one workgroup working on one instance at a
// time.  Team reductions are wave butterflies (fixed order, so results are
// bitwise reproducible) followed, for NT > 64, by a pass over per-wave
// partials in LDS.
#pragma once

#include <type_traits>

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
    ST_BADDESC = 32,
};

// cs_unrolled_vjp phases (cs_solver_params.flags)
enum : int { ST_BOTH = 0, ST_REC = 1, ST_REP = 2 };

// Device view of the batch descriptor.  B is the number of instances a
// launch walks (order[0 .. B-1]); Bfull, nmax, mmax and the totals are what
// the launch was sized for (the host describes them).
struct BatchView {
    int B, nv_u, nr_u;
    const int32_t *nv, *nr;
    const int64_t *off_nn, *off_mn, *off_n, *off_m;
    const int32_t *order;
    int Bfull, nmax, mmax;
    int64_t tot_nn, tot_mn, tot_n, tot_m;
};

// One instance's shape and element offsets.  ok: the descriptor is well
// formed (below); bvalid: the instance index itself is in range, so its
// status word may be written.
struct Inst {
    int b, n, m;
    int64_t onn, omn, on, om;
    bool ok, bvalid;
};

// A packed instance's descriptor is well formed when its shape fits what the
// launch was sized for and every array it addresses lies inside the batch's
// totals: 1 <= n <= nmax, 0 <= m <= mmax, offsets >= 0 and offset + extent
// <= total for M (n^2), J (m n), the n-vectors and the m-vectors (the saved
// factor, the active set and the tape follow from these).
__host__ __device__ inline bool desc_ok(int n, int m, int64_t onn, int64_t omn, int64_t on,
                                        int64_t om, int nmax, int mmax, int64_t tot_nn,
                                        int64_t tot_mn, int64_t tot_n, int64_t tot_m) {
    return n >= 1 && n <= nmax && m >= 0 && m <= mmax && onn >= 0 && omn >= 0 && on >= 0 &&
           om >= 0 && onn <= tot_nn - (int64_t)n * n && omn <= tot_mn - (int64_t)m * n &&
           on <= tot_n - n && om <= tot_m - m;
}

__device__ inline Inst inst_at(const BatchView &bv, int w) {
    Inst I;
    I.b = bv.order ? bv.order[w] : w;
    I.bvalid = I.b >= 0 && I.b < bv.Bfull;
    I.n = 1;
    I.m = 0;
    I.onn = I.omn = I.on = I.om = 0;
    if (!I.bvalid) {
        I.ok = false;
        return I;
    }
    if (bv.nv) {
        I.n = bv.nv[I.b];
        I.m = bv.nr[I.b];
        I.onn = bv.off_nn[I.b];
        I.omn = bv.off_mn[I.b];
        I.on = bv.off_n[I.b];
        I.om = bv.off_m[I.b];
        I.ok = desc_ok(I.n, I.m, I.onn, I.omn, I.on, I.om, bv.nmax, bv.mmax, bv.tot_nn, bv.tot_mn,
                       bv.tot_n, bv.tot_m);
    } else {
        const int64_t b = I.b;
        I.n = bv.nv_u;
        I.m = bv.nr_u;
        I.onn = b * I.n * I.n;
        I.omn = b * I.m * I.n;
        I.on = b * I.n;
        I.om = b * I.m;
        I.ok = true;
    }
    return I;
}

// A malformed descriptor is reported in the instance's status word (when the
// instance index is in range) and the instance is skipped.
__device__ inline void mark_bad(const Inst &I, int32_t *status, int32_t *iters, bool leader) {
    if (leader && I.bvalid) {
        if (status) status[I.b] = ST_BADDESC;
        if (iters) iters[I.b] = 0;
    }
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

// Wave-wide sum and max for a fully active wave, every lane receiving the
// result: DPP within each row of 16 lanes (quad xor 1 and 2, half-row and row
// mirrors; the value stays in vector registers), then the four row results
// from lanes 0, 16, 32 and 48 by lane reads.  Fixed order: reproducible.
template <int CTRL> __device__ inline float dpp_row(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ inline double dpp_row(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline float lane_read(float v, int k) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}
__device__ inline double lane_read(double v, int k) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename T> __device__ inline T wave_sum(T v) {
    v += dpp_row<0xB1>(v);
    v += dpp_row<0x4E>(v);
    v += dpp_row<0x141>(v);
    v += dpp_row<0x140>(v);
    return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

template <typename T> __device__ inline T wave_max(T v) {
    auto mx = [](T x, T y) { return x > y ? x : y; };
    v = mx(v, dpp_row<0xB1>(v));
    v = mx(v, dpp_row<0x4E>(v));
    v = mx(v, dpp_row<0x141>(v));
    v = mx(v, dpp_row<0x140>(v));
    return mx(mx(lane_read(v, 0), lane_read(v, 16)), mx(lane_read(v, 32), lane_read(v, 48)));
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

// Value of v in lane k of the wave (k wave-uniform), for every lane.
__device__ inline float lane_bcast(float v, int k) {
    k = __builtin_amdgcn_readfirstlane(k);
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}
__device__ inline double lane_bcast(double v, int k) {
    k = __builtin_amdgcn_readfirstlane(k);
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Value of v in lane k of the lane's own row of 16 (k a compile-time
// constant), by a DPP row broadcast: the result stays in a vector register.
template <int K> __device__ inline float row_bcast16(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + K, 0xF, 0xF, false));
}
template <int K> __device__ inline double row_bcast16(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x150 + K, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + K, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Compile-time loop: f(integral_constant<int, I>) for I = 0 .. N-1.
template <int I, int N, typename F> __device__ inline void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Trailing update of the blocked Cholesky: for c1 <= j <= i < n,
//   H[i][j] -= sum_{k < 16} H[i][c0 + k] H[j][c0 + k]
// over 16 x 16 tiles of the lower triangle (tile origin c1).  FP32 runs each
// tile on the matrix cores (v_mfma_f32_16x16x4f32, four K-slices of 4; lane l
// feeds row l % 16, slice column l / 16, and receives rows 4 (l / 16) + r);
// FP64 gives each thread whole entries on the VALU.
template <int NT>
__device__ inline void chol_trailing(float *H, int n, int ld, int c0, int c1) {
    const int nt = (n - c1 + 15) / 16;
    const int ntiles = nt * (nt + 1) / 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    for (int t = wave; t < ntiles; t += NT / 64) {
        int ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        const int tj = t - ti * (ti + 1) / 2;
        const int ra = c1 + 16 * ti + li, rb = c1 + 16 * tj + li;
        const int col = c1 + 16 * tj + li;
        // every load (operands and the entries updated) issued before any
        // use, from clamped addresses; the empty asm keeps the compiler from
        // turning each into a branch that waits for it
        float a[4], b[4], h[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kc = c0 + 4 * ks + lk;
            a[ks] = H[min(ra, n - 1) * ld + kc];
            b[ks] = H[min(rb, n - 1) * ld + kc];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            h[r] = H[min(c1 + 16 * ti + 4 * lk + r, n - 1) * ld + min(col, n - 1)];
#pragma unroll
        for (int q = 0; q < 4; ++q) asm volatile("" : "+v"(a[q]), "+v"(b[q]), "+v"(h[q]));
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ra < n ? a[ks] : 0.f, rb < n ? b[ks] : 0.f,
                                                       acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = c1 + 16 * ti + 4 * lk + r;
            if (row < n && col <= row) H[row * ld + col] = h[r] - acc[r];
        }
    }
}

template <int NT>
__device__ inline void chol_trailing(double *H, int n, int ld, int c0, int c1) {
    const int nt = (n - c1 + 15) / 16;
    const int cnt = nt * (nt + 1) / 2 * 256;
    for (int e = threadIdx.x; e < cnt; e += NT) {
        const int t = e >> 8, w = e & 255;
        int ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        const int tj = t - ti * (ti + 1) / 2;
        const int row = c1 + 16 * ti + (w >> 4), col = c1 + 16 * tj + (w & 15);
        if (row < n && col <= row) {
            const double *hr = H + row * ld + c0, *hc = H + col * ld + c0;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) s += hr[k] * hc[k];
            H[row * ld + col] -= s;
        }
    }
}

// The team routines below work on the launching kernel's dynamic LDS (every
// caller carves its LDS from that one region) and are inlined into every
// caller: no call boundary, so no callee addresses the kernel's dynamic LDS
// through a pointer or a base handed across a call.  They take element
// offsets into that region and rebuild their pointers against the LDS
// symbol, which keeps every access a ds_* instruction.
template <typename T> __device__ inline T *lds_at(int off) {
    extern __shared__ __align__(16) unsigned char smem[];
    return reinterpret_cast<T *>(smem) + off;
}
template <typename T> __device__ inline int lds_off(const T *p) {
    extern __shared__ __align__(16) unsigned char smem[];
    return (int)(p - reinterpret_cast<const T *>(smem));
}

// 1 / sqrt(x) for a positive, normal pivot: the hardware estimate refined by
// two Newton steps r <- r + r (1 - x r^2) / 2 in FP64 (quadratic convergence
// from the estimate's ~2^-22 to rounding level); FP32 takes the estimate.
__device__ inline double wave_rsq(double x) {
    double r = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * r, r, 1.0);
        r = fma(0.5 * r, e, r);
    }
    return r;
}
__device__ inline float wave_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
template <typename T> __device__ inline T chol_rcp(T x);
template <> __device__ inline float chol_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double chol_rcp<double>(double x) { return 1.0 / x; }

// The lane index as a value the compiler cannot treat as loop-invariant.
// Lane masks such as (l == j) for every compile-time j would otherwise be
// hoisted out of loops and held in scalar register pairs, more of them than
// the scalar file holds (they then spill through vector lanes).
__device__ inline int opaque_lane(int l) {
    asm volatile("" : "+v"(l));
    return l;
}

// In-place Cholesky H = L L^T of the n x n row-major matrix in LDS (row
// stride ld): the lower triangle is read, L is written strictly below the
// diagonal and L_jj goes to diag[j].  Right-looking over 16-column blocks:
// every wave factors the diagonal block in registers (one row per lane,
// DPP row broadcasts); wave 0 stores L_D and the 16 reciprocals 1 / L_jj (to
// work).  Each panel row below the block is then a triangular solve
// l_i L_D^T = h_i done by one thread in registers (L_D read from LDS as a
// broadcast), and the trailing lower triangle takes the block's rank-16
// update.  Odd row strides keep the panel rows of a wave in distinct LDS
// banks.  n <= 128 for NT = 256.  The caller has synchronised the team after
// writing H.  Returns false (team-uniform) when a pivot is not positive.
template <int NT, typename T>
__device__ __attribute__((always_inline)) inline bool team_cholesky_lds(int ho, int dgo, int n, int ld, int wko) {
    // sizes are team-uniform: keep them (and every branch on them) scalar
    n = __builtin_amdgcn_readfirstlane(n);
    ld = __builtin_amdgcn_readfirstlane(ld);
    T *H = lds_at<T>(__builtin_amdgcn_readfirstlane(ho));
    T *diag = lds_at<T>(__builtin_amdgcn_readfirstlane(dgo));
    T *work = lds_at<T>(__builtin_amdgcn_readfirstlane(wko));
    bool ok = true;
    for (int c0 = 0; c0 < n; c0 += 16) {
        const int bs = min(16, n - c0);
        {
            const int l = threadIdx.x & 63;
            const bool w0 = threadIdx.x < 64;
            // Row l of the block (clamped, always in-bounds loads; the empty
            // asm keeps the compiler from sinking each load into a branch of
            // its own that waits for it).  Entries above the diagonal and
            // rows past the block hold whatever H holds there: the lower
            // triangle of rows < bs never reads them (each update of L_lk,
            // k <= l, reads L_kj and L_lj with j < k), and nothing else is
            // stored from them.  Lanes 16..63 repeat rows of their own row
            // of 16 and store nothing.
            T d[16];
            const T *hr = H + (c0 + min(l & 15, bs - 1)) * ld + c0;
#pragma unroll
            for (int k = 0; k < 16; ++k) d[k] = hr[min(k, bs - 1)];
#pragma unroll
            for (int k = 0; k < 16; ++k) asm volatile("" : "+v"(d[k]));
            // every wave has its copy before wave 0 stores the factored rows
            // (each wave's ok below comes from its own copy, so all must see
            // the same block)
            __syncthreads();
            // right-looking, one DPP row broadcast per entry; columns past bs
            // take pivot 1
            static_for<0, 16>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const T pv = row_bcast16<j>(d[j]);
                d[j] *= wave_rsq((j < bs) ? pv : T(1));
                static_for<j + 1, 16>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    d[k] -= d[j] * row_bcast16<k>(d[j]);
                });
            });
            T dl = d[0];   // this lane's L_ll, picked in one pass
            const int lo = opaque_lane(l & 15);
#pragma unroll
            for (int k = 1; k < 16; ++k) dl = (k == lo) ? d[k] : dl;
            // every wave holds the whole block: positive definiteness from a
            // ballot of the block's diagonal (NaN fails), no LDS round trip
            ok = ok && __builtin_amdgcn_ballot_w64(l < bs && !(dl > T(0))) == 0;
            // whole rows of the block (a team-uniform bound, no lane masks):
            // the block's upper triangle in H is free storage (readers take L
            // strictly below the diagonal and L_jj from diag)
            if (w0 && l < bs) {
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    if (k < bs) H[(c0 + l) * ld + c0 + k] = d[k];
                diag[c0 + l] = dl;
            }
            if (w0 && l < bs) work[l] = chol_rcp(dl);
        }
        __syncthreads();
        const int c1 = c0 + bs;
        if (c1 < n) {
            // panel: row i solves l_i L_D^T = h_i, right-looking (each l_ik
            // feeds the later entries of the row at once).  Only the last
            // block has bs < 16, and it has no panel.
            for (int i = c1 + (int)threadIdx.x; i < n; i += NT) {
                T h[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) h[k] = H[i * ld + c0 + k];
                static_for<0, 16>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    const T lk = h[k] * work[k];
                    h[k] = lk;
                    static_for<k + 1, 16>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        h[j] -= lk * H[(c0 + j) * ld + c0 + k];
                    });
                });
#pragma unroll
                for (int k = 0; k < 16; ++k) H[i * ld + c0 + k] = h[k];
            }
            __syncthreads();
            chol_trailing<NT>(H, n, ld, c0, c1);
            __syncthreads();
        }
    }
    return ok;
}

// Solve L L^T x = b with the factor from team_cholesky.  b is overwritten;
// the solution is returned in x.  Blocked like the factorisation: wave 0
// solves each 16 x 16 diagonal block with DPP row broadcasts, then every thread
// updates one remaining entry with the block's 16 values; two barriers per
// block and direction.  The caller has synchronised the team after writing b.
template <int NT, typename T>
__device__ __attribute__((always_inline)) inline void team_chol_solve_lds(int lo, int dgo, int bo, int xo, int n,
                                                             int ld) {
    n = __builtin_amdgcn_readfirstlane(n);
    ld = __builtin_amdgcn_readfirstlane(ld);
    const T *L = lds_at<T>(__builtin_amdgcn_readfirstlane(lo));
    const T *diag = lds_at<T>(__builtin_amdgcn_readfirstlane(dgo));
    T *b = lds_at<T>(__builtin_amdgcn_readfirstlane(bo));
    T *x = lds_at<T>(__builtin_amdgcn_readfirstlane(xo));
    // forward: L y = b, y stored in x
    for (int c0 = 0; c0 < n; c0 += 16) {
        const int bs = min(16, n - c0);
        if (threadIdx.x < 64) {
            const int l = threadIdx.x;
            const int lr = c0 + min(l, bs - 1);       // clamped row: loads stay in bounds
            T y = b[lr];
            // the lane's row of the block up front (clamped columns) and the
            // reciprocal of its own pivot, then 16 unrolled steps; lanes past
            // the block never store and only feed broadcasts read by such lanes
            T lrow[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) lrow[c] = L[lr * ld + c0 + min(c, bs - 1)];
            const T rdl = chol_rcp(diag[lr]);
            static_for<0, 16>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                const T yc = row_bcast16<c>(y * rdl);   // y_c = (lane c's value) / L_cc
                y = (l == c) ? yc : ((l > c) ? y - lrow[c] * yc : y);
            });
            if (l < bs) x[c0 + l] = y;
        }
        __syncthreads();
        const int c1 = c0 + bs;
        if (c1 < n) {
            for (int i = c1 + (int)threadIdx.x; i < n; i += NT) {
                T v = b[i];
#pragma unroll
                for (int k = 0; k < 16; ++k) v -= L[i * ld + c0 + k] * x[c0 + k];
                b[i] = v;
            }
            __syncthreads();
        }
    }
    // backward: L^T x = y (in place in x)
    const int nb = (n + 15) / 16;
    for (int kb = nb - 1; kb >= 0; --kb) {
        const int c0 = 16 * kb, bs = min(16, n - c0);
        if (threadIdx.x < 64) {
            const int l = threadIdx.x;
            const int lc = c0 + min(l, bs - 1);       // clamped column: loads stay in bounds
            T v = x[lc];
            T lcol[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) lcol[c] = L[(c0 + min(c, bs - 1)) * ld + lc];
            const T rdl = chol_rcp(diag[lc]);
            // columns past the block update nobody (c < bs), so the lanes of
            // the block see exactly the bs steps
            static_for<0, 16>([&](auto ic) {
                constexpr int c = 15 - decltype(ic)::value;
                const T xc = row_bcast16<c>(v * rdl);
                v = (l == c) ? xc : ((l < c && c < bs) ? v - lcol[c] * xc : v);
            });
            if (l < bs) x[c0 + l] = v;
        }
        __syncthreads();
        if (c0 > 0) {
            for (int i = threadIdx.x; i < c0; i += NT) {
                T v = x[i];
                for (int k = 0; k < bs; ++k) v -= L[(c0 + k) * ld + i] * x[c0 + k];
                x[i] = v;
            }
            __syncthreads();
        }
    }
}

// Cholesky H = L L^T for a one-wave team (n <= NB <= 64; NB a compile-time
// bound): lane i holds row i of the lower triangle in registers (rows past n
// repeat row n-1 and are never read).  Right-looking by columns: the pivot
// and each column entry L_kj reach every lane by a lane read (a scalar
// broadcast), so column j costs one reciprocal square root and one FMA per
// trailing column in every lane, with no LDS traffic and no barrier.  Writes
// L strictly below the diagonal of H and L_jj to diag[j], the layout of the
// blocked factor (the diagonal and upper triangle of H take other values).
// Returns false (wave-uniform) when a pivot is not positive (the remaining
// columns then take pivot 1 and the factor is not used).
template <int NB, typename T>
__device__ __attribute__((always_inline)) inline bool wave_cholesky_regs(T *H, T *diag, int n, int ld) {
    n = __builtin_amdgcn_readfirstlane(n);
    ld = __builtin_amdgcn_readfirstlane(ld);
    const int il = opaque_lane((int)threadIdx.x & 63);
    const T *hr = H + min(il, n - 1) * ld;
    T h[NB];
    // unconditional loads at clamped (in-bounds) columns, then selects: no
    // branch between the loads, so they issue back to back
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const T t = hr[min(k, n - 1)];
        h[k] = k < n ? t : T(0);
    }
    bool ok = true;
    static_for<0, NB>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        // n again as an opaque scalar per column: the compiler would
        // otherwise precompute every (k < n) test of the unrolled loops and
        // hold them all in scalar registers
        int nj = n;
        asm volatile("" : "+s"(nj));
        if (__builtin_expect(j < nj, 1)) {
            const T d = lane_read(h[j], j);
            ok = ok && d > T(0);
            h[j] *= wave_rsq(ok ? d : T(1));   // lane j: sqrt(d); lanes below: L_ij
            // trailing columns in groups of four (entries of columns >= n are
            // never read: they may take updates); the four lane reads of a
            // group go to distinct scalar registers before its FMAs, so they
            // issue back to back
            static_for<0, (NB - j + 2) / 4>([&](auto cc) {
                constexpr int k0 = j + 1 + 4 * decltype(cc)::value;
                if (__builtin_expect(k0 < nj, 1)) {
                    T c[4];
                    static_for<0, 4>([&](auto kc) {
                        constexpr int k = k0 + decltype(kc)::value;
                        c[decltype(kc)::value] = k < NB ? lane_read(h[j], k) : T(0);
                    });
                    asm volatile("" ::"s"(c[0]), "s"(c[1]), "s"(c[2]), "s"(c[3]));
                    static_for<0, 4>([&](auto kc) {
                        constexpr int k = k0 + decltype(kc)::value;
                        if constexpr (k < NB) h[k] -= h[j] * c[decltype(kc)::value];
                    });
                }
            });
        }
    });
    // whole rows (one exec mask for the lanes of rows < n): entries on and
    // above the diagonal of H are free storage afterwards (readers take L
    // strictly below it and L_jj from diag)
    T dl = h[0];
#pragma unroll
    for (int k = 1; k < NB; ++k) dl = k == il ? h[k] : dl;
    if (il < n) {
        T *row = H + il * ld;
#pragma unroll
        for (int k = 0; k < NB; ++k)
            if (k < n) row[k] = h[k];
        diag[il] = dl;
    }
    __syncthreads();
    return ok;
}

// Solve L L^T x = b with that factor (L strictly below the diagonal of L_,
// L_jj in diag), one wave, n <= NB: lane i keeps its entry of the running
// right-hand side in a register and its row (forward) or column (backward)
// of L in registers, zero where the triangle ends, so every step is one
// FMA per lane with no lane masks; the solved entry of step j, scaled by
// 1 / L_jj, comes from lane j by a lane read.  b is only read (b and x may
// be the same array: one wave reads before it writes); x is written and
// synchronised.
template <int NB, typename T>
__device__ __attribute__((always_inline)) inline void wave_chol_solve_regs(const T *L_, const T *diag, const T *b,
                                                                           T *x, int n, int ld) {
    n = __builtin_amdgcn_readfirstlane(n);
    ld = __builtin_amdgcn_readfirstlane(ld);
    const int il = opaque_lane((int)threadIdx.x & 63);
    const int ri = min(il, n - 1);
    const T rd = T(1) / diag[ri];
    T v = il < n ? b[ri] : T(0);
    T l[NB];
    // forward L y = b: v_i <- v_i - L_ij y_j, y_j = v_j / L_jj
#pragma unroll
    for (int k = 0; k < NB; ++k) l[k] = (k < n && k < il) ? L_[ri * ld + k] : T(0);
    static_for<0, NB>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        int nj = n;
        asm volatile("" : "+s"(nj));
        // y_j = v_j / L_jj, formed in lane j and read once (the same product as
        // two lane reads multiplied)
        if (__builtin_expect(j < nj, 1)) v -= l[j] * lane_read(v * rd, j);
    });
    v *= rd;
    // backward L^T x = y: v_i <- v_i - L_ji x_j, x_j = v_j / L_jj
#pragma unroll
    for (int k = 0; k < NB; ++k) l[k] = (k < n && k > il) ? L_[k * ld + min(il, k)] : T(0);
    static_for<0, NB>([&](auto jc) {
        constexpr int j = NB - 1 - decltype(jc)::value;
        int nj = n;
        asm volatile("" : "+s"(nj));
        if (j < nj) v -= l[j] * lane_read(v * rd, j);
    });
    v *= rd;
    if (il < n) x[il] = v;
    __syncthreads();
}

// Dispatch on n (<= 16, <= 24, <= 32).  Every pointer points into the dynamic LDS;
// rebuilt from its offset so that the accesses are LDS ones.
template <typename T>
__device__ __attribute__((always_inline)) inline bool wave_cholesky(T *H, T *diag, int n, int ld) {
    H = lds_at<T>(__builtin_amdgcn_readfirstlane(lds_off(H)));
    diag = lds_at<T>(__builtin_amdgcn_readfirstlane(lds_off(diag)));
    if (n <= 16) return wave_cholesky_regs<16, T>(H, diag, n, ld);
    if (n <= 24) return wave_cholesky_regs<24, T>(H, diag, n, ld);
    return wave_cholesky_regs<32, T>(H, diag, n, ld);
}
template <typename T>
__device__ __attribute__((always_inline)) inline void wave_chol_solve(const T *L_, const T *diag, const T *b, T *x, int n, int ld) {
    L_ = lds_at<T>(__builtin_amdgcn_readfirstlane(lds_off(L_)));
    diag = lds_at<T>(__builtin_amdgcn_readfirstlane(lds_off(diag)));
    b = lds_at<T>(__builtin_amdgcn_readfirstlane(lds_off(b)));
    x = lds_at<T>(__builtin_amdgcn_readfirstlane(lds_off(x)));
    if (n <= 16) wave_chol_solve_regs<16, T>(L_, diag, b, x, n, ld);
    else if (n <= 24) wave_chol_solve_regs<24, T>(L_, diag, b, x, n, ld);
    else wave_chol_solve_regs<32, T>(L_, diag, b, x, n, ld);
}

// Pointer forms for the callers (all arguments point into the dynamic LDS).
// A one-wave team (NT = 64, n <= 32) factors and solves in registers; larger
// teams take the blocked forms (a one-wave register solve for them, two rows
// per lane, was faster alone for n <= 64 but not inside the chunked forward).
template <int NT, typename T>
__device__ __attribute__((always_inline)) inline bool team_cholesky(T *H, T *diag, int n, int ld, T *work) {
    if constexpr (NT == 64) {
        (void)work;
        return wave_cholesky(H, diag, n, ld);
    } else {
        return team_cholesky_lds<NT, T>(lds_off(H), lds_off(diag), n, ld, lds_off(work));
    }
}
template <int NT, typename T>
__device__ __attribute__((always_inline)) inline void team_chol_solve(const T *L, const T *diag, T *b, T *x, int n, int ld) {
    if constexpr (NT == 64) wave_chol_solve(L, diag, b, x, n, ld);
    else team_chol_solve_lds<NT, T>(lds_off(L), lds_off(diag), lds_off(b), lds_off(x), n, ld);
}
template <int NT, typename T>
__device__ __attribute__((always_inline)) inline void team_chol_solve(const T *L, const T *diag, T *b, T *x, int n) {
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
// The same search for a one-wave team with m <= 256 rows: each lane's (up to)
// four rows are read once and kept in registers with D q^2 and D q r
// precomputed, each trial's piece sums are two wave reductions, and the
// unchanged-piece test is a ballot.  Every lane adds its rows in the same
// order as the general form, so the sums, and the result, are bitwise the
// same.
template <typename T>
__device__ inline T wave_line_search(int m, const T *r, const T *q, const T *D, T c0, T b0,
                                     uint32_t &bits_out, T &c_out, int &fail) {
    constexpr int RPL = 4;
    const int tid = threadIdx.x & 63;
    T rr[RPL], qq[RPL], dqq[RPL], dqr[RPL];
#pragma unroll
    for (int jj = 0; jj < RPL; ++jj) {
        const int i = tid + 64 * jj;
        // rows past m (m may be 0): q = 0 and r = 1 keep them off every piece
        T qi = T(0), ri = T(1), dq = T(0);
        if (i < m) {
            qi = q[i];
            ri = r[i];
            dq = D[i] * qi;
        }
        rr[jj] = ri;
        qq[jj] = qi;
        dqq[jj] = dq * qi;
        dqr[jj] = dq * ri;
    }
    auto piece = [&](T t, uint32_t &bb, T &sc, T &sb) {
        sc = T(0);
        sb = T(0);
        bb = 0;
#pragma unroll
        for (int jj = 0; jj < RPL; ++jj) {
            const bool pa = rr[jj] + t * qq[jj] < T(0);
            sc += pa ? dqq[jj] : T(0);
            sb += pa ? dqr[jj] : T(0);
            bb |= (pa ? 1u : 0u) << jj;
        }
        sc = wave_sum(sc);
        sb = wave_sum(sb);
    };
    T t = T(1), c, b;
    uint32_t bits;
    piece(t, bits, c, b);
    c += c0;
    b += b0;
    T lo = T(0), hi = inf_val<T>();
    T alpha = t;
    fail = 1;
    const T eps = T(sizeof(T) == 4 ? 1.1920929e-7 : 2.220446049250313e-16);
    for (int it = 0; it < 96; ++it) {
        const T g = c * t + b;
        if (g == T(0)) { alpha = t; fail = 0; break; }
        if (g < T(0)) lo = t; else hi = t;
        if (hi < inf_val<T>() && hi - lo <= T(32) * eps * hi) { alpha = t; fail = 0; break; }
        T cand = -b / c;
        const bool newton = (cand > lo) && (cand < hi);
        if (!newton) cand = (hi < inf_val<T>()) ? T(0.5) * (lo + hi) : T(2) * lo + T(1);
        uint32_t nb;
        T sc, sb;
        piece(cand, nb, sc, sb);
        const bool same = __builtin_amdgcn_ballot_w64(nb != bits) == 0;
        bits = nb;
        c = c0 + sc;
        b = b0 + sb;
        t = cand;
        alpha = cand;
        if (newton && same) { fail = 0; break; }
    }
    bits_out = bits;
    c_out = c;
    return alpha;
}

template <int NT, typename T>
__device__ inline T team_line_search(int m, const T *r, const T *q, const T *D, T c0, T b0,
                                     T *sred, uint32_t &bits_out, T &c_out, int &fail) {
    const int tid = threadIdx.x;
    if constexpr (NT == 64) {
        if (m <= 256) return wave_line_search(m, r, q, D, c0, b0, bits_out, c_out, fail);
    }
    T t = T(1);
    uint32_t bits = 0;
    T c, b;
    {
        T v[2] = {T(0), T(0)};
        // every row's values read, then selected (a read under the row's
        // predicate would be a branch waiting on it); a row off the piece adds
        // +0, which leaves the sums bitwise as skipping it would
        for (int i = tid, jj = 0; i < m; i += NT, ++jj) {
            const T qi = q[i], ri = r[i], dq = D[i] * qi;
            const bool pa = ri + t * qi < T(0);
            v[0] += pa ? dq * qi : T(0);
            v[1] += pa ? dq * ri : T(0);
            bits |= (pa ? 1u : 0u) << jj;
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
            const T qi = q[i], ri = r[i], dq = D[i] * qi;
            const bool pa = ri + cand * qi < T(0);
            v[0] += pa ? dq * qi : T(0);
            v[1] += pa ? dq * ri : T(0);
            nb |= (pa ? 1u : 0u) << jj;
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
