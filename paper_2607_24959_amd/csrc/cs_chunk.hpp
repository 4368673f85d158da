// cs_chunk.hpp -- team kernels for instances whose J does not stay in LDS.
//
// One workgroup (NT = 64 for n <= 32, 256 otherwise) solves one instance at
// a time.  Forward, per Newton step: the residuals r = J a - aref (the
// first step straight from global memory, eight lanes per row, many rows'
// loads in flight, no staging; later steps from the previous step's second
// pass, r_{k+1} = (J a_k - aref) + alpha_k J p_k), each wave listing its
// active rows (r < 0) in row order; the listed rows are then gathered into
// LDS in chunks of CR rows (row stride npa + 1, conflict-free) for the
// Newton-matrix contribution J_A^T diag(D_A) J_A and the gradient J_A^T w --
// inactive rows add nothing to either.  In FP32 the contraction runs on the
// matrix cores (v_mfma_f32_16x16x4f32 on 16 x 16 tiles of the lower
// triangle, tiles spread over the waves and interleaved per K-step,
// accumulators in registers), and when n is not a multiple of 16 the
// residual rides in column n so the same pass yields J^T w; in FP64 lanes
// accumulate lower-triangle entries on the VALU.  A second direct pass forms
// q = J p for the line search and, from the same read of J, J a - aref
// afresh for the next step.  The VJP reads only the active rows of J (the
// saved A*), gathered the same way.  H (row stride npa + 1), the row arrays
// and the chunk buffer live in LDS; the FP32 forward also keeps M there when
// it fits, otherwise M is read from global memory column-wise (coalesced, as
// a symmetric matrix).
#pragma once

#include "cs_device.hpp"

namespace cs {

constexpr int CR = 64;   // rows per chunk

__host__ __device__ inline int round16(int n) { return (n + 15) & ~15; }

template <typename T>
struct ChLds {
    T *H, *diag, *a, *a0, *F, *p, *y, *v, *u, *red;
    T *r, *q, *Dv, *ar, *rx, *Jc, *Wc, *Wr;   // rx: forward, J a_k from pass B
    T *Lw;          // (not used: the contraction takes its weights from Wc)
    int *Lr, *Lc;   // slot rows (forward: Lr[e] = e; VJP: the slot's row of J), and
                    // each wave segment's slot count padded to whole K-steps
    int *Li, *Ln;   // each wave's active rows (row order), and their counts
    uint8_t *A;
};

// Capacity of one wave's active-row list: the rows dotted by a wave's lanes
// in ch_rows_dot are 8 of every NT / 8.
__host__ __device__ inline int ch_list_cap(int mmax, int NT) {
    const int rpb = NT / 8;
    return 8 * ((mmax + rpb - 1) / rpb);
}

// H (npa x (npa + 1)), eight n-vectors and the diagonal, reduction scratch,
// five row arrays, the chunk (CR x (npa + 1)), two chunk-row arrays, the
// per-wave active-row lists, A.
__host__ __device__ inline size_t ch_lds_bytes(int npa, int mmax, int NT, size_t s) {
    const size_t ld = (size_t)npa + 1;
    const size_t nT = (size_t)npa * ld + 9 * (size_t)npa + 16 * (size_t)(NT / 64) +
                      5 * (size_t)mmax + CR * ld + 4 * CR + 8;
    const size_t lists = 4 * ((size_t)(NT / 64) * ch_list_cap(mmax, NT) + 8);
    return nT * s + lists + (size_t)mmax + 64;
}

// Forward with M resident in LDS (FP32, when it fits): the n x n copy sits
// 16-byte aligned after everything above.
__host__ __device__ inline size_t ch_m_offset(int npa, int mmax, int NT, size_t s) {
    return (ch_lds_bytes(npa, mmax, NT, s) + 15) & ~size_t(15);
}
__host__ __device__ inline size_t ch_lds_bytes_mlds(int npa, int mmax, int NT, size_t s) {
    return ch_m_offset(npa, mmax, NT, s) + (size_t)npa * npa * s;
}

template <typename T>
__device__ inline ChLds<T> ch_carve(unsigned char *smem, int npa, int mmax, int NT) {
    ChLds<T> L;
    T *p = reinterpret_cast<T *>(smem);
    L.H = p; p += (size_t)npa * (npa + 1);
    L.diag = p; p += npa;
    L.a = p; p += npa;
    L.a0 = p; p += npa;
    L.F = p; p += npa;
    L.p = p; p += npa;
    L.y = p; p += npa;
    L.v = p; p += npa;
    L.u = p; p += npa;
    L.red = p; p += 16 * (NT / 64);
    L.r = p; p += mmax;
    L.q = p; p += mmax;
    L.Dv = p; p += mmax;
    L.ar = p; p += mmax;
    L.rx = p; p += mmax;
    L.Jc = p; p += (size_t)CR * (npa + 1);
    L.Wc = p; p += CR;
    L.Wr = p; p += CR;
    L.Lw = p; p += CR;
    L.Lr = reinterpret_cast<int *>(p); p += CR;
    L.Lc = reinterpret_cast<int *>(p); p += 8;
    int *ip = reinterpret_cast<int *>(p);
    L.Li = ip; ip += (NT / 64) * ch_list_cap(mmax, NT);
    L.Ln = ip; ip += 8;
    L.A = reinterpret_cast<uint8_t *>(ip);
    return L;
}

// Dot products of the chunk's rows with one or two LDS vectors; NT / CR
// lanes per row, two partial sums per lane, combined with butterflies.
// Every lane of the row's group gets the full dots; rho is the lane's row.
template <int NT, typename T>
__device__ inline T ch_row_dot(int n, int ldj, const T *Jc, const T *x, int &rho, int &part) {
    constexpr int TPR = NT / CR;
    rho = threadIdx.x / TPR;
    part = threadIdx.x % TPR;
    const T *row = Jc + rho * ldj;
    T s0 = T(0), s1 = T(0);
    int j = part;
    for (; j + TPR < n; j += 2 * TPR) {
        s0 += row[j] * x[j];
        s1 += row[j + TPR] * x[j + TPR];
    }
    if (j < n) s0 += row[j] * x[j];
    T s = s0 + s1;
#pragma unroll
    for (int o = 1; o < TPR; o <<= 1) s += __shfl_xor(s, o, 64);
    return s;
}

template <int NT, typename T>
__device__ inline void ch_row_dot2(int n, int ldj, const T *Jc, const T *x, const T *y, T &sx,
                                   T &sy, int &rho, int &part) {
    constexpr int TPR = NT / CR;
    rho = threadIdx.x / TPR;
    part = threadIdx.x % TPR;
    const T *row = Jc + rho * ldj;
    T a = T(0), b = T(0);
    for (int j = part; j < n; j += TPR) {
        const T jr = row[j];
        a += jr * x[j];
        b += jr * y[j];
    }
#pragma unroll
    for (int o = 1; o < TPR; o <<= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    sx = a;
    sy = b;
}

// Sum over the 8 lanes of an aligned lane octet, every lane gets the sum.
template <typename T> __device__ inline T osum8(T v);
template <> __device__ inline float osum8<float>(float v) {
    // quad xor 1, quad xor 2, half-row mirror
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
    return v;
}
template <> __device__ inline double osum8<double>(double v) {
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) v += __shfl_xor(v, o, 8);
    return v;
}

// Dot products of every row of the instance's row-major J (m x n, global
// memory) with an LDS vector x.  Eight lanes per row; lane `part` of an
// octet always takes columns part, part + 8, ... (CPL of them), so x is read
// from LDS once per pass.  Rows go in blocks of NT / 8 (octet o of the
// workgroup takes row o of each block), 32 / CPL blocks' loads issued before
// any use; addresses are clamped so every load is unconditional.  fn(i, s) runs
// on every lane of every octet with the row's dot s (rows i >= m included,
// so calls stay wave-convergent).
template <int NT, int CPL, typename T, typename Fn>
__device__ inline void ch_rows_dot_t(const T *__restrict__ J, int n, int m, const T *x, Fn &fn) {
    constexpr int RPB = NT / 8, UN = 32 / CPL > 1 ? 32 / CPL : 1;
    const int part = threadIdx.x & 7, oct = threadIdx.x >> 3;
    T xv[CPL];
    int cl[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int c = part + 8 * k;
        xv[k] = c < n ? x[c] : T(0);
        cl[k] = min(c, n - 1);
    }
    for (int b0 = 0; b0 < m; b0 += UN * RPB) {
        T v[UN][CPL];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const T *row = J + (int64_t)min(b0 + u * RPB + oct, m - 1) * n;
#pragma unroll
            for (int k = 0; k < CPL; ++k) v[u][k] = row[cl[k]];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            T s0 = T(0), s1 = T(0);
#pragma unroll
            for (int k = 0; k + 1 < CPL; k += 2) {
                s0 += v[u][k] * xv[k];
                s1 += v[u][k + 1] * xv[k + 1];
            }
            fn(b0 + u * RPB + oct, osum8(s0 + s1));
        }
    }
}

// The same with the columns per lane chosen from n (ceil(n / 8) rounded up
// to a multiple of 4; n <= 32 when NT = 64, n <= 128 otherwise).
template <int NT, typename T, typename Fn>
__device__ inline void ch_rows_dot(const T *__restrict__ J, int n, int m, const T *x, Fn &&fn) {
    if constexpr (NT == 64) {
        ch_rows_dot_t<NT, 4>(J, n, m, x, fn);
    } else {
        if (n <= 32) ch_rows_dot_t<NT, 4>(J, n, m, x, fn);
        else if (n <= 64) ch_rows_dot_t<NT, 8>(J, n, m, x, fn);
        else if (n <= 96) ch_rows_dot_t<NT, 12>(J, n, m, x, fn);
        else ch_rows_dot_t<NT, 16>(J, n, m, x, fn);
    }
}

// Two dot products per row from one read of J: fn(i, J_i . x, J_i . y).
template <int NT, int CPL, typename T, typename Fn>
__device__ inline void ch_rows_dot2_t(const T *__restrict__ J, int n, int m, const T *x,
                                      const T *y, Fn &fn) {
    constexpr int RPB = NT / 8, UN = 32 / CPL > 1 ? 32 / CPL : 1;
    const int part = threadIdx.x & 7, oct = threadIdx.x >> 3;
    T xv[CPL], yv[CPL];
    int cl[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int c = part + 8 * k;
        xv[k] = c < n ? x[c] : T(0);
        yv[k] = c < n ? y[c] : T(0);
        cl[k] = min(c, n - 1);
    }
    for (int b0 = 0; b0 < m; b0 += UN * RPB) {
        T v[UN][CPL];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const T *row = J + (int64_t)min(b0 + u * RPB + oct, m - 1) * n;
#pragma unroll
            for (int k = 0; k < CPL; ++k) v[u][k] = row[cl[k]];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            T sx = T(0), sy = T(0);
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                sx += v[u][k] * xv[k];
                sy += v[u][k] * yv[k];
            }
            fn(b0 + u * RPB + oct, osum8(sx), osum8(sy));
        }
    }
}

template <int NT, typename T, typename Fn>
__device__ inline void ch_rows_dot2(const T *__restrict__ J, int n, int m, const T *x, const T *y,
                                    Fn &&fn) {
    if constexpr (NT == 64) {
        ch_rows_dot2_t<NT, 4>(J, n, m, x, y, fn);
    } else {
        if (n <= 32) ch_rows_dot2_t<NT, 4>(J, n, m, x, y, fn);
        else if (n <= 64) ch_rows_dot2_t<NT, 8>(J, n, m, x, y, fn);
        else if (n <= 96) ch_rows_dot2_t<NT, 12>(J, n, m, x, y, fn);
        else ch_rows_dot2_t<NT, 16>(J, n, m, x, y, fn);
    }
}

// Visit the rows without reading J, every lane taking one: each wave meets
// the rows ch_rows_dot gives it (rows 8 w .. 8 w + 7 of each block of NT / 8)
// in the same order -- lane 8 b + j takes row j of the wave's eight in block
// b of a group of eight blocks -- so lists built in lane order come out the
// same.  fn(i) runs on every lane (rows i >= m included).
template <int NT, typename Fn>
__device__ inline void ch_rows_each(int m, Fn &&fn) {
    constexpr int RPB = NT / 8;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nblk = (m + RPB - 1) / RPB;
    for (int b0 = 0; b0 < nblk; b0 += 8) fn((b0 + (lane >> 3)) * RPB + 8 * w + (lane & 7));
}

// Per-thread partial of J^T x over the chunks: column fj, rows fp, fp + fparts, ...
template <int NT, typename T>
struct ChColSum {
    int fj, fp, fparts;
    T acc;
    __device__ inline void plan(int n) {
        fparts = min(4, NT / n);
        fp = (int)threadIdx.x / n;
        fj = (int)threadIdx.x - fp * n;
        acc = T(0);
    }
    __device__ inline void add_chunk(int ldj, const T *Jc, const T *x) {
        if (fp < fparts) {
            T s0 = T(0), s1 = T(0);
            int rr = fp;
            for (; rr + fparts < CR; rr += 2 * fparts) {
                s0 += x[rr] * Jc[rr * ldj + fj];
                s1 += x[rr + fparts] * Jc[(rr + fparts) * ldj + fj];
            }
            if (rr < CR) s0 += x[rr] * Jc[rr * ldj + fj];
            acc += s0 + s1;
        }
    }
    // out[j] = base[j] + sum of the partials; uses scratch (fparts x ldj),
    // synchronises the team before and after.
    __device__ inline void finish(int n, int ldj, T *scratch, const T *base, T *out) const {
        __syncthreads();
        if (fp < fparts) scratch[fp * ldj + fj] = acc;
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += NT) {
            T s = base ? base[j] : T(0);
            for (int q = 0; q < fparts; ++q) s += scratch[q * ldj + j];
            out[j] = s;
        }
        __syncthreads();
    }
};

typedef float chf4 __attribute__((ext_vector_type(4)));

// Tiles of the lower triangle: t = ti (ti + 1) / 2 + tj, tj <= ti.
__device__ inline void tile_of(int t, int &ti, int &tj) {
    ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    tj = t - ti * (ti + 1) / 2;
}

// Newton-matrix accumulator of one workgroup.
template <typename T, int NT> struct ChAcc;

// FP32: MFMA tiles, MAXT per wave.
template <int NT> struct ChAcc<float, NT> {
    static constexpr int NW = NT / 64;
    static constexpr int MAXT = NT == 64 ? 3 : 9;   // n <= 32 resp. n <= 128
    chf4 acc[MAXT];
    int ti[MAXT], tj[MAXT], ntiles;

    __device__ inline void init(int npa) {
        const int nt = npa / 16;
        ntiles = nt * (nt + 1) / 2;
        const int wave = threadIdx.x >> 6;
#pragma unroll
        for (int s = 0; s < MAXT; ++s) {
            tile_of(wave + NW * s, ti[s], tj[s]);
            acc[s] = chf4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __device__ inline void zero() {
#pragma unroll
        for (int s = 0; s < MAXT; ++s) acc[s] = chf4{0.f, 0.f, 0.f, 0.f};
    }
    // acc += J_c^T diag(D o A) J_c over the chunk's gathered active rows
    // (slot e holds chunk row Lr[e] = e with weight Lw[e]; slots past the
    // list's end are zero rows of weight 0), walked in CR / NW-slot segments,
    // each up to its count padded to whole K-steps (Lc).  The row index is
    // read rather than taken as e: dropping that read let the compiler hoist
    // enough loads to spill the kernel's registers.  The wave's tile count is
    // a compile-time constant in each instance of the body, so a K-step
    // issues all its LDS loads, then all its MFMAs, with no branches in
    // between.
    template <int TPW>
    __device__ inline void add_chunk_t(int ldj, const float *Jc, const int *Lr, const float *Lw,
                                       const int *Lc) {
        constexpr int SEG = CR / NW;
        const int lane = threadIdx.x & 63;
        const int kq = lane >> 4, idx = lane & 15;
        int ca[TPW], cb[TPW];
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            ca[s] = 16 * ti[s] + idx;
            cb[s] = 16 * tj[s] + idx;
        }
        for (int sg = 0; sg < NW; ++sg) {
            const int nk = __builtin_amdgcn_readfirstlane(Lc[sg]) >> 2;
#pragma unroll 2
            for (int kb = 0; kb < nk; ++kb) {
                const int e = sg * SEG + 4 * kb + kq;
                const float wr = Lw[e];
                const float *jr = Jc + Lr[e] * ldj;
                float av[TPW], bv[TPW];
#pragma unroll
                for (int s = 0; s < TPW; ++s) {
                    av[s] = jr[ca[s]];
                    bv[s] = jr[cb[s]];
                }
#pragma unroll
                for (int s = 0; s < TPW; ++s)
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], wr * bv[s], acc[s], 0, 0, 0);
            }
        }
    }
    __device__ inline void add_chunk(int ldj, const float *Jc, const float *, const int *Lr,
                                     const float *Lw, const int *Lc) {
        const int wave = threadIdx.x >> 6;
        const int ntl = (ntiles - wave + NW - 1) / NW;   // tiles of this wave (wave-uniform)
        switch (ntl) {
            case 1: add_chunk_t<1>(ldj, Jc, Lr, Lw, Lc); break;
            case 2: add_chunk_t<2>(ldj, Jc, Lr, Lw, Lc); break;
            case 3: add_chunk_t<3>(ldj, Jc, Lr, Lw, Lc); break;
            case 4: if constexpr (MAXT >= 4) add_chunk_t<4>(ldj, Jc, Lr, Lw, Lc); break;
            case 5: if constexpr (MAXT >= 5) add_chunk_t<5>(ldj, Jc, Lr, Lw, Lc); break;
            case 6: if constexpr (MAXT >= 6) add_chunk_t<6>(ldj, Jc, Lr, Lw, Lc); break;
            case 7: if constexpr (MAXT >= 7) add_chunk_t<7>(ldj, Jc, Lr, Lw, Lc); break;
            case 8: if constexpr (MAXT >= 8) add_chunk_t<8>(ldj, Jc, Lr, Lw, Lc); break;
            case 9: if constexpr (MAXT >= 9) add_chunk_t<9>(ldj, Jc, Lr, Lw, Lc); break;
            default: break;
        }
    }
    // H (lower, stride ldh) = M + acc.  Each tile's M entries are read
    // before any store, from clamped (in-bounds) addresses; the empty asm
    // keeps the compiler from sinking each read into a masked branch of its
    // own that waits for it.
    __device__ inline void store(int n, int ldh, const float *__restrict__ M, float *H) const {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int kq = lane >> 4, idx = lane & 15;
#pragma unroll
        for (int s = 0; s < MAXT; ++s) {
            if (wave + NW * s < ntiles) {
                const int col = 16 * tj[s] + idx, cc = min(col, n - 1);
                float mv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) mv[r] = M[min(16 * ti[s] + 4 * kq + r, n - 1) * n + cc];
#pragma unroll
                for (int r = 0; r < 4; ++r) asm volatile("" : "+v"(mv[r]));
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * ti[s] + 4 * kq + r;
                    if (row < n && col <= row) H[row * ldh + col] = acc[s][r] + mv[r];
                }
            }
        }
    }
    // As store, when the chunk's column n held the residual: row n of the
    // product is J^T diag(D o A) r = J^T w, so F = u + that row.
    __device__ inline void store_hf(int n, int ldh, const float *__restrict__ M, float *H,
                                    const float *u, float *F) const {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int kq = lane >> 4, idx = lane & 15;
#pragma unroll
        for (int s = 0; s < MAXT; ++s) {
            if (wave + NW * s < ntiles) {
                const int col = 16 * tj[s] + idx, cc = min(col, n - 1);
                float mv[4], uv = u[cc];
#pragma unroll
                for (int r = 0; r < 4; ++r) mv[r] = M[min(16 * ti[s] + 4 * kq + r, n - 1) * n + cc];
#pragma unroll
                for (int r = 0; r < 4; ++r) asm volatile("" : "+v"(mv[r]));
                asm volatile("" : "+v"(uv));
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * ti[s] + 4 * kq + r;
                    if (row < n && col <= row) H[row * ldh + col] = acc[s][r] + mv[r];
                    if (row == n && col < n) F[col] = acc[s][r] + uv;
                }
            }
        }
    }
    // The residual rides along as column n when the padded width n + 1 still
    // fits the workgroup's tile budget.
    __device__ static inline bool fits_residual(int n) {
        const int nt = round16(n + 1) / 16;
        return nt * (nt + 1) / 2 <= NW * MAXT;
    }
};

// FP64: lower-triangle entries e = tid + NT s on the VALU.
template <int NT> struct ChAcc<double, NT> {
    static constexpr int MAXE = NT == 64 ? 9 : 33;   // ceil(n (n+1) / 2 / NT)
    double acc[MAXE];
    int ej[MAXE], el[MAXE], ne;

    __device__ inline void init(int n) {
        ne = n * (n + 1) / 2;
        // (j, l) of entry tid, then advanced by NT entries at a time
        int j = 0, l = threadIdx.x;
        while (l > j) { l -= j + 1; ++j; }
#pragma unroll
        for (int s = 0; s < MAXE; ++s) {
            ej[s] = j;
            el[s] = l;
            acc[s] = 0.0;
            l += NT;
            while (l > j) { l -= j + 1; ++j; }
        }
    }
    __device__ inline void zero() {
#pragma unroll
        for (int s = 0; s < MAXE; ++s) acc[s] = 0.0;
    }
    __device__ inline void add_chunk(int ldj, const double *Jc, const double *Wc, const int *,
                                     const double *, const int *) {
#pragma unroll
        for (int s = 0; s < MAXE; ++s) {
            if ((int)threadIdx.x + NT * s < ne) {
                double h0 = 0.0, h1 = 0.0;
                const double *cj = Jc + ej[s], *cl = Jc + el[s];
                for (int rho = 0; rho < CR; rho += 2) {
                    h0 += Wc[rho] * cj[rho * ldj] * cl[rho * ldj];
                    h1 += Wc[rho + 1] * cj[(rho + 1) * ldj] * cl[(rho + 1) * ldj];
                }
                acc[s] += h0 + h1;
            }
        }
    }
    __device__ inline void store(int n, int ldh, const double *__restrict__ M, double *H) const {
#pragma unroll
        for (int s = 0; s < MAXE; ++s)
            if ((int)threadIdx.x + NT * s < ne)
                H[ej[s] * ldh + el[s]] = acc[s] + M[ej[s] * n + el[s]];
    }
};

// Walk the packed lower triangle (j, l), l <= j, in steps of NT entries
// starting at entry tid: no division per element.
struct TriWalk {
    int j, l;
    template <int NT> __device__ inline void start() {
        j = 0;
        l = threadIdx.x;
        while (l > j) { l -= j + 1; ++j; }
    }
    template <int NT> __device__ inline void next() {
        l += NT;
        while (l > j) { l -= j + 1; ++j; }
    }
};

template <int NT, typename T>
__device__ inline T team_max(T v, T *sred) {
    v = wave_max(v);
    if constexpr (NT > 64) {
        constexpr int NW = NT / 64;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = v;
        __syncthreads();
        v = sred[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) v = fmax(v, sred[i]);
    }
    return v;
}

// Entry pos (< total) of the concatenated per-wave active-row lists.
template <int NT, typename T>
__device__ inline int ch_list_at(const ChLds<T> &L, const int (&off)[NT / 64], int cap, int pos) {
    int w = 0, o = 0;
#pragma unroll
    for (int q = 1; q < NT / 64; ++q)
        if (pos >= off[q]) { w = q; o = off[q]; }
    return L.Li[w * cap + pos - o];
}

// Chunk c of the active-row list (entries c CR .. c CR + CR - 1 of the
// per-wave lists taken wave after wave) into LDS: slot s of Jc gets the
// row of J, Wc[s] its weight D_i, Wr[s] = D_i r_i and, when fused, Jc[s][n]
// = r_i; slots past the list's end are zero rows of weight zero.  Lc gets
// each wave segment's slot count padded to whole K-steps.  Synchronises the
// team before the LDS stores and after them.
template <int NT, int CPL, typename T>
__device__ inline void ch_gather_t(const T *__restrict__ J, int n, int ldj, int c, int total,
                                   const int (&off)[NT / 64], int cap, bool fused,
                                   const ChLds<T> &L) {
    constexpr int RPB = NT / 8, GP = CR / RPB, NW = NT / 64;
    const int part = threadIdx.x & 7, oct = threadIdx.x >> 3;
    T v[GP][CPL];
    int rows[GP];
#pragma unroll
    for (int g = 0; g < GP; ++g) {
        const int pos = c * CR + g * RPB + oct;
        const int row = pos < total ? ch_list_at<NT>(L, off, cap, pos) : -1;
        rows[g] = row;
        const T *src = J + (int64_t)max(row, 0) * n;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const T x = src[min(part + 8 * k, n - 1)];
            v[g][k] = row >= 0 ? x : T(0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < GP; ++g) {
        const int slot = g * RPB + oct;
        T *dst = L.Jc + slot * ldj;
#pragma unroll
        for (int k = 0; k < CPL; ++k)
            if (part + 8 * k < n) dst[part + 8 * k] = v[g][k];
        if (part == 0) {
            const int row = rows[g];
            const T r = row >= 0 ? L.r[row] : T(0);
            const T wd = row >= 0 ? L.Dv[row] : T(0);
            L.Wc[slot] = wd;
            L.Wr[slot] = wd * r;
            if (fused) dst[n] = r;
        }
    }
    if ((int)threadIdx.x < NW) {
        const int left = min(CR, total - c * CR) - (CR / NW) * (int)threadIdx.x;
        L.Lc[threadIdx.x] = min(CR / NW, (max(left, 0) + 3) & ~3);
    }
    __syncthreads();
}

template <int NT, typename T>
__device__ inline void ch_gather(const T *__restrict__ J, int n, int ldj, int c, int total,
                                 const int (&off)[NT / 64], int cap, bool fused,
                                 const ChLds<T> &L) {
    if constexpr (NT == 64) {
        ch_gather_t<NT, 4>(J, n, ldj, c, total, off, cap, fused, L);
    } else {
        if (n <= 32) ch_gather_t<NT, 4>(J, n, ldj, c, total, off, cap, fused, L);
        else if (n <= 64) ch_gather_t<NT, 8>(J, n, ldj, c, total, off, cap, fused, L);
        else if (n <= 96) ch_gather_t<NT, 12>(J, n, ldj, c, total, off, cap, fused, L);
        else ch_gather_t<NT, 16>(J, n, ldj, c, total, off, cap, fused, L);
    }
}

template <typename T, int NT, bool MLDS>
__global__ __launch_bounds__(NT) void k_forward_chunk(
    BatchView bv, int count, int max_iter, T tol, int npa, int mmax, const T *__restrict__ gM,
    const T *__restrict__ gJ, const T *__restrict__ ga0, const T *__restrict__ garef,
    const T *__restrict__ gD, const T *__restrict__ gainit, T *__restrict__ gaout,
    T *__restrict__ gfac, uint8_t *__restrict__ gmask, int32_t *__restrict__ gstatus,
    int32_t *__restrict__ giters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const ChLds<T> L = ch_carve<T>(smem, npa, mmax, NT);
    const int tid = threadIdx.x;
    const int ldj = npa + 1, ldh = npa + 1;
    const int cap = ch_list_cap(mmax, NT);
    T *Ms = MLDS ? reinterpret_cast<T *>(smem + ch_m_offset(npa, mmax, NT, sizeof(T))) : nullptr;
    for (int e = tid; e < CR; e += NT) L.Lr[e] = e;   // gathered chunks: slot e is row e
    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) {   // team-uniform
            mark_bad(I, gstatus, giters, tid == 0);
            continue;
        }
        const int n = I.n, m = I.m;
        const T *M = gM + I.onn, *J = gJ + I.omn;
        ChColSum<NT, T> cs;
        bool bad = false;
        for (int j = tid; j < n; j += NT) {
            const T x = ga0[I.on + j];
            const T y = gainit ? gainit[I.on + j] : x;
            L.a0[j] = x;
            L.a[j] = y;
            bad |= !finite_val(x) || !finite_val(y);
        }
        for (int i = tid; i < m; i += NT) {
            const T d = gD[I.om + i], ar = garef[I.om + i];
            L.Dv[i] = d;
            L.ar[i] = ar;
            L.A[i] = 0;
            bad |= !finite_val(d) || !finite_val(ar);
        }
        {   // H = M (row stride ldh) for the definiteness check
            int rr = tid / n, jj = tid - rr * n;
            const int dr = NT / n, dc = NT - dr * n;
            for (int e = tid; e < n * n; e += NT) {
                const T x = M[e];
                L.H[rr * ldh + jj] = x;
                if constexpr (MLDS) Ms[e] = x;
                bad |= !finite_val(x);
                rr += dr;
                jj += dc;
                if (jj >= n) { jj -= n; ++rr; }
            }
        }
        // J is checked by the first residual pass (a non-finite entry makes
        // its row's dot non-finite, a being finite); only when M fails does
        // it get a scan of its own, so that NONFINITE still takes precedence
        const int anybad = __syncthreads_or(bad);
        const T *Mk = MLDS ? Ms : M;   // M for the rest of the solve
        int st = 0, k = 0;
        if (anybad) {
            st = ST_NONFINITE;
        } else if (!team_cholesky<NT>(L.H, L.diag, n, ldh, L.Jc)) {
            bool jb = false;
            for (int e = tid; e < m * n; e += NT) jb |= !finite_val(J[e]);
            st = __syncthreads_or(jb) ? ST_NONFINITE : ST_NOTSPD;
        }
        // FP32: the residual rides in column n of the staged chunk (which
        // the row stride npa + 1 always has), so one matrix-core pass gives
        // H and J^T w; tiles of this instance's own width, not the class's
        bool fused = false;
        if constexpr (sizeof(T) == 4) fused = ChAcc<T, NT>::fits_residual(n);
        ChAcc<T, NT> acc;
        acc.init(sizeof(T) == 4 ? round16(fused ? n + 1 : n) : n);
        if (st == 0) {
            T trM = T(0);
            for (int j = 0; j < n; ++j) trM += Mk[j * n + j];
            // u = M (a - a0), kept up to date across steps
            for (int j = tid; j < n; j += NT) {
                T s = T(0);
#pragma unroll 16
                for (int l = 0; l < n; ++l) s += Mk[l * n + j] * (L.a[l] - L.a0[l]);
                L.u[j] = s;
            }
            T step_inf = T(-1), alpha_prev = T(0);
            int lsfail = 0;
            for (k = 0;; ++k) {
                // pass A: r, A, F = M (a - a0) + J^T w and H = M + J^T diag(D o A) J.
                // The first step's residuals come straight from global memory;
                // later ones from the previous step's pass B, which read J
                // once for both J a_k and J p_k: r_{k+1} = (J a_k - aref) +
                // alpha_k J p_k (one rounding from the direct product, never
                // accumulated across steps).  Each wave lists its active rows
                // in row order; the listed rows are then gathered into LDS
                // chunks for the contraction and J^T w (inactive rows add
                // nothing to either).
                acc.zero();
                cs.plan(n);
                bool changed = false, nonfin = false;
                {
                    int cntw = 0;   // wave-uniform
                    int *lw = L.Li + (tid >> 6) * cap;
                    auto visit = [&](int i, bool mine, T r) {
                        int was = L.A[min(i, m - 1)];
                        asm volatile("" : "+v"(was));   // read with the others, not under mine
                        bool an = false;
                        if (mine) {
                            nonfin |= !finite_val(r);
                            an = r < T(0);
                            changed |= an != (was != 0);
                            L.A[i] = an;
                            L.r[i] = r;
                        }
                        const uint64_t bal = __builtin_amdgcn_ballot_w64(an);
                        if (an)
                            lw[cntw + (int)__builtin_amdgcn_mbcnt_hi(
                                          (uint32_t)(bal >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] = i;
                        cntw += (int)__builtin_popcountll(bal);
                    };
                    // (row reads from clamped indices, unconditional: a read
                    // under the lane's predicate would become a branch of its
                    // own that waits for it)
                    if (k == 0) {
                        ch_rows_dot<NT>(J, n, m, L.a, [&](int i, T s) {
                            const bool mine = (tid & 7) == 0 && i < m;
                            visit(i, mine, s - L.ar[min(i, m - 1)]);
                        });
                    } else {
                        ch_rows_each<NT>(m, [&](int i) {
                            const int ic = min(i, m - 1);
                            visit(i, i < m, (L.rx[ic] - L.ar[ic]) + alpha_prev * L.q[ic]);
                        });
                    }
                    if ((tid & 63) == 0) L.Ln[tid >> 6] = cntw;
                }
                if (__syncthreads_or(k == 0 && nonfin)) { st = ST_NONFINITE; break; }
                // H depends on the active set only: when it is unchanged the
                // previous step's factor (still in L.H / L.diag) is H's, and
                // the step needs only J^T w from the gathered rows
                const bool same = !__syncthreads_or(changed);
                const bool reuse = k > 0 && same;
                {
                    int off[NT / 64], total = 0;
#pragma unroll
                    for (int w = 0; w < NT / 64; ++w) {
                        off[w] = total;
                        total += L.Ln[w];
                    }
                    const int ncha = (total + CR - 1) / CR;
                    for (int c = 0; c < ncha; ++c) {
                        ch_gather<NT>(J, n, ldj, c, total, off, cap, fused && !reuse, L);
                        if (!fused || reuse) cs.add_chunk(ldj, L.Jc, L.Wr);
                        if (!reuse) acc.add_chunk(ldj, L.Jc, L.Wc, L.Lr, L.Wc, L.Lc);
                    }
                }
                if (reuse) {
                    cs.finish(n, ldj, L.Jc, L.u, L.F);
                } else if constexpr (sizeof(T) == 4) {
                    if (fused) {
                        acc.store_hf(n, ldh, Mk, L.H, L.u, L.F);
                        __syncthreads();
                    } else {
                        acc.store(n, ldh, Mk, L.H);
                        cs.finish(n, ldj, L.Jc, L.u, L.F);
                    }
                } else {
                    acc.store(n, ldh, Mk, L.H);
                    cs.finish(n, ldj, L.Jc, L.u, L.F);
                }
                T g2 = T(0), an = T(0);
                for (int j = tid; j < n; j += NT) {
                    g2 += L.F[j] * L.F[j];
                    an = fmax(an, fabs(L.a[j]));
                }
                {
                    T v1[1] = {g2};
                    team_sum<NT>(v1, L.red);
                    g2 = v1[0];
                }
                const T anorm = team_max<NT>(an, L.red);
                if (!reuse && !team_cholesky<NT>(L.H, L.diag, n, ldh, L.Jc)) { st = ST_NOTSPD; break; }
                if (sqrt(g2) <= tol * trM ||
                    (k > 0 && step_inf >= T(0) && same && step_inf <= tol * (T(1) + anorm))) {
                    st = ST_CONVERGED;
                    break;
                }
                if (k == max_iter) { st = ST_MAXITER; break; }
                for (int j = tid; j < n; j += NT) L.y[j] = -L.F[j];
                __syncthreads();
                team_chol_solve<NT>(L.H, L.diag, L.y, L.p, n, ldh);
                // pass B (straight from global memory): q = J p and, from the
                // same read of J, J a afresh for the next step's residuals
                // (kept apart from r: the line search works with the r that
                // formed F and p, so p stays a descent direction); and v = M p
                ch_rows_dot2<NT>(J, n, m, L.a, L.p, [&](int i, T sa, T sp) {
                    if ((tid & 7) == 0 && i < m) {
                        L.rx[i] = sa;
                        L.q[i] = sp;
                    }
                });
                T c0 = T(0), b0 = T(0);
                for (int j = tid; j < n; j += NT) {
                    T mp = T(0);
#pragma unroll 16
                    for (int l = 0; l < n; ++l) mp += Mk[l * n + j] * L.p[l];
                    L.v[j] = mp;
                    c0 += L.p[j] * mp;
                    b0 += L.p[j] * L.u[j];
                }
                {
                    T v2[2] = {c0, b0};
                    team_sum<NT>(v2, L.red);   // synchronises: q and v are visible after it
                    c0 = v2[0];
                    b0 = v2[1];
                }
                __syncthreads();
                uint32_t bits;
                T cpiece;
                int fl;
                const T alpha = team_line_search<NT>(m, L.r, L.q, L.Dv, c0, b0, L.red, bits,
                                                     cpiece, fl);
                lsfail |= fl;
                alpha_prev = alpha;
                T si = T(0);
                for (int j = tid; j < n; j += NT) {
                    const T s = alpha * L.p[j];
                    si = fmax(si, fabs(s));
                    L.a[j] += s;
                    // u = M (a - a0) for the new iterate, from the products of this step
                    L.u[j] += alpha * L.v[j];
                }
                step_inf = team_max<NT>(si, L.red);
                __syncthreads();
            }
            if (lsfail) st |= ST_LSFAIL;
        }
        const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
        const T nanv = T(__builtin_nan(""));
        for (int j = tid; j < n; j += NT) gaout[I.on + j] = ok ? L.a[j] : nanv;
        T *fac = gfac + fac_offset(I);
        {
            TriWalk tw;
            tw.start<NT>();
            for (int e = tid; e < n * (n + 1) / 2; e += NT) {
                fac[e] = ok ? (tw.l < tw.j ? L.H[tw.j * ldh + tw.l] : L.diag[tw.j]) : nanv;
                tw.next<NT>();
            }
        }
        for (int i = tid; i < m; i += NT) gmask[I.om + i] = ok ? L.A[i] : 0;
        if (tid == 0) {
            gstatus[I.b] = st;
            if (giters) giters[I.b] = k;
        }
        __syncthreads();
    }
}

// IFT VJP (eq. 17).  Every row-level term carries A*: an inactive row has
// arefbar = Dbar = 0 and Jbar_i = -(0 lambda + 0 a), and adds nothing to
// J^T (D o A* o J v).  So only the active rows of J are read, gathered into
// LDS in chunks as in the forward; the inactive rows' outputs are written
// without touching J.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_ift_vjp_chunk(
    BatchView bv, int count, int npa, int mmax, const T *__restrict__ gfac,
    const uint8_t *__restrict__ gmask, const T *__restrict__ gM, const T *__restrict__ gJ,
    const T *__restrict__ ga0, const T *__restrict__ garef, const T *__restrict__ gD,
    const T *__restrict__ ga, const T *__restrict__ gabar, T *__restrict__ ga0bar,
    T *__restrict__ garefbar, T *__restrict__ gJbar, T *__restrict__ gDbar,
    T *__restrict__ gMbar) {
    extern __shared__ __align__(16) unsigned char smem[];
    const ChLds<T> L = ch_carve<T>(smem, npa, mmax, NT);
    const int tid = threadIdx.x;
    const int ldj = npa + 1, ldh = npa + 1;
    const int cap = ch_list_cap(mmax, NT);
    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) continue;   // team-uniform: outputs untouched
        const int n = I.n, m = I.m;
        const T *M = gM + I.onn, *J = gJ + I.omn;
        const T *fac = gfac + fac_offset(I);
        ChColSum<NT, T> cs;
        {
            TriWalk tw;
            tw.start<NT>();
            for (int e = tid; e < n * (n + 1) / 2; e += NT) {
                if (tw.l < tw.j) L.H[tw.j * ldh + tw.l] = fac[e];
                else L.diag[tw.j] = fac[e];
                tw.next<NT>();
            }
        }
        for (int j = tid; j < n; j += NT) {
            L.a[j] = ga[I.on + j];
            L.a0[j] = ga0[I.on + j];
            L.y[j] = gabar[I.on + j];
        }
        for (int i = tid; i < m; i += NT) {
            L.Dv[i] = gD[I.om + i];
            L.ar[i] = garef[I.om + i];
            L.A[i] = gmask[I.om + i];
            L.r[i] = T(0);   // read (not used) by the gather
        }
        __syncthreads();
        // the active rows, listed per wave in row order
        {
            int cntw = 0;   // wave-uniform
            int *lw = L.Li + (tid >> 6) * cap;
            ch_rows_each<NT>(m, [&](int i) {
                const bool an = i < m && L.A[min(i, m - 1)] != 0;   // read unconditionally
                const uint64_t bal = __builtin_amdgcn_ballot_w64(an);
                if (an)
                    lw[cntw + (int)__builtin_amdgcn_mbcnt_hi(
                                  (uint32_t)(bal >> 32),
                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] = i;
                cntw += (int)__builtin_popcountll(bal);
            });
            if ((tid & 63) == 0) L.Ln[tid >> 6] = cntw;
        }
        __syncthreads();
        int off[NT / 64], total = 0;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) {
            off[q] = total;
            total += L.Ln[q];
        }
        const int ncha = (total + CR - 1) / CR;
        // lambda = H^{-1} abar with one refinement step, H v = M v + J^T (D o A* o J v)
        team_chol_solve<NT>(L.H, L.diag, L.y, L.u, n, ldh);
        cs.plan(n);
        for (int c = 0; c < ncha; ++c) {
            ch_gather<NT>(J, n, ldj, c, total, off, cap, false, L);   // Wc = D of each row
            int rho, part;
            const T sv = ch_row_dot<NT>(n, ldj, L.Jc, L.u, rho, part);
            if (part == 0) L.Wr[rho] = L.Wc[rho] * sv;
            __syncthreads();
            cs.add_chunk(ldj, L.Jc, L.Wr);
        }
        cs.finish(n, ldj, L.Jc, nullptr, L.F);
        for (int j = tid; j < n; j += NT) {
            T sv = gabar[I.on + j] - L.F[j];
#pragma unroll 16
            for (int l = 0; l < n; ++l) sv -= M[(int64_t)l * n + j] * L.u[l];
            L.y[j] = sv;
        }
        __syncthreads();
        team_chol_solve<NT>(L.H, L.diag, L.y, L.p, n, ldh);
        for (int j = tid; j < n; j += NT) L.u[j] += L.p[j];
        // per-row cotangents and J-bar of the active rows, chunk by chunk
        for (int c = 0; c < ncha; ++c) {
            ch_gather<NT>(J, n, ldj, c, total, off, cap, false, L);
            int rho, part;
            T ja, sig;
            ch_row_dot2<NT>(n, ldj, L.Jc, L.a, L.u, ja, sig, rho, part);
            if (part == 0) {
                const int pos = c * CR + rho;
                if (pos < total) {
                    const int i = ch_list_at<NT>(L, off, cap, pos);
                    const T r = ja - L.ar[i];
                    const T arb = L.Dv[i] * sig;
                    if (garefbar) garefbar[I.om + i] = arb;
                    if (gDbar) gDbar[I.om + i] = -r * sig;
                    L.Wc[rho] = L.Dv[i] * r;
                    L.Wr[rho] = arb;
                    L.Lr[rho] = i;
                } else {
                    L.Lr[rho] = -1;
                }
            }
            __syncthreads();
            if (gJbar) {
                // eight lanes per slot: the slot's row and weights read once,
                // each lane writing every eighth entry of the row
                const int part = tid & 7;
                for (int sl = tid >> 3; sl < CR; sl += NT >> 3) {
                    const int row = L.Lr[sl];
                    if (row >= 0) {
                        const T wv = L.Wc[sl], arb = L.Wr[sl];
                        T *dst = gJbar + I.omn + (int64_t)row * n;
                        for (int j = part; j < n; j += 8) dst[j] = -(wv * L.u[j] + arb * L.a[j]);
                    }
                }
            }
        }
        // the inactive rows: no read of J
        for (int i = tid; i < m; i += NT) {
            if (!L.A[i]) {
                if (garefbar) garefbar[I.om + i] = T(0);
                if (gDbar) gDbar[I.om + i] = T(0);
            }
        }
        if (gJbar) {
            // eight lanes per row: the row's flag read once
            const int part = tid & 7;
            for (int i = tid >> 3; i < m; i += NT >> 3) {
                if (!L.A[i]) {
                    T *dst = gJbar + I.omn + (int64_t)i * n;
                    for (int j = part; j < n; j += 8) dst[j] = -(T(0) * L.u[j] + T(0) * L.a[j]);
                }
            }
        }
        if (ga0bar) {
            for (int j = tid; j < n; j += NT) {
                T sv = T(0);
#pragma unroll 16
                for (int l = 0; l < n; ++l) sv += M[(int64_t)l * n + j] * L.u[l];
                ga0bar[I.on + j] = sv;
            }
        }
        if (gMbar) {
            int jr = tid / n, lc = tid - jr * n;
            const int dr = NT / n, dc = NT - dr * n;
            for (int e = tid; e < n * n; e += NT) {
                gMbar[I.onn + e] = -L.u[jr] * (L.a[lc] - L.a0[lc]);
                jr += dr;
                lc += dc;
                if (lc >= n) { lc -= n; ++jr; }
            }
        }
        __syncthreads();
    }
}

// Host side --------------------------------------------------------------

inline int chunk_nt(int nmax) { return nmax <= 32 ? 64 : 256; }

inline bool chunk_supported(int nmax, int mmax, int s) {
    if (nmax > 128 || mmax > 2048) return false;
    const int NT = chunk_nt(nmax);
    if (s == 8 && nmax > (NT == 64 ? 32 : 128)) return false;
    return ch_lds_bytes(round16(nmax), mmax, NT, (size_t)s) <= 160 * 1024;
}

template <typename K>
inline int chunk_prepare(K kernel, size_t lds) {
    return ensure_lds(reinterpret_cast<const void *>(kernel), lds) ? 0 : -3;
}

inline unsigned chunk_grid(int count) { return (unsigned)(count < (1 << 20) ? count : (1 << 20)); }

template <typename T>
int launch_chunk_forward(const BatchView &bv, int count, int nmax, int mmax, int max_iter, T tol,
                         const T *M, const T *J, const T *a0, const T *aref, const T *D,
                         const T *a_init, T *a_out, T *fac, uint8_t *mask, int32_t *status,
                         int32_t *iters, hipStream_t stream) {
    const int npa = round16(nmax);
    const int NT = chunk_nt(nmax);
    // FP32 keeps M in LDS whenever the copy fits beside the rest
    const size_t lds_m = ch_lds_bytes_mlds(npa, mmax, NT, sizeof(T));
    const bool mlds = sizeof(T) == 4 && lds_m <= 160 * 1024;
    const size_t lds = mlds ? lds_m : ch_lds_bytes(npa, mmax, NT, sizeof(T));
    auto go = [&](auto k, int nt) {
        if (chunk_prepare(k, lds)) return -3;
        hipLaunchKernelGGL(k, dim3(chunk_grid(count)), dim3(nt), lds, stream, bv, count, max_iter,
                           tol, npa, mmax, M, J, a0, aref, D, a_init, a_out, fac, mask, status, iters);
        return hipGetLastError() == hipSuccess ? 0 : -3;
    };
    if constexpr (sizeof(T) == 4) {
        if (mlds) return NT == 64 ? go(k_forward_chunk<T, 64, true>, 64)
                                  : go(k_forward_chunk<T, 256, true>, 256);
    }
    return NT == 64 ? go(k_forward_chunk<T, 64, false>, 64) : go(k_forward_chunk<T, 256, false>, 256);
}

template <typename T>
int launch_chunk_vjp(const BatchView &bv, int count, int nmax, int mmax, const T *fac,
                     const uint8_t *mask, const T *M, const T *J, const T *a0, const T *aref,
                     const T *D, const T *a, const T *abar, T *a0bar, T *arefbar, T *Jbar,
                     T *Dbar, T *Mbar, hipStream_t stream) {
    const int npa = round16(nmax);
    const int NT = chunk_nt(nmax);
    const size_t lds = ch_lds_bytes(npa, mmax, NT, sizeof(T));
    if (NT == 64) {
        auto k = k_ift_vjp_chunk<T, 64>;
        if (chunk_prepare(k, lds)) return -3;
        hipLaunchKernelGGL(k, dim3(chunk_grid(count)), dim3(64), lds, stream, bv, count, npa, mmax,
                           fac, mask, M, J, a0, aref, D, a, abar, a0bar, arefbar, Jbar, Dbar, Mbar);
    } else {
        auto k = k_ift_vjp_chunk<T, 256>;
        if (chunk_prepare(k, lds)) return -3;
        hipLaunchKernelGGL(k, dim3(chunk_grid(count)), dim3(256), lds, stream, bv, count, npa, mmax,
                           fac, mask, M, J, a0, aref, D, a, abar, a0bar, arefbar, Jbar, Dbar, Mbar);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cs
