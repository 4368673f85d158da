// cs_chunk.hpp -- team kernels that stream the rows of J through LDS.
//
// One workgroup (NT = 64 for n <= 32, 256 otherwise) solves one instance at
// a time.  Each Newton pass reads J in chunks of CR rows: a chunk is copied
// to LDS with coalesced loads, then the residual of its rows (NT / CR lanes
// per row), the gradient J^T w (lanes over columns) and the Newton-matrix
// contribution J_c^T diag(D o A) J_c are formed from LDS.  In FP32 the
// contraction runs on the matrix cores (v_mfma_f32_16x16x4f32 on 16 x 16
// tiles of the lower triangle, tiles spread over the waves, accumulators in
// registers); in FP64 lanes accumulate lower-triangle entries on the VALU.
// A second pass forms q = J p for the line search.  H (row stride npa, the
// padded n), the row arrays r, q, D, aref and the chunk buffer live in LDS.
#pragma once

#include "cs_device.hpp"

namespace cs {

constexpr int CR = 64;   // rows per chunk

__host__ __device__ inline int round16(int n) { return (n + 15) & ~15; }

template <typename T>
struct ChLds {
    T *H, *diag, *a, *a0, *F, *p, *y, *v, *u, *red;
    T *r, *q, *Dv, *ar, *Jc, *Wc, *Wr;
    uint8_t *A;
};

__host__ __device__ inline size_t ch_lds_bytes(int npa, int mmax, int NT, size_t s) {
    const size_t ldj = (size_t)npa + 1;
    const size_t nT = (size_t)npa * npa + 9 * (size_t)npa + 16 * (size_t)(NT / 64) +
                      4 * (size_t)mmax + CR * ldj + 2 * CR;
    return nT * s + (size_t)mmax + 64;
}

template <typename T>
__device__ inline ChLds<T> ch_carve(unsigned char *smem, int npa, int mmax, int NT) {
    ChLds<T> L;
    T *p = reinterpret_cast<T *>(smem);
    L.H = p; p += (size_t)npa * npa;
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
    L.Jc = p; p += (size_t)CR * (npa + 1);
    L.Wc = p; p += CR;
    L.Wr = p; p += CR;
    L.A = reinterpret_cast<uint8_t *>(p);
    return L;
}

// Copy rows [c CR, c CR + CR) of J (row-major, n columns) into the chunk
// buffer (row stride ldj).  Rows past m are left as they are.
template <int NT, typename T>
__device__ inline void ch_load(const T *__restrict__ J, int n, int m, int c, int ldj, T *Jc) {
    const int r0 = c * CR;
    const int rows = min(CR, m - r0);
    const int cnt = rows * n;
    const T *src = J + (int64_t)r0 * n;
    for (int e = threadIdx.x; e < cnt; e += NT) {
        const int rho = e / n, j = e - rho * n;
        Jc[rho * ldj + j] = src[e];
    }
}

// Dot products of the chunk's rows with the LDS vector x; NT / CR lanes per
// row, combined with butterflies.  Returns the full dot in every lane of the
// row's lane group; rho is this lane's chunk row.
template <int NT, typename T>
__device__ inline T ch_row_dot(int n, int ldj, const T *Jc, const T *x, int &rho, int &part) {
    constexpr int TPR = NT / CR;
    rho = threadIdx.x / TPR;
    part = threadIdx.x % TPR;
    T s = T(0);
    for (int j = part; j < n; j += TPR) s += Jc[rho * ldj + j] * x[j];
#pragma unroll
    for (int o = 1; o < TPR; o <<= 1) s += __shfl_xor(s, o, 64);
    return s;
}

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
    // acc += J_c^T diag(Wc) J_c over the chunk (rows past m carry Wc = 0)
    __device__ inline void add_chunk(int ldj, const float *Jc, const float *Wc) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int kq = lane >> 4, idx = lane & 15;
#pragma unroll
        for (int s = 0; s < MAXT; ++s) {
            if (wave + NW * s < ntiles) {
                const float *ca = Jc + 16 * ti[s] + idx;
                const float *cb = Jc + 16 * tj[s] + idx;
#pragma unroll 4
                for (int kb = 0; kb < CR / 4; ++kb) {
                    const int row = kb * 4 + kq;
                    const float av = ca[row * ldj];
                    const float bv = Wc[row] * cb[row * ldj];
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[s], 0, 0, 0);
                }
            }
        }
    }
    // H (lower, stride npa) = M + acc
    __device__ inline void store(int n, int npa, const float *__restrict__ M, float *H) const {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int kq = lane >> 4, idx = lane & 15;
#pragma unroll
        for (int s = 0; s < MAXT; ++s) {
            if (wave + NW * s < ntiles) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * ti[s] + 4 * kq + r, col = 16 * tj[s] + idx;
                    if (row < n && col <= row) H[row * npa + col] = acc[s][r] + M[row * n + col];
                }
            }
        }
    }
};

// FP64: lower-triangle entries e = tid + NT s on the VALU.
template <int NT> struct ChAcc<double, NT> {
    static constexpr int MAXE = NT == 64 ? 9 : 33;   // ceil(n (n+1) / 2 / NT)
    double acc[MAXE];
    int ej[MAXE], el[MAXE], ne;

    __device__ inline void init(int n) {
        ne = n * (n + 1) / 2;
#pragma unroll
        for (int s = 0; s < MAXE; ++s) {
            const int e = threadIdx.x + NT * s;
            int j = 0;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            ej[s] = j;
            el[s] = e - j * (j + 1) / 2;
            acc[s] = 0.0;
        }
    }
    __device__ inline void zero() {
#pragma unroll
        for (int s = 0; s < MAXE; ++s) acc[s] = 0.0;
    }
    __device__ inline void add_chunk(int ldj, const double *Jc, const double *Wc) {
#pragma unroll
        for (int s = 0; s < MAXE; ++s) {
            if ((int)threadIdx.x + NT * s < ne) {
                double h = acc[s];
                for (int rho = 0; rho < CR; ++rho)
                    h += Wc[rho] * Jc[rho * ldj + ej[s]] * Jc[rho * ldj + el[s]];
                acc[s] = h;
            }
        }
    }
    __device__ inline void store(int n, int npa, const double *__restrict__ M, double *H) const {
#pragma unroll
        for (int s = 0; s < MAXE; ++s)
            if ((int)threadIdx.x + NT * s < ne)
                H[ej[s] * npa + el[s]] = acc[s] + M[ej[s] * n + el[s]];
    }
};

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_forward_chunk(
    BatchView bv, int count, int max_iter, T tol, int npa, int mmax, const T *__restrict__ gM,
    const T *__restrict__ gJ, const T *__restrict__ ga0, const T *__restrict__ garef,
    const T *__restrict__ gD, const T *__restrict__ gainit, T *__restrict__ gaout,
    T *__restrict__ gfac, uint8_t *__restrict__ gmask, int32_t *__restrict__ gstatus,
    int32_t *__restrict__ giters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const ChLds<T> L = ch_carve<T>(smem, npa, mmax, NT);
    const int tid = threadIdx.x;
    const int ldj = npa + 1;
    // stale chunk rows are multiplied by zero weights: keep them finite
    for (int e = tid; e < CR * ldj; e += NT) L.Jc[e] = T(0);
    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        const int n = I.n, m = I.m;
        const int nch = (m + CR - 1) / CR;
        const T *M = gM + I.onn, *J = gJ + I.omn;
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
        for (int e = tid; e < n * n; e += NT) {
            const T x = M[e];
            L.H[(e / n) * npa + (e % n)] = x;
            bad |= !finite_val(x);
        }
        for (int e = tid; e < m * n; e += NT) bad |= !finite_val(J[e]);
        const int anybad = __syncthreads_or(bad);
        int st = 0, k = 0;
        if (anybad) st = ST_NONFINITE;
        else if (!team_cholesky<NT>(L.H, L.diag, n, npa)) st = ST_NOTSPD;
        ChAcc<T, NT> acc;
        acc.init(sizeof(T) == 4 ? npa : n);
        if (st == 0) {
            T trM = T(0);
            for (int j = 0; j < n; ++j) trM += M[(int64_t)j * n + j];
            T step_inf = T(-1);
            int lsfail = 0;
            for (k = 0;; ++k) {
                // pass A: r, A, F = M (a - a0) + J^T w and H = M + J^T diag(D o A) J
                for (int j = tid; j < n; j += NT) {
                    T f = T(0);
#pragma unroll 4
                    for (int l = 0; l < n; ++l) f += M[(int64_t)l * n + j] * (L.a[l] - L.a0[l]);
                    L.F[j] = f;
                }
                acc.zero();
                bool changed = false;
                for (int c = 0; c < nch; ++c) {
                    __syncthreads();
                    ch_load<NT>(J, n, m, c, ldj, L.Jc);
                    __syncthreads();
                    int rho, part;
                    const T s = ch_row_dot<NT>(n, ldj, L.Jc, L.a, rho, part);
                    if (part == 0) {
                        const int i = c * CR + rho;
                        if (i < m) {
                            const T r = s - L.ar[i];
                            const uint8_t an = r < T(0);
                            changed |= an != L.A[i];
                            L.A[i] = an;
                            L.r[i] = r;
                            const T wd = an ? L.Dv[i] : T(0);
                            L.Wc[rho] = wd;
                            L.Wr[rho] = wd * r;
                        } else {
                            L.Wc[rho] = T(0);
                            L.Wr[rho] = T(0);
                        }
                    }
                    __syncthreads();
                    for (int j = tid; j < n; j += NT) {
                        T f = L.F[j];
                        for (int rr = 0; rr < CR; ++rr) f += L.Wr[rr] * L.Jc[rr * ldj + j];
                        L.F[j] = f;
                    }
                    acc.add_chunk(ldj, L.Jc, L.Wc);
                }
                const bool same = !__syncthreads_or(changed);
                acc.store(n, npa, M, L.H);
                __syncthreads();
                T g2 = T(0), anorm = T(0);
                for (int j = 0; j < n; ++j) {
                    g2 += L.F[j] * L.F[j];
                    anorm = fmax(anorm, fabs(L.a[j]));
                }
                if (!team_cholesky<NT>(L.H, L.diag, n, npa)) { st = ST_NOTSPD; break; }
                if (sqrt(g2) <= tol * trM ||
                    (k > 0 && step_inf >= T(0) && same && step_inf <= tol * (T(1) + anorm))) {
                    st = ST_CONVERGED;
                    break;
                }
                if (k == max_iter) { st = ST_MAXITER; break; }
                for (int j = tid; j < n; j += NT) L.y[j] = -L.F[j];
                __syncthreads();
                team_chol_solve<NT>(L.H, L.diag, L.y, L.p, n, npa);
                // pass B: q = J p
                for (int c = 0; c < nch; ++c) {
                    __syncthreads();
                    ch_load<NT>(J, n, m, c, ldj, L.Jc);
                    __syncthreads();
                    int rho, part;
                    const T s = ch_row_dot<NT>(n, ldj, L.Jc, L.p, rho, part);
                    const int i = c * CR + rho;
                    if (part == 0 && i < m) L.q[i] = s;
                }
                for (int j = tid; j < n; j += NT) {
                    T mp = T(0), md = T(0);
#pragma unroll 4
                    for (int l = 0; l < n; ++l) {
                        const T mlj = M[(int64_t)l * n + j];   // = M[j][l]: M is symmetric
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
        }
        const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
        const T nanv = T(__builtin_nan(""));
        for (int j = tid; j < n; j += NT) gaout[I.on + j] = ok ? L.a[j] : nanv;
        T *fac = gfac + fac_offset(I);
        for (int e = tid; e < n * (n + 1) / 2; e += NT) {
            int j = 0;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int l = e - j * (j + 1) / 2;
            fac[e] = ok ? (l < j ? L.H[j * npa + l] : L.diag[j]) : nanv;
        }
        for (int i = tid; i < m; i += NT) gmask[I.om + i] = ok ? L.A[i] : 0;
        if (tid == 0) {
            gstatus[I.b] = st;
            if (giters) giters[I.b] = k;
        }
        __syncthreads();
    }
}

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
    const int ldj = npa + 1;
    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        const int n = I.n, m = I.m;
        const int nch = (m + CR - 1) / CR;
        const T *M = gM + I.onn, *J = gJ + I.omn;
        const T *fac = gfac + fac_offset(I);
        for (int e = tid; e < n * (n + 1) / 2; e += NT) {
            int j = 0;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int l = e - j * (j + 1) / 2;
            if (l < j) L.H[j * npa + l] = fac[e];
            else L.diag[j] = fac[e];
        }
        for (int j = tid; j < n; j += NT) {
            L.a[j] = ga[I.on + j];
            L.a0[j] = ga0[I.on + j];
            L.y[j] = gabar[I.on + j];
            L.F[j] = T(0);
        }
        for (int i = tid; i < m; i += NT) {
            L.Dv[i] = gD[I.om + i];
            L.ar[i] = garef[I.om + i];
            L.A[i] = gmask[I.om + i];
        }
        __syncthreads();
        // lambda = H^{-1} abar with one refinement step, H v = M v + J^T (D o A* o J v)
        team_chol_solve<NT>(L.H, L.diag, L.y, L.u, n, npa);
        for (int c = 0; c < nch; ++c) {
            __syncthreads();
            ch_load<NT>(J, n, m, c, ldj, L.Jc);
            __syncthreads();
            int rho, part;
            const T s = ch_row_dot<NT>(n, ldj, L.Jc, L.u, rho, part);
            const int i = c * CR + rho;
            if (part == 0) L.Wr[rho] = (i < m && L.A[i]) ? L.Dv[i] * s : T(0);
            __syncthreads();
            for (int j = tid; j < n; j += NT) {
                T f = L.F[j];
                for (int rr = 0; rr < CR; ++rr) f += L.Wr[rr] * L.Jc[rr * ldj + j];
                L.F[j] = f;
            }
        }
        __syncthreads();
        for (int j = tid; j < n; j += NT) {
            T s = gabar[I.on + j] - L.F[j];
#pragma unroll 4
            for (int l = 0; l < n; ++l) s -= M[(int64_t)l * n + j] * L.u[l];
            L.y[j] = s;
        }
        __syncthreads();
        team_chol_solve<NT>(L.H, L.diag, L.y, L.p, n, npa);
        for (int j = tid; j < n; j += NT) L.u[j] += L.p[j];
        __syncthreads();
        // per-row cotangents and J-bar, chunk by chunk
        for (int c = 0; c < nch; ++c) {
            __syncthreads();
            ch_load<NT>(J, n, m, c, ldj, L.Jc);
            __syncthreads();
            int rho, part;
            const T ja = ch_row_dot<NT>(n, ldj, L.Jc, L.a, rho, part);
            const T sig = ch_row_dot<NT>(n, ldj, L.Jc, L.u, rho, part);
            const int i = c * CR + rho;
            if (part == 0) {
                if (i < m) {
                    const bool act = L.A[i] != 0;
                    const T r = ja - L.ar[i];
                    const T wv = act ? L.Dv[i] * r : T(0);
                    const T arb = act ? L.Dv[i] * sig : T(0);
                    if (garefbar) garefbar[I.om + i] = arb;
                    if (gDbar) gDbar[I.om + i] = act ? -r * sig : T(0);
                    L.Wc[rho] = wv;
                    L.Wr[rho] = arb;
                } else {
                    L.Wc[rho] = T(0);
                    L.Wr[rho] = T(0);
                }
            }
            __syncthreads();
            if (gJbar) {
                const int r0 = c * CR;
                const int cnt = min(CR, m - r0) * n;
                T *dst = gJbar + I.omn + (int64_t)r0 * n;
                for (int e = tid; e < cnt; e += NT) {
                    const int rr = e / n, j = e - rr * n;
                    dst[e] = -(L.Wc[rr] * L.u[j] + L.Wr[rr] * L.a[j]);
                }
            }
        }
        if (ga0bar) {
            for (int j = tid; j < n; j += NT) {
                T s = T(0);
                for (int l = 0; l < n; ++l) s += M[(int64_t)l * n + j] * L.u[l];
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
    const size_t lds = ch_lds_bytes(npa, mmax, NT, sizeof(T));
    if (NT == 64) {
        auto k = k_forward_chunk<T, 64>;
        if (chunk_prepare(k, lds)) return -3;
        hipLaunchKernelGGL(k, dim3(chunk_grid(count)), dim3(64), lds, stream, bv, count, max_iter,
                           tol, npa, mmax, M, J, a0, aref, D, a_init, a_out, fac, mask, status, iters);
    } else {
        auto k = k_forward_chunk<T, 256>;
        if (chunk_prepare(k, lds)) return -3;
        hipLaunchKernelGGL(k, dim3(chunk_grid(count)), dim3(256), lds, stream, bv, count, max_iter,
                           tol, npa, mmax, M, J, a0, aref, D, a_init, a_out, fac, mask, status, iters);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
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
