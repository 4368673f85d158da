// cs_wave.hpp -- one-wave forward kernel for mid-size FP32 instances.
//
// One 64-lane wave solves one instance (n <= 31, m <= 1024), with all of J
// resident in LDS for the whole solve (row stride NPA + 1, conflict-free), so
// J crosses HBM once per instance instead of twice per Newton step.  Lane l
// owns rows l, l + 64, ... for the residuals, the active set and q = J p;
// lane j < n owns coordinate j of a, a0, p, F and row j of M and of the
// Newton matrix.  One matrix-core pass per step forms the lower triangle of
//   [J | r]^T diag(D o A) [J | r]
// (v_mfma_f32_16x16x4f32, K-steps of four rows), whose first n columns give
// J^T diag(D o A) J (eq. 9) and whose row n gives J^T w (eq. 6): the residual
// is kept in the spare column n of the LDS copy of J.  The Cholesky keeps
// row i of the Newton matrix in lane i's registers and broadcasts each
// column through LDS; the triangular solves broadcast through lanes.  An
// unchanged active set reuses the previous factor.  The line search is the
// team one with 64 threads (rows from LDS, wave reductions only).
#pragma once

#include "cs_device.hpp"

namespace cs {

// Padded width: n + 1 columns (J and the residual), a multiple of 16.
__host__ __device__ inline int wave_npa(int n) { return (n + 1 + 15) & ~15; }
__host__ __device__ inline int wave_rows(int m) { return (m + 63) & ~63; }

// LDS: J (mp x (NPA + 1)), H (NPA x (NPA + 1)), five row arrays (r, q, D,
// aref, weights), two NPA vectors, reduction scratch, the active bytes.
__host__ __device__ inline size_t wave_lds_bytes(int npa, int mmax) {
    const size_t ld = (size_t)npa + 1, mp = (size_t)wave_rows(mmax);
    return (mp * ld + (size_t)npa * ld + 5 * mp + 2 * (size_t)npa + 16) * sizeof(float) + mp;
}

typedef float wf4 __attribute__((ext_vector_type(4)));

// Value of v in lane k (k a compile-time or wave-uniform index).
__device__ inline float wave_lane(float v, int k) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

template <int NPA>
__global__ __launch_bounds__(64) void k_forward_wave(
    BatchView bv, int count, int max_iter, float tol, int mmax, const float *__restrict__ gM,
    const float *__restrict__ gJ, const float *__restrict__ ga0, const float *__restrict__ garef,
    const float *__restrict__ gD, const float *__restrict__ gainit, float *__restrict__ gaout,
    float *__restrict__ gfac, uint8_t *__restrict__ gmask, int32_t *__restrict__ gstatus,
    int32_t *__restrict__ giters) {
    static_assert(NPA == 16 || NPA == 32, "padded width");
    constexpr int LD = NPA + 1;
    constexpr int NTL = (NPA / 16) * (NPA / 16 + 1) / 2;   // lower-triangle tiles
    extern __shared__ __align__(16) unsigned char smem[];
    const int mp = wave_rows(mmax);
    float *Js = reinterpret_cast<float *>(smem);
    float *Hs = Js + (size_t)mp * LD;
    float *Rs = Hs + NPA * LD, *Qs = Rs + mp, *Ds = Qs + mp, *As_ref = Ds + mp, *Wc = As_ref + mp;
    float *Fs = Wc + mp, *Vs = Fs + NPA, *red = Vs + NPA;
    uint8_t *Ab = reinterpret_cast<uint8_t *>(red + 16);
    const int l = threadIdx.x;
    const int kq = l >> 4, idx = l & 15;

    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        const int n = I.n, m = I.m;
        const int m4 = (m + 3) & ~3;
        const float *M = gM + I.onn, *J = gJ + I.omn;
        bool bad = false;
        // J into LDS (columns < n), rows m .. m4-1 zero in every column
        {
            int rr = l / n, cc = l - (l / n) * n;
            const int dr = 64 / n, dc = 64 - dr * n;
            for (int e = l; e < m * n; e += 64) {
                const float x = J[e];
                Js[rr * LD + cc] = x;
                bad |= !finite_val(x);
                rr += dr;
                cc += dc;
                if (cc >= n) { cc -= n; ++rr; }
            }
            for (int e = l; e < (m4 - m) * LD; e += 64) Js[m * LD + e] = 0.f;
        }
        for (int i = l; i < m; i += 64) {
            const float d = gD[I.om + i], ar = garef[I.om + i];
            Ds[i] = d;
            As_ref[i] = ar;
            Ab[i] = 0;
            bad |= !finite_val(d) || !finite_val(ar);
        }
        for (int i = m + l; i < m4; i += 64) Wc[i] = 0.f;
        // lane j < n: row j of M, a_j, a0_j
        float Mrow[NPA];
#pragma unroll
        for (int c = 0; c < NPA; ++c) {
            const float x = (l < n && c < n) ? M[l * n + c] : 0.f;
            bad |= !finite_val(x);
            Mrow[c] = x;
        }
        float aj = 0.f, a0j = 0.f;
        if (l < n) {
            a0j = ga0[I.on + l];
            aj = gainit ? gainit[I.on + l] : a0j;
            bad |= !finite_val(a0j) || !finite_val(aj);
        }
        const bool anybad = __syncthreads_or(bad);

        // Cholesky of the rows h (lane i holds row i, entries c <= i), in
        // place; returns false when a pivot is not positive.  Entries above
        // the diagonal are updated too and never used.
        auto factor = [&](float (&h)[NPA]) -> bool {
            bool ok = true;
#pragma unroll
            for (int j = 0; j < NPA; ++j) {
                if (j < n) {
                    const float piv = wave_lane(h[j], j);
                    ok = ok && (piv > 0.f);
                    const float ljj = sqrtf(piv);
                    const float inv = 1.f / ljj;
                    h[j] = (l == j) ? ljj : h[j] * inv;
                    if (l < NPA) Vs[l] = h[j];   // column j of L (rows >= n hold 0)
                    __syncthreads();
#pragma unroll
                    for (int k = j + 1; k < NPA; ++k)
                        if (k < n) h[k] -= h[j] * Vs[k];
                    __syncthreads();
                }
            }
            return ok;
        };

        int st = 0, k = 0;
        float h[NPA];
        if (anybad) {
            st = ST_NONFINITE;
        } else {
#pragma unroll
            for (int c = 0; c < NPA; ++c) h[c] = Mrow[c];
            if (!factor(h)) st = ST_NOTSPD;
        }
        if (st == 0) {
            // trace of M, Md = M (a - a0) (lane j holds entry j)
            float trM = 0.f, Md = 0.f;
            {
                const float dj = aj - a0j;
#pragma unroll
                for (int c = 0; c < NPA; ++c) {
                    trM += wave_lane(Mrow[c], c);       // M_cc from lane c
                    Md += Mrow[c] * wave_lane(dj, c);
                }
            }
            float step_inf = -1.f;
            int lsfail = 0;
            bool have_factor = false;
            for (k = 0;; ++k) {
                // residuals and active set of the lane's rows; r into column n
                float av[NPA];
#pragma unroll
                for (int c = 0; c < NPA; ++c) av[c] = wave_lane(aj, c);
                bool changed = false;
                for (int i = l; i < m; i += 64) {
                    const float *row = Js + i * LD;
                    float s0 = 0.f, s1 = 0.f;
#pragma unroll
                    for (int c = 0; c < NPA; c += 2) {
                        if (c < n) s0 += row[c] * av[c];
                        if (c + 1 < n) s1 += row[c + 1] * av[c + 1];
                    }
                    const float r = s0 + s1 - As_ref[i];
                    const uint8_t an = r < 0.f;
                    changed |= an != Ab[i];
                    Ab[i] = an;
                    Rs[i] = r;
                    Js[i * LD + n] = r;
                    Wc[i] = an ? Ds[i] : 0.f;
                }
                const bool same = !__syncthreads_or(changed);
                // lower triangle of [J | r]^T diag(Wc) [J | r] on the matrix cores
                wf4 acc[NTL];
#pragma unroll
                for (int t = 0; t < NTL; ++t) acc[t] = wf4{0.f, 0.f, 0.f, 0.f};
                for (int ks = 0; ks < m4 / 4; ++ks) {
                    const int row = 4 * ks + kq;
                    const float wr = Wc[row];
                    const float *jr = Js + row * LD + idx;
                    float cb[NPA / 16];
#pragma unroll
                    for (int b = 0; b < NPA / 16; ++b) cb[b] = jr[16 * b];
#pragma unroll
                    for (int ti = 0, t = 0; ti < NPA / 16; ++ti)
#pragma unroll
                        for (int tj = 0; tj <= ti; ++tj, ++t)
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[ti], wr * cb[tj], acc[t], 0, 0, 0);
                }
                // H part to Hs (rows < n), J^T w (row n) to Fs
#pragma unroll
                for (int ti = 0, t = 0; ti < NPA / 16; ++ti)
#pragma unroll
                    for (int tj = 0; tj <= ti; ++tj, ++t)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int row = 16 * ti + 4 * kq + q, col = 16 * tj + idx;
                            if (row < n && col <= row) Hs[row * LD + col] = acc[t][q];
                            if (row == n && col < n) Fs[col] = acc[t][q];
                        }
                __syncthreads();
                const float Fj = (l < n) ? Md + Fs[l] : 0.f;
                float g2 = Fj * Fj, an = fabsf(aj);
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    g2 += __shfl_xor(g2, o, 64);
                    an = fmaxf(an, __shfl_xor(an, o, 64));
                }
                if (!(same && have_factor)) {
#pragma unroll
                    for (int c = 0; c < NPA; ++c)
                        h[c] = (l < n && c <= l) ? Hs[l * LD + c] + Mrow[c] : 0.f;
                    if (!factor(h)) { st = ST_NOTSPD; break; }
                    have_factor = true;
                }
                if (sqrtf(g2) <= tol * trM ||
                    (k > 0 && step_inf >= 0.f && same && step_inf <= tol * (1.f + an))) {
                    st = ST_CONVERGED;
                    break;
                }
                if (k == max_iter) { st = ST_MAXITER; break; }
                // p = -H^{-1} F: forward L y = -F (y in lane j), then L^T p = y
                float y = -Fj;
#pragma unroll
                for (int j = 0; j < NPA; ++j) {
                    if (j < n) {
                        const float yj = wave_lane(y / h[j], j);
                        y = (l == j) ? yj : ((l > j) ? y - h[j] * yj : y);
                    }
                }
                // L rows to LDS for the transposed solve
#pragma unroll
                for (int c = 0; c < NPA; ++c)
                    if (l < n && c <= l) Hs[l * LD + c] = h[c];
                __syncthreads();
                float pj = y;
#pragma unroll
                for (int j = NPA - 1; j >= 0; --j) {
                    if (j < n) {
                        const float xj = wave_lane(pj / h[j], j);
                        const float lji = Hs[j * LD + (l < n ? l : 0)];
                        pj = (l == j) ? xj : ((l < j) ? pj - lji * xj : pj);
                    }
                }
                if (l >= n) pj = 0.f;
                // q = J p for the lane's rows; M p and the line-search coefficients
                float pv[NPA];
#pragma unroll
                for (int c = 0; c < NPA; ++c) pv[c] = wave_lane(pj, c);
                for (int i = l; i < m; i += 64) {
                    const float *row = Js + i * LD;
                    float s0 = 0.f, s1 = 0.f;
#pragma unroll
                    for (int c = 0; c < NPA; c += 2) {
                        if (c < n) s0 += row[c] * pv[c];
                        if (c + 1 < n) s1 += row[c + 1] * pv[c + 1];
                    }
                    Qs[i] = s0 + s1;
                }
                float Mp = 0.f;
#pragma unroll
                for (int c = 0; c < NPA; ++c) Mp += Mrow[c] * pv[c];
                float c0 = pj * Mp, b0 = pj * Md;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    c0 += __shfl_xor(c0, o, 64);
                    b0 += __shfl_xor(b0, o, 64);
                }
                __syncthreads();
                uint32_t bits;
                float cpiece;
                int fl;
                const float alpha = team_line_search<64>(m, Rs, Qs, Ds, c0, b0, red, bits, cpiece, fl);
                lsfail |= fl;
                float si = fabsf(alpha * pj);
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) si = fmaxf(si, __shfl_xor(si, o, 64));
                step_inf = si;
                aj += alpha * pj;
                Md += alpha * Mp;
                __syncthreads();
            }
            if (lsfail) st |= ST_LSFAIL;
        }
        const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
        const float nanv = __builtin_nanf("");
        if (l < n) gaout[I.on + l] = ok ? aj : nanv;
        // factor: lane i's row of L (diagonal included) through LDS
#pragma unroll
        for (int c = 0; c < NPA; ++c)
            if (l < n && c <= l) Hs[l * LD + c] = h[c];
        __syncthreads();
        {
            float *fac = gfac + fac_offset(I);
            int j = 0, c = l;
            while (c > j) { c -= j + 1; ++j; }
            for (int e = l; e < n * (n + 1) / 2; e += 64) {
                fac[e] = ok ? Hs[j * LD + c] : nanv;
                c += 64;
                while (c > j) { c -= j + 1; ++j; }
            }
        }
        for (int i = l; i < m; i += 64) gmask[I.om + i] = ok ? Ab[i] : 0;
        if (l == 0) {
            gstatus[I.b] = st;
            if (giters) giters[I.b] = k;
        }
        __syncthreads();
    }
}

// Host side --------------------------------------------------------------

inline bool wave_supported(int nmax, int mmax, int s) {
    if (s != 4 || nmax > 31 || mmax > 1024) return false;
    return wave_lds_bytes(wave_npa(nmax), mmax) <= 160 * 1024;
}

inline int launch_wave_forward(const BatchView &bv, int count, int nmax, int mmax, int max_iter,
                               float tol, const float *M, const float *J, const float *a0,
                               const float *aref, const float *D, const float *a_init,
                               float *a_out, float *fac, uint8_t *mask, int32_t *status,
                               int32_t *iters, hipStream_t stream) {
    const int npa = wave_npa(nmax);
    const size_t lds = wave_lds_bytes(npa, mmax);
    const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
    if (npa == 16) {
        auto k = k_forward_wave<16>;
        if (!ensure_lds(reinterpret_cast<const void *>(k), lds)) return -3;
        hipLaunchKernelGGL(k, dim3(grid), dim3(64), lds, stream, bv, count, max_iter, tol, mmax, M, J,
                           a0, aref, D, a_init, a_out, fac, mask, status, iters);
    } else {
        auto k = k_forward_wave<32>;
        if (!ensure_lds(reinterpret_cast<const void *>(k), lds)) return -3;
        hipLaunchKernelGGL(k, dim3(grid), dim3(64), lds, stream, bv, count, max_iter, tol, mmax, M, J,
                           a0, aref, D, a_init, a_out, fac, mask, status, iters);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cs
