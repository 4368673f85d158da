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

#include <type_traits>

#include "cs_device.hpp"

namespace cs {

// Padded width: n + 1 columns (J and the residual), a multiple of 16.
__host__ __device__ inline int wave_npa(int n) { return (n + 1 + 15) & ~15; }
__host__ __device__ inline int wave_rows(int m) { return m < 64 ? 64 : (m + 63) & ~63; }

// LDS: J (mp x (NPA + 1)), H (NPA x (NPA + 1)), the weights of the active
// rows (compacted), two NPA vectors, the indices of the active rows.
__host__ __device__ inline size_t wave_lds_bytes(int npa, int mmax) {
    const size_t ld = (size_t)npa + 1, mp = (size_t)wave_rows(mmax);
    return (mp * ld + (size_t)npa * ld + mp + 2 * (size_t)npa + mp) * sizeof(float);
}

// Rows per lane for up to mmax rows.
inline int wave_rpl(int mmax) {
    const int r = (mmax + 63) / 64;
    return r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : r <= 8 ? 8 : 16;
}

typedef float wf4 __attribute__((ext_vector_type(4)));


// Value of v in lane k (k a compile-time or wave-uniform index).
__device__ inline float wave_lane(float v, int k) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

// Wave-wide sum and max, every lane receives the result: DPP within each
// row of 16 lanes (quad xor 1 and 2, half-row and row mirrors), then the
// four row totals from lanes 0, 16, 32, 48.  Fixed order: reproducible.
template <int CTRL> __device__ inline float wv_dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ inline float wave_total(float v) {
    v += wv_dpp<0xB1>(v);
    v += wv_dpp<0x4E>(v);
    v += wv_dpp<0x141>(v);
    v += wv_dpp<0x140>(v);
    return (wave_lane(v, 0) + wave_lane(v, 16)) + (wave_lane(v, 32) + wave_lane(v, 48));
}
__device__ inline float wave_maximum(float v) {
    v = fmaxf(v, wv_dpp<0xB1>(v));
    v = fmaxf(v, wv_dpp<0x4E>(v));
    v = fmaxf(v, wv_dpp<0x141>(v));
    v = fmaxf(v, wv_dpp<0x140>(v));
    return fmaxf(fmaxf(wave_lane(v, 0), wave_lane(v, 16)), fmaxf(wave_lane(v, 32), wave_lane(v, 48)));
}

// Exact line search (Sec. III-B, eq. 10) with the lane's rows in registers;
// the safeguarded piece Newton of team_line_search (rows past m carry
// D = q = 0, so they are never active).
template <int RPL>
__device__ inline float wave_line_search(const float (&r)[RPL], const float (&q)[RPL],
                                         const float (&D)[RPL], float c0, float b0, int &fail) {
    float dqq[RPL], dqr[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const float dq = D[t] * q[t];
        dqq[t] = dq * q[t];
        dqr[t] = dq * r[t];
    }
    auto piece = [&](float tr, float &c, float &b) {
        float sc = 0.f, sb = 0.f;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const bool pa = r[t] + tr * q[t] < 0.f;
            sc += pa ? dqq[t] : 0.f;
            sb += pa ? dqr[t] : 0.f;
        }
        c = c0 + wave_total(sc);
        b = b0 + wave_total(sb);
    };
    float t = 1.f, c, b;
    piece(t, c, b);
    float lo = 0.f, hi = __builtin_huge_valf(), alpha = t;
    fail = 1;
    const float eps = 1.1920929e-7f;
    for (int it = 0; it < 96; ++it) {
        const float g = c * t + b;
        if (g == 0.f) { alpha = t; fail = 0; break; }
        if (g < 0.f) lo = t; else hi = t;
        if (hi < __builtin_huge_valf() && hi - lo <= 32.f * eps * hi) { alpha = t; fail = 0; break; }
        float cand = -b / c;
        const bool newton = (cand > lo) && (cand < hi);
        if (!newton) cand = (hi < __builtin_huge_valf()) ? 0.5f * (lo + hi) : 2.f * lo + 1.f;
        float nc, nbv;
        piece(cand, nc, nbv);
        // the piece is unchanged when its sums come out bitwise equal (same
        // rows, same partials, same reduction order); a different row set
        // with equal sums has the same linear phi' there, whose root is cand
        const bool same = (nc == c) && (nbv == b);
        c = nc;
        b = nbv;
        t = cand;
        alpha = cand;
        if (newton && same) { fail = 0; break; }
    }
    return alpha;
}

template <int NPA, int RPL>
__global__ __launch_bounds__(64) void k_forward_wave(
    BatchView bv, int count, int max_iter, float tol, int mmax, const float *__restrict__ gM,
    const float *__restrict__ gJ, const float *__restrict__ ga0, const float *__restrict__ garef,
    const float *__restrict__ gD, const float *__restrict__ gainit, float *__restrict__ gaout,
    float *__restrict__ gfac, uint8_t *__restrict__ gmask, int32_t *__restrict__ gstatus,
    int32_t *__restrict__ giters) {
    static_assert(NPA == 16 || NPA == 32, "padded width");
    constexpr int LD = NPA + 1;
    constexpr int NB = NPA / 16;                     // column blocks
    constexpr int NTL = NB * (NB + 1) / 2;           // lower-triangle tiles
    extern __shared__ __align__(16) unsigned char smem[];
    const int mp = wave_rows(mmax);
    float *Js = reinterpret_cast<float *>(smem);
    float *Hs = Js + (size_t)mp * LD;
    float *Wc = Hs + NPA * LD;
    float *Fs = Wc + mp, *Vs = Fs + NPA;
    int *Lr = reinterpret_cast<int *>(Vs + NPA);    // active rows, compacted
    const int l = threadIdx.x;
    const int kq = l >> 4, idx = l & 15;

    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) {   // wave-uniform
            mark_bad(I, gstatus, giters, l == 0);
            continue;
        }
        const int n = I.n, m = I.m;
        const int m4 = (m + 3) & ~3;
        const float *M = gM + I.onn, *J = gJ + I.omn;
        bool bad = false;
        // J into LDS (columns < n); columns n .. NPA-1 of the live rows and
        // rows m .. m4-1 start at zero, so row products run over all NPA
        // columns (a and p are zero past n)
        {
            // eight coalesced loads in flight per lane (clamped indices, no
            // predicates), then the LDS stores along the (row, column) walk
            const int tot = m * n;
            int rr = l / n, cc = l - (l / n) * n;
            const int dr = 64 / n, dc = 64 - dr * n;
            for (int e0 = 0; e0 < tot; e0 += 64 * 8) {
                float x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = J[min(e0 + l + 64 * u, tot - 1)];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (e0 + l + 64 * u < tot) {
                        Js[rr * LD + cc] = x[u];
                        bad |= !finite_val(x[u]);
                    }
                    rr += dr;
                    cc += dc;
                    if (cc >= n) { cc -= n; ++rr; }
                }
            }
            for (int e = l; e < (m4 - m) * LD; e += 64) Js[m * LD + e] = 0.f;
            for (int i = l; i < m; i += 64)
                for (int c = n; c < NPA; ++c) Js[i * LD + c] = 0.f;
        }
        // the lane's rows l + 64 t: D and aref in registers (zero past m)
        float Dr[RPL], ar[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int i = l + 64 * t;
            Dr[t] = i < m ? gD[I.om + i] : 0.f;
            ar[t] = i < m ? garef[I.om + i] : 0.f;
            bad |= !finite_val(Dr[t]) || !finite_val(ar[t]);
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

        // Cholesky of the rows h (lane i holds row i), in place, ending
        // strictly lower: the diagonal L_ii goes to dl and 1 / L_ii to idl,
        // and the diagonal and everything right of it are cleared at the
        // end.  Right-looking with register broadcasts: after
        // column j is scaled, its entries L_kj (lane k's h[j]) are read into
        // scalar registers and every lane updates its row, with no LDS round
        // trip or barrier on the per-column chain.  Branch-free over NC
        // columns (a branch that changes h[] makes the compiler copy the
        // whole row at its join); NC >= n is a compile-time 16, 20, 24, 28
        // or 32 chosen per instance, and columns n .. NC-1 (zero rows and columns)
        // take pivot 1.  False when a pivot of the first n columns is not
        // positive.
        float idl = 1.f, dl = 1.f;
        auto factor_nc = [&](auto ncc, float (&h)[NPA]) -> bool {
            constexpr int NC = decltype(ncc)::value;
            bool ok = true;
            if constexpr (NC == 16) {
                // every row in lanes 0..15: column entries by DPP row
                // broadcast (they stay in vector registers; lanes 16..63 hold
                // zero rows and broadcast zeros among themselves); the pivot
                // by a lane read, so ok stays wave-uniform
                static_for<0, 16>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    const float pv = wave_lane(h[j], j);   // unconditional
                    const bool live = j < n;
                    const float piv = live ? pv : 1.f;
                    ok = ok && (!live || piv > 0.f);
                    h[j] *= __builtin_amdgcn_rsqf(piv);
                    static_for<j + 1, 16>([&](auto kc) {
                        constexpr int k2 = decltype(kc)::value;
                        h[k2] -= h[j] * row_bcast16<k2>(h[j]);
                    });
                });
            } else {
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const bool live = j < n;
                    const float pv = wave_lane(h[j], j);   // unconditional: no branch around it
                    const float piv = live ? pv : 1.f;
                    ok = ok && (!live || piv > 0.f);
                    // lane j: the pivot times 1 / sqrt(pivot) = L_jj, final from here
                    h[j] *= __builtin_amdgcn_rsqf(piv);
#pragma unroll
                    for (int k2 = j + 1; k2 < NC; ++k2) h[k2] -= h[j] * wave_lane(h[j], k2);
                }
            }
            // lane l's diagonal is h[l]; the updates also reached entries right
            // of it (never read above).  One pass picks the diagonal and clears
            // the diagonal and everything right of it (no per-column lane
            // masks, so the column loop is one scheduling region).
            const int lo = opaque_lane(l);
            float d = 1.f;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                d = (c == lo) ? h[c] : d;
                h[c] = (c < lo) ? h[c] : 0.f;
            }
            dl = (lo < n) ? d : 1.f;    // rows past n are zero: identity there
            idl = __builtin_amdgcn_rcpf(dl);
            return ok;
        };
        // Calls f with the compile-time column count for this instance.
        auto with_nc = [&](auto f) {
            if constexpr (NPA == 16) {
                return f(std::integral_constant<int, 16>{});
            } else {
                if (n <= 16) return f(std::integral_constant<int, 16>{});
                if (n <= 20) return f(std::integral_constant<int, 20>{});
                if (n <= 24) return f(std::integral_constant<int, 24>{});
                if (n <= 28) return f(std::integral_constant<int, 28>{});
                return f(std::integral_constant<int, 32>{});
            }
        };
        auto factor = [&](float (&h)[NPA]) -> bool {
            return with_nc([&](auto ncc) { return factor_nc(ncc, h); });
        };
        // the lane's row of `src`, lower triangle and diagonal (zero elsewhere
        // and in lanes >= n), as the starting h of a factorisation
        // (every value read before any select: the empty asm keeps the
        // compiler from sinking each LDS read into a branch of its own that
        // waits for it)
        auto lower_row = [&](float (&h)[NPA], auto &&src) {
            const int lo = opaque_lane(l);
            const bool rowok = lo < n;
#pragma unroll
            for (int c = 0; c < NPA; ++c) h[c] = src(c);
#pragma unroll
            for (int c = 0; c < NPA; ++c) asm volatile("" : "+v"(h[c]));
#pragma unroll
            for (int c = 0; c < NPA; ++c) h[c] = (rowok && c <= lo) ? h[c] : 0.f;
        };

        int st = 0, k = 0;
        float h[NPA];
        uint32_t act = 0;   // activity of the lane's rows
        if (anybad) {
            st = ST_NONFINITE;
        } else {
            lower_row(h, [&](int c) { return Mrow[c]; });
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
            float rr[RPL];
            for (k = 0;; ++k) {
                // residuals and active set of the lane's rows; r into column n
                // (av[n] is zero: the previous residual there drops out)
                float av[NPA];
#pragma unroll
                for (int c = 0; c < NPA; ++c) av[c] = wave_lane(aj, c);
                uint32_t nact = 0;
                int cnt = 0;    // active rows so far (wave-uniform)
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const int i = l + 64 * t;
                    const float *row = Js + min(i, m4 > 0 ? m4 - 1 : 0) * LD;
                    float s0 = 0.f, s1 = 0.f;
#pragma unroll
                    for (int c = 0; c < NPA; c += 2) {
                        s0 += row[c] * av[c];
                        s1 += row[c + 1] * av[c + 1];
                    }
                    rr[t] = (i < m) ? s0 + s1 - ar[t] : 0.f;
                    const bool an = rr[t] < 0.f && i < m;
                    nact |= (an ? 1u : 0u) << t;
                    if (i < m) Js[i * LD + n] = rr[t];
                    // the active rows and their weights, compacted in row order
                    const uint64_t bal = __builtin_amdgcn_ballot_w64(an);
                    if (an) {
                        const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                        Lr[pos] = i;
                        Wc[pos] = Dr[t];
                    }
                    cnt += (int)__builtin_popcountll(bal);
                }
                // pad the list to whole K-steps with zero weights on row 0
                const int cnt4 = (cnt + 3) & ~3;
                if (l < cnt4 - cnt) {
                    Lr[cnt + l] = 0;
                    Wc[cnt + l] = 0.f;
                }
                const bool same = !__syncthreads_or(nact != act);
                act = nact;
                // lower triangle of [J | r]^T diag(D o A) [J | r] over the
                // active rows on the matrix cores; the next K-step's operands
                // (and the row index after it) load while this one runs
                wf4 acc[NTL];
#pragma unroll
                for (int t = 0; t < NTL; ++t) acc[t] = wf4{0.f, 0.f, 0.f, 0.f};
                const int nks = cnt4 / 4;
                if (nks > 0) {
                    float wr = Wc[kq];
                    float cb[NB];
                    {
                        const int r0 = Lr[kq];
#pragma unroll
                        for (int bb = 0; bb < NB; ++bb) cb[bb] = Js[r0 * LD + idx + 16 * bb];
                    }
                    int rnext = Lr[4 * min(1, nks - 1) + kq];
                    for (int ks = 0; ks < nks; ++ks) {
                        const float wn = Wc[4 * min(ks + 1, nks - 1) + kq];
                        float cn[NB];
#pragma unroll
                        for (int bb = 0; bb < NB; ++bb) cn[bb] = Js[rnext * LD + idx + 16 * bb];
                        rnext = Lr[4 * min(ks + 2, nks - 1) + kq];
#pragma unroll
                        for (int ti = 0, t = 0; ti < NB; ++ti)
#pragma unroll
                            for (int tj = 0; tj <= ti; ++tj, ++t)
                                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(cb[ti], wr * cb[tj], acc[t], 0, 0, 0);
                        wr = wn;
#pragma unroll
                        for (int bb = 0; bb < NB; ++bb) cb[bb] = cn[bb];
                    }
                }
                // H part to Hs (rows < n), J^T w (row n) to Fs
#pragma unroll
                for (int ti = 0, t = 0; ti < NB; ++ti)
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
                const float g2 = wave_total(Fj * Fj), an = wave_maximum(fabsf(aj));
                if (!(same && have_factor)) {
                    lower_row(h, [&](int c) { return Hs[min(l, NPA - 1) * LD + c] + Mrow[c]; });
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
                // (h strictly lower, diagonal in dl / idl: every lane applies
                // every column update, no selects; lane j's value is final
                // once column j is reached and is scaled by 1 / L_jj at the end)
                float y = -Fj;          // zero in lanes >= n
                with_nc([&](auto ncc) {
                    constexpr int NC = decltype(ncc)::value;
                    if constexpr (NC == 16) {
                        static_for<0, 16>([&](auto jc) {
                            constexpr int j = decltype(jc)::value;
                            y -= h[j] * row_bcast16<j>(y * idl);
                        });
                    } else {
#pragma unroll
                        for (int j = 0; j < NC; ++j) y -= h[j] * wave_lane(y * idl, j);
                    }
                    return 0;
                });
                y *= idl;
                // strictly lower rows of L to LDS for the transposed solve
                if (l < NPA) {
#pragma unroll
                    for (int c = 0; c < NPA; ++c) Hs[l * LD + c] = h[c];
                }
                __syncthreads();
                float pj = y;
                with_nc([&](auto ncc) {
                    constexpr int NC = decltype(ncc)::value;
                    const float *col = Hs + min(l, NPA - 1);    // L_jl at col[j * LD]
                    if constexpr (NC == 16) {
                        static_for<0, 16>([&](auto ic) {
                            constexpr int j = 15 - decltype(ic)::value;
                            pj -= col[j * LD] * row_bcast16<j>(pj * idl);
                        });
                    } else {
#pragma unroll
                        for (int j = NC - 1; j >= 0; --j) pj -= col[j * LD] * wave_lane(pj * idl, j);
                    }
                    return 0;
                });
                pj = (l < n) ? pj * idl : 0.f;
                // q = J p for the lane's rows; M p and the line-search coefficients
                float pv[NPA];
#pragma unroll
                for (int c = 0; c < NPA; ++c) pv[c] = wave_lane(pj, c);
                float qr[RPL];
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const int i = l + 64 * t;
                    const float *row = Js + min(i, m4 > 0 ? m4 - 1 : 0) * LD;
                    float s0 = 0.f, s1 = 0.f;
#pragma unroll
                    for (int c = 0; c < NPA; c += 2) {
                        s0 += row[c] * pv[c];
                        s1 += row[c + 1] * pv[c + 1];
                    }
                    qr[t] = (i < m) ? s0 + s1 : 0.f;
                }
                float Mp = 0.f;
#pragma unroll
                for (int c = 0; c < NPA; ++c) Mp += Mrow[c] * pv[c];
                const float c0 = wave_total(pj * Mp), b0 = wave_total(pj * Md);
                int fl;
                const float alpha = wave_line_search<RPL>(rr, qr, Dr, c0, b0, fl);
                lsfail |= fl;
                step_inf = wave_maximum(fabsf(alpha * pj));
                aj += alpha * pj;
                Md += alpha * Mp;
                __syncthreads();
            }
            if (lsfail) st |= ST_LSFAIL;
        }
        const bool ok = !(st & (ST_NONFINITE | ST_NOTSPD));
        const float nanv = __builtin_nanf("");
        if (l < n) gaout[I.on + l] = ok ? aj : nanv;
        // factor: lane i's row of L (strictly lower part, then the diagonal)
        // through LDS
        if (l < NPA) {
#pragma unroll
            for (int c = 0; c < NPA; ++c) Hs[l * LD + c] = h[c];
            Hs[l * LD + l] = dl;
        }
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
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int i = l + 64 * t;
            if (i < m) gmask[I.om + i] = (ok && ((act >> t) & 1u)) ? 1 : 0;
        }
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
    const int rpl = wave_rpl(mmax);
    int rc = -3;
#define CS_WAVE_CALL(NPAV, RPLV)                                                                 \
    if (npa == NPAV && rpl == RPLV) {                                                          \
        auto k = k_forward_wave<NPAV, RPLV>;                                                   \
        if (!ensure_lds(reinterpret_cast<const void *>(k), lds)) return -3;                    \
        hipLaunchKernelGGL(k, dim3(grid), dim3(64), lds, stream, bv, count, max_iter, tol, mmax, M, \
                           J, a0, aref, D, a_init, a_out, fac, mask, status, iters);           \
        rc = 0;                                                                                \
    }
    CS_WAVE_CALL(16, 1) CS_WAVE_CALL(16, 2) CS_WAVE_CALL(16, 4) CS_WAVE_CALL(16, 8) CS_WAVE_CALL(16, 16)
    CS_WAVE_CALL(32, 1) CS_WAVE_CALL(32, 2) CS_WAVE_CALL(32, 4) CS_WAVE_CALL(32, 8) CS_WAVE_CALL(32, 16)
#undef CS_WAVE_CALL
    if (rc != 0) return -3;
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cs
