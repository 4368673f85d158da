// cs_vjp_team.hpp -- FP64-arithmetic team kernels for FP32 batches (one
// workgroup per instance): the IFT VJP (Sec. III-C, eq. 17) and the final
// refinement of the forward solve.
//
// Storage stays FP32 (inputs, the saved factor, outputs); every sum is taken
// in FP64 (the FP64 rate equals the unpacked FP32 rate on this chip and the
// kernel waits on memory, not on arithmetic):
//   lambda = H^{-1} abar: one solve with the saved FP32 factor, then two steps
//   of iterative refinement whose residual abar - H lambda (H v = M v +
//   J^T (D o A* o J v), eq. 9 at A*) is formed in FP64 from the stored inputs;
//   sigma = J lambda and r* = J a* - aref in FP64, then the cotangents of
//   eq. 17, each rounded once to FP32.
// So lambda carries the accuracy of the inputs rather than the factor's
// condition-number-sized rounding, and r* carries no cancellation of its own.
//
// The refinement (launched after the FP32 forward of the team families, for
// instances that met the stopping rule) takes one Newton step on the
// converged active set A*, with the gradient F(a*) = M (a* - a0) +
// J^T (D o A* o (J a* - aref)) (eq. 6) formed in FP64 and the step solved with
// the saved factor of H(A*): a* <- a* - H^{-1} F(a*).  In exact arithmetic the
// step is zero (a* is the root of F on A*); in FP32 it removes the iterate's
// rounding error, which the gradients of eq. 17 would otherwise inherit.
//
// Only the active rows of J are read (every row term of eq. 6 and eq. 17
// carries A*):
// they are listed in row order, gathered into LDS in chunks of `cr` rows and,
// when one chunk holds them all, kept there for every pass.
#pragma once

#include "cs_device.hpp"

namespace cs {

// Byte offsets of the LDS arrays (the host sizes the launch with the same
// function).
struct VtLayout {
    int npa, ld, cr, parts;
    uint32_t lam, a, a0, ab, part, tw, sw;   // FP64 arrays
    uint32_t H, diag, b, x, Jc;              // FP32 arrays
    uint32_t list, cnt, act;                 // int arrays, then bytes
    uint32_t bytes;
};

__host__ __device__ inline VtLayout vt_layout(int nmax, int mmax, int NT, int cr) {
    VtLayout L;
    L.npa = (nmax + 15) & ~15;
    L.ld = L.npa + 1;
    L.cr = cr;
    L.parts = NT / nmax < 1 ? 1 : (NT / nmax > 8 ? 8 : NT / nmax);
    uint32_t o = 0;
    auto take = [&o](uint64_t bytes) {
        const uint32_t r = o;
        o += (uint32_t)((bytes + 15) & ~uint64_t(15));
        return r;
    };
    L.lam = take(8ull * L.npa);
    L.a = take(8ull * L.npa);
    L.a0 = take(8ull * L.npa);
    L.ab = take(8ull * L.npa);
    L.part = take(8ull * L.parts * L.npa);
    L.tw = take(8ull * cr);
    L.sw = take(8ull * cr);
    L.H = take(4ull * L.npa * L.ld);
    L.diag = take(4ull * L.npa);
    L.b = take(4ull * L.npa);
    L.x = take(4ull * L.npa);
    L.Jc = take(4ull * cr * L.ld);
    L.list = take(4ull * (mmax > 0 ? mmax : 1));
    L.cnt = take(4ull * 16);
    L.act = take(mmax > 0 ? mmax : 1);
    L.bytes = o;
    return L;
}

template <int NT, bool POLISH>
__global__ __launch_bounds__(NT) void k_team_mixed(
    BatchView bv, int count, int nmax, int mmax, int cr, const int32_t *__restrict__ gstatus,
    float *__restrict__ gapol, const float *__restrict__ gfac,
    const uint8_t *__restrict__ gmask, const float *__restrict__ gM, const float *__restrict__ gJ,
    const float *__restrict__ ga0, const float *__restrict__ garef, const float *__restrict__ gD,
    const float *__restrict__ ga, const float *__restrict__ gabar, float *__restrict__ ga0bar,
    float *__restrict__ garefbar, float *__restrict__ gJbar, float *__restrict__ gDbar,
    float *__restrict__ gMbar) {
    constexpr int NW = NT / 64;
    constexpr int TPR = NT / 64;   // lanes per row in the row dots (64 rows per pass)
    extern __shared__ __align__(16) unsigned char smem[];
    const VtLayout Lo = vt_layout(nmax, mmax, NT, cr);
    double *lam = reinterpret_cast<double *>(smem + Lo.lam);
    double *av = reinterpret_cast<double *>(smem + Lo.a);
    double *a0v = reinterpret_cast<double *>(smem + Lo.a0);
    double *abv = reinterpret_cast<double *>(smem + Lo.ab);
    double *part = reinterpret_cast<double *>(smem + Lo.part);
    double *tw = reinterpret_cast<double *>(smem + Lo.tw);
    double *sw = reinterpret_cast<double *>(smem + Lo.sw);
    float *H = reinterpret_cast<float *>(smem + Lo.H);
    float *diag = reinterpret_cast<float *>(smem + Lo.diag);
    float *bb = reinterpret_cast<float *>(smem + Lo.b);
    float *xx = reinterpret_cast<float *>(smem + Lo.x);
    float *Jc = reinterpret_cast<float *>(smem + Lo.Jc);
    int *list = reinterpret_cast<int *>(smem + Lo.list);
    int *cnt = reinterpret_cast<int *>(smem + Lo.cnt);
    uint8_t *act = smem + Lo.act;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ld = Lo.ld, npa = Lo.npa, P = Lo.parts;

    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) continue;   // team-uniform: a malformed descriptor is skipped
        const int n = I.n, m = I.m;
        const float *M = gM + I.onn, *J = gJ + I.omn, *aref = garef + I.om, *D = gD + I.om;
        const uint8_t *mk = gmask + I.om;
        const float *fac = gfac + fac_offset(I);
        if constexpr (POLISH) {
            if ((gstatus[I.b] & ST_CONVERGED) == 0) continue;   // team-uniform
        }
        // the saved factor: packed lower triangle -> strictly lower rows + diagonal
        for (int e = tid; e < n * (n + 1) / 2; e += NT) {
            int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            while (j * (j + 1) / 2 > e) --j;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int l = e - j * (j + 1) / 2;
            const float v = fac[e];
            if (l < j) H[j * ld + l] = v;
            else diag[j] = v;
        }
        for (int j = tid; j < n; j += NT) {
            av[j] = (double)(POLISH ? gapol[I.on + j] : ga[I.on + j]);
            a0v[j] = (double)ga0[I.on + j];
            if constexpr (!POLISH) {
                const float abj = gabar[I.on + j];
                abv[j] = (double)abj;
                bb[j] = abj;
            }
        }
        // active rows listed in row order (fixed order: results are bitwise
        // reproducible); an inactive row's arefbar and Dbar are 0
        int total = 0;
        for (int base = 0; base < m; base += NT) {
            const int i = base + tid;
            const bool an = i < m && mk[i] != 0;
            if (i < m) {
                act[i] = an ? 1 : 0;
                if (!POLISH && !an) {
                    if (garefbar) garefbar[I.om + i] = 0.f;
                    if (gDbar) gDbar[I.om + i] = 0.f;
                }
            }
            const uint64_t bal = __builtin_amdgcn_ballot_w64(an);
            if (lane == 0) cnt[wv] = (int)__builtin_popcountll(bal);
            __syncthreads();
            int off = total, tot = total;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const int c = cnt[q];
                off += q < wv ? c : 0;
                tot += c;
            }
            if (an)
                list[off + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] = i;
            total = tot;
            __syncthreads();
        }
        __syncthreads();
        if constexpr (!POLISH) {
            team_chol_solve<NT, float>(H, diag, bb, xx, n, ld);
            for (int j = tid; j < n; j += NT) lam[j] = (double)xx[j];
            __syncthreads();
        }

        const int nch = (total + cr - 1) / cr;
        const bool resident = nch <= 1;
        // chunk c of the list into Jc (row stride ld), every load issued
        // before the stores, addresses clamped
        auto gather = [&](int c) {
            const int s0 = c * cr, cc = min(cr, total - s0), tot = cc * n;
            const int ds = NT / n, dj = NT - (NT / n) * n;
            int s = tid / n, j = tid - (tid / n) * n;
            for (int e0 = tid; e0 < tot; e0 += 4 * NT) {
                float v[4];
                int ss[4], jj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    ss[u] = s;
                    jj[u] = j;
                    v[u] = J[(int64_t)list[s0 + min(s, cc - 1)] * n + j];
                    s += ds;
                    j += dj;
                    if (j >= n) { j -= n; ++s; }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (e0 + u * NT < tot) Jc[ss[u] * ld + jj[u]] = v[u];
            }
        };
        // row dots of the chunk's rows with u (and v): fn(s, J_s u, J_s v)
        auto rowdot = [&](int cc, const double *u, const double *v, auto &&fn) {
            const int pr = tid % TPR;
            const bool two = v != nullptr;
            for (int s0 = 0; s0 < cc; s0 += 64) {
                const int s = s0 + tid / TPR;
                const float *row = Jc + min(s, cc - 1) * ld;
                double x = 0.0, y = 0.0;
                for (int j = pr; j < n; j += TPR) {
                    const double jv = (double)row[j];
                    x += jv * u[j];
                    if (two) y += jv * v[j];
                }
#pragma unroll
                for (int o = 1; o < TPR; o <<= 1) {
                    x += __shfl_xor(x, o, 64);
                    if (two) y += __shfl_xor(y, o, 64);
                }
                if (s < cc && pr == 0) fn(s, x, y);
            }
        };
        const int cp = tid / n, cj = tid - (tid / n) * n;

        if constexpr (POLISH) {
            // F = M (a - a0) + J^T (D o A* o (J a - aref)) in FP64, then a -= H^{-1} F
            double acc = 0.0;
            for (int c = 0; c < nch; ++c) {
                const int cc = min(cr, total - c * cr);
                gather(c);
                __syncthreads();
                rowdot(cc, av, nullptr, [&](int s, double x, double) {
                    const int i = list[c * cr + s];
                    tw[s] = (double)D[i] * (x - (double)aref[i]);
                });
                __syncthreads();
                if (cp < P)
                    for (int s = cp; s < cc; s += P) acc += (double)Jc[s * ld + cj] * tw[s];
                __syncthreads();
            }
            if (cp < P) part[cp * npa + cj] = acc;
            __syncthreads();
            for (int j = tid; j < n; j += NT) {
                double f = 0.0;
                for (int l = 0; l < n; ++l) f += (double)M[(int64_t)l * n + j] * (av[l] - a0v[l]);
                for (int q = 0; q < P; ++q) f += part[q * npa + j];
                bb[j] = (float)(-f);
            }
            __syncthreads();
            team_chol_solve<NT, float>(H, diag, bb, xx, n, ld);
            for (int j = tid; j < n; j += NT) gapol[I.on + j] = (float)(av[j] + (double)xx[j]);
            __syncthreads();
            continue;
        }

        // two refinement steps: lambda += H^{-1} (abar - H lambda)
#pragma unroll 1
        for (int it = 0; it < 2; ++it) {
            double acc = 0.0;
            for (int c = 0; c < nch; ++c) {
                const int cc = min(cr, total - c * cr);
                if (!resident || it == 0) {
                    gather(c);
                    __syncthreads();
                }
                rowdot(cc, lam, nullptr, [&](int s, double x, double) {
                    tw[s] = (double)D[list[c * cr + s]] * x;
                });
                __syncthreads();
                if (cp < P)
                    for (int s = cp; s < cc; s += P) acc += (double)Jc[s * ld + cj] * tw[s];
                __syncthreads();
            }
            if (cp < P) part[cp * npa + cj] = acc;
            __syncthreads();
            for (int j = tid; j < n; j += NT) {
                double s = abv[j];
                for (int l = 0; l < n; ++l) s -= (double)M[(int64_t)l * n + j] * lam[l];
                for (int q = 0; q < P; ++q) s -= part[q * npa + j];
                bb[j] = (float)s;
            }
            __syncthreads();
            team_chol_solve<NT, float>(H, diag, bb, xx, n, ld);
            for (int j = tid; j < n; j += NT) lam[j] += (double)xx[j];
            __syncthreads();
        }

        // per-row cotangents and J-bar rows of the active rows
        for (int c = 0; c < nch; ++c) {
            const int cc = min(cr, total - c * cr);
            if (!resident) {
                gather(c);
                __syncthreads();
            }
            rowdot(cc, lam, av, [&](int s, double sig, double ja) {
                const int i = list[c * cr + s];
                const double r = ja - (double)aref[i], d = (double)D[i];
                const double arb = d * sig;
                if (garefbar) garefbar[I.om + i] = (float)arb;
                if (gDbar) gDbar[I.om + i] = (float)(-r * sig);
                tw[s] = d * r;
                sw[s] = arb;
            });
            __syncthreads();
            if (gJbar) {
                const int ds = NT / n, dj = NT - (NT / n) * n;
                int s = tid / n, j = tid - (tid / n) * n;
                for (int e = tid; e < cc * n; e += NT) {
                    const int i = list[c * cr + s];
                    gJbar[I.omn + (int64_t)i * n + j] = (float)(-(tw[s] * lam[j] + sw[s] * av[j]));
                    s += ds;
                    j += dj;
                    if (j >= n) { j -= n; ++s; }
                }
            }
            __syncthreads();
        }
        // J-bar rows of the inactive rows: -(0 lambda + 0 a), no read of J
        if (gJbar) {
            const int di = NT / n, dj = NT - (NT / n) * n;
            int i = tid / n, j = tid - (tid / n) * n;
            for (int e = tid; e < m * n; e += NT) {
                if (!act[i]) gJbar[I.omn + e] = -0.f;
                i += di;
                j += dj;
                if (j >= n) { j -= n; ++i; }
            }
        }
        if (ga0bar) {
            for (int j = tid; j < n; j += NT) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += (double)M[(int64_t)l * n + j] * lam[l];
                ga0bar[I.on + j] = (float)s;
            }
        }
        if (gMbar) {
            const int dr = NT / n, dc = NT - (NT / n) * n;
            int jr = tid / n, lc = tid - (tid / n) * n;
            for (int e = tid; e < n * n; e += NT) {
                gMbar[I.onn + e] = (float)(-lam[jr] * (av[lc] - a0v[lc]));
                jr += dr;
                lc += dc;
                if (lc >= n) { lc -= n; ++jr; }
            }
        }
        __syncthreads();
    }
}

// Host side --------------------------------------------------------------

inline int vt_nt(int nmax) { return nmax <= 32 ? 64 : 256; }

// Rows per chunk: the largest multiple of 64 (up to the batch's row count)
// that keeps the workgroup within 96 KiB of LDS.
inline int vt_cr(int nmax, int mmax) {
    const int NT = vt_nt(nmax);
    const int cap = ((mmax > 64 ? mmax : 64) + 63) & ~63;
    int cr = 64;
    while (cr * 2 <= cap && vt_layout(nmax, mmax, NT, cr * 2).bytes <= 96 * 1024) cr *= 2;
    return cr;
}

inline bool vjp_team_supported(int nmax, int mmax) {
    return nmax >= 1 && nmax <= 128 &&
           vt_layout(nmax, mmax, vt_nt(nmax), vt_cr(nmax, mmax)).bytes <= 160 * 1024;
}

inline int launch_vjp_team(const BatchView &bv, int count, int nmax, int mmax, const float *fac,
                           const uint8_t *mask, const float *M, const float *J, const float *a0,
                           const float *aref, const float *D, const float *a, const float *abar,
                           float *a0bar, float *arefbar, float *Jbar, float *Dbar, float *Mbar,
                           hipStream_t stream) {
    const int NT = vt_nt(nmax), cr = vt_cr(nmax, mmax);
    const size_t lds = vt_layout(nmax, mmax, NT, cr).bytes;
    const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
    auto go = [&](auto k) {
        if (!ensure_lds(reinterpret_cast<const void *>(k), lds)) return -3;
        hipLaunchKernelGGL(k, dim3(grid), dim3(NT), lds, stream, bv, count, nmax, mmax, cr,
                           (const int32_t *)nullptr, (float *)nullptr, fac, mask, M, J, a0, aref,
                           D, a, abar, a0bar, arefbar, Jbar, Dbar, Mbar);
        return hipGetLastError() == hipSuccess ? 0 : -3;
    };
    return NT == 64 ? go(k_team_mixed<64, false>) : go(k_team_mixed<256, false>);
}

// The forward's final refinement: a (in place) for every instance whose
// status has ST_CONVERGED, from the state the forward wrote.
inline int launch_polish_team(const BatchView &bv, int count, int nmax, int mmax,
                              const int32_t *status, float *a, const float *fac,
                              const uint8_t *mask, const float *M, const float *J,
                              const float *a0, const float *aref, const float *D,
                              hipStream_t stream) {
    const int NT = vt_nt(nmax), cr = vt_cr(nmax, mmax);
    const size_t lds = vt_layout(nmax, mmax, NT, cr).bytes;
    const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
    auto go = [&](auto k) {
        if (!ensure_lds(reinterpret_cast<const void *>(k), lds)) return -3;
        hipLaunchKernelGGL(k, dim3(grid), dim3(NT), lds, stream, bv, count, nmax, mmax, cr, status,
                           a, fac, mask, M, J, a0, aref, D, (const float *)nullptr,
                           (const float *)nullptr, (float *)nullptr, (float *)nullptr,
                           (float *)nullptr, (float *)nullptr, (float *)nullptr);
        return hipGetLastError() == hipSuccess ? 0 : -3;
    };
    return NT == 64 ? go(k_team_mixed<64, true>) : go(k_team_mixed<256, true>);
}

}  // namespace cs
