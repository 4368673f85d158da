// cs_jvp.hpp -- IFT Jacobian-vector products (Sec. III-C, eq. 15, forward
// mode) for k tangent directions of (a0, aref) per instance:
//   da_j = -F_a^{-1} F_theta (da0_j, daref_j) = H^{-1} (M da0_j + J^T (D o A* o daref_j)),
// with H = M + J^T diag(D o A*) J factored by the forward (the saved state).
// These are the columns iLQR needs for its linearised dynamics: a direction
// of the actuation enters through a0, a direction of the velocity through
// aref.
//
// One workgroup per instance (grid-stride over the batch), one thread per
// direction (threads loop over directions past 64): the factor, the row
// weights D o A* and the active-row list sit in LDS and every thread reads
// the same entries at the same time (broadcasts); each thread keeps its two
// working vectors in LDS, laid out [column][thread] so consecutive threads
// touch consecutive words.  Every sum is taken in FP64: the right-hand side is
// solved with the saved factor, then two steps of iterative refinement with
// the residual rhs - H x formed in FP64 from M, J and D (H x = M x +
// J^T (D o A* o J x)) bring x to the accuracy of the inputs.
#pragma once

#include "cs_device.hpp"

namespace cs {

constexpr int JVP_NT = 64;
constexpr int JVP_NMAX = 96;

struct JvpLayout {
    int npa;
    uint32_t fac, w, list, x, y, bytes;
};

__host__ __device__ inline JvpLayout jvp_layout(int nmax, int mmax, int s) {
    JvpLayout L;
    L.npa = (nmax + 15) & ~15;
    uint32_t o = 0;
    auto take = [&o](uint64_t bytes) {
        const uint32_t r = o;
        o += (uint32_t)((bytes + 15) & ~uint64_t(15));
        return r;
    };
    L.x = take(8ull * L.npa * JVP_NT);
    L.y = take(8ull * L.npa * JVP_NT);
    L.fac = take((uint64_t)s * L.npa * (L.npa + 1) / 2);
    L.w = take((uint64_t)s * (mmax > 0 ? mmax : 1));
    L.list = take(4ull * (mmax > 0 ? mmax : 1) + 16 * 4);
    L.bytes = o;
    return L;
}

template <typename T>
__global__ __launch_bounds__(JVP_NT) void k_ift_jvp(
    BatchView bv, int count, int nmax, int mmax, int k, const T *__restrict__ gfac,
    const uint8_t *__restrict__ gmask, const T *__restrict__ gM, const T *__restrict__ gJ,
    const T *__restrict__ gD, const T *__restrict__ gda0, const T *__restrict__ gdaref,
    T *__restrict__ gda) {
    typedef double C;
    extern __shared__ __align__(16) unsigned char smem[];
    const JvpLayout Lo = jvp_layout(nmax, mmax, (int)sizeof(T));
    C *xs = reinterpret_cast<C *>(smem + Lo.x);
    C *ys = reinterpret_cast<C *>(smem + Lo.y);
    T *fac = reinterpret_cast<T *>(smem + Lo.fac);
    T *wt = reinterpret_cast<T *>(smem + Lo.w);
    int *list = reinterpret_cast<int *>(smem + Lo.list);
    const int tid = threadIdx.x;
    constexpr int NT = JVP_NT;
    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const Inst I = inst_at(bv, w);
        if (!I.ok) continue;   // team-uniform: outputs untouched
        const int n = I.n, m = I.m;
        const T *M = gM + I.onn, *J = gJ + I.omn;
        const T *fp = gfac + fac_offset(I);
        for (int e = tid; e < n * (n + 1) / 2; e += NT) fac[e] = fp[e];
        // active rows (row order) and their weights D_i
        int total = 0;
        for (int base = 0; base < m; base += NT) {
            const int i = base + tid;
            const bool an = i < m && gmask[I.om + i] != 0;
            if (i < m) wt[i] = an ? gD[I.om + i] : T(0);
            const uint64_t bal = __builtin_amdgcn_ballot_w64(an);
            if (an)
                list[total + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] = i;
            total += (int)__builtin_popcountll(bal);
        }
        __syncthreads();
        // column c of the thread's vectors at c * NT + tid
        auto X = [&](int c) -> C & { return xs[c * NT + tid]; };
        auto Y = [&](int c) -> C & { return ys[c * NT + tid]; };
        auto Lf = [&](int j, int l) { return C(fac[j * (j + 1) / 2 + l]); };
        for (int d = tid; d < k; d += NT) {
            const T *d0 = gda0 ? gda0 + (int64_t)k * I.on + (int64_t)d * n : nullptr;
            const T *dr = gdaref ? gdaref + (int64_t)k * I.om + (int64_t)d * m : nullptr;
            // Y = rhs - (H X if `sub`): rhs = M da0 + J^T (D o A* o daref)
            auto residual = [&](bool sub) {
                for (int l = 0; l < n; ++l) {
                    C s = C(0);
                    if (d0)
                        for (int c = 0; c < n; ++c) s += C(M[(int64_t)l * n + c]) * C(d0[c]);
                    if (sub)
                        for (int c = 0; c < n; ++c) s -= C(M[(int64_t)l * n + c]) * X(c);
                    Y(l) = s;
                }
                for (int q = 0; q < total; ++q) {
                    const int i = __builtin_amdgcn_readfirstlane(list[q]);
                    const T *Ji = J + (int64_t)i * n;
                    C t = dr ? C(dr[i]) : C(0);
                    if (sub) {
                        C jx = C(0);
                        for (int c = 0; c < n; ++c) jx += C(Ji[c]) * X(c);
                        t -= jx;
                    }
                    t *= C(wt[i]);
                    for (int l = 0; l < n; ++l) Y(l) += C(Ji[l]) * t;
                }
            };
            // Y <- (L L^T)^{-1} Y in place
            auto solve = [&]() {
                for (int l = 0; l < n; ++l) {
                    C s = Y(l);
                    for (int c = 0; c < l; ++c) s -= Lf(l, c) * Y(c);
                    Y(l) = s / Lf(l, l);
                }
                for (int l = n - 1; l >= 0; --l) {
                    C s = Y(l);
                    for (int c = l + 1; c < n; ++c) s -= Lf(c, l) * Y(c);
                    Y(l) = s / Lf(l, l);
                }
            };
            residual(false);
            solve();
            for (int c = 0; c < n; ++c) X(c) = Y(c);
            for (int it = 0; it < 2; ++it) {
                residual(true);
                solve();
                for (int c = 0; c < n; ++c) X(c) += Y(c);
            }
            T *out = gda + (int64_t)k * I.on + (int64_t)d * n;
            for (int c = 0; c < n; ++c) out[c] = T(X(c));
        }
        __syncthreads();
    }
}

inline bool jvp_supported(int nmax, int mmax, int s) {
    return nmax >= 1 && nmax <= JVP_NMAX && jvp_layout(nmax, mmax, s).bytes <= 160 * 1024;
}

template <typename T>
int launch_ift_jvp(const BatchView &bv, int count, int nmax, int mmax, int k, const T *fac,
                   const uint8_t *mask, const T *M, const T *J, const T *D, const T *da0,
                   const T *daref, T *da, hipStream_t stream) {
    const size_t lds = jvp_layout(nmax, mmax, (int)sizeof(T)).bytes;
    auto kern = k_ift_jvp<T>;
    if (!ensure_lds(reinterpret_cast<const void *>(kern), lds)) return -3;
    const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(JVP_NT), lds, stream, bv, count, nmax, mmax, k, fac,
                       mask, M, J, D, da0, daref, da);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cs
