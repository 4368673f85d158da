// cs_api.hip -- extern "C" entry points of libcs.so (see include/cs.h).
//
// Host side only: argument validation, buffer-size queries, the choice of
// kernel family for the batch's shapes, and launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "cs.h"
#include "cs_chunk.hpp"
#include "cs_generic.hpp"
#include "cs_jvp.hpp"
#include "cs_rollout.hpp"
#include "cs_ell.hpp"
#include "cs_rows.hpp"
#include "cs_small.hpp"
#include "cs_vjp_team.hpp"
#include "cs_wave.hpp"

// The tape of cs_unrolled_vjp_static: one array per GPU, for the life of the
// process.  Host code never uses this name as an address (it is a host-side
// stand-in); static_tape_ptr() gives the device address on the current GPU.
static __device__ __align__(256) unsigned char scratch[CS_STATIC_TAPE_BYTES];

namespace {

constexpr int kAbiVersion = 1;
constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current GPU, looked up once per device
// (with that device current) and kept.
int static_tape_ptr(void **out) {
    static std::mutex mu;
    static void *ptr[kMaxDevices];
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return CS_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return CS_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CS_EHIP;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return CS_OK;
}
constexpr int kMaxIterCap = 100000;
constexpr size_t kLdsLimit = 160 * 1024;

struct HostBatch {
    int B, dtype, nmax, mmax, path;
    bool packed;
    int64_t tot_nn, tot_mn, tot_n, tot_m;
    cs::BatchView bv;
    size_t s;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int describe(const cs_batch *b, HostBatch &hb) {
    if (!b) return CS_EINVAL;
    if (b->B < 0) return CS_EINVAL;
    if (b->dtype != CS_F32 && b->dtype != CS_F64) return CS_EINVAL;
    if (b->path < CS_PATH_AUTO || b->path > CS_PATH_WAVE) return CS_EINVAL;
    if (b->count < 0 || b->count > b->B) return CS_EINVAL;
    if (b->count > 0 && b->count != b->B && !b->order) return CS_EINVAL;
    hb.path = b->path;
    hb.B = b->B;
    hb.dtype = b->dtype;
    hb.s = b->dtype == CS_F32 ? sizeof(float) : sizeof(double);
    hb.packed = b->nv != nullptr || b->nrows != nullptr || b->off_nn != nullptr ||
                b->off_mn != nullptr || b->off_n != nullptr || b->off_m != nullptr;
    if (hb.packed) {
        if (!b->nv || !b->nrows || !b->off_nn || !b->off_mn || !b->off_n || !b->off_m)
            return CS_EINVAL;
        if (b->nv_max < 1 || b->nv_max > CS_NV_MAX) return CS_EINVAL;
        if (b->nrows_max < 0 || b->nrows_max > CS_NROWS_MAX) return CS_EINVAL;
        if (b->total_nn < 0 || b->total_mn < 0 || b->total_n < 0 || b->total_m < 0)
            return CS_EINVAL;
        hb.nmax = b->nv_max;
        hb.mmax = b->nrows_max;
        hb.tot_nn = b->total_nn;
        hb.tot_mn = b->total_mn;
        hb.tot_n = b->total_n;
        hb.tot_m = b->total_m;
    } else {
        if (b->nv_uniform < 1 || b->nv_uniform > CS_NV_MAX) return CS_EINVAL;
        if (b->nrows_uniform < 0 || b->nrows_uniform > CS_NROWS_MAX) return CS_EINVAL;
        const int64_t B = b->B, n = b->nv_uniform, m = b->nrows_uniform;
        hb.nmax = (int)n;
        hb.mmax = (int)m;
        hb.tot_nn = B * n * n;
        hb.tot_mn = B * m * n;
        hb.tot_n = B * n;
        hb.tot_m = B * m;
    }
    // kernels loop over the instances they solve: order[0 .. count-1]
    hb.bv.B = b->count > 0 ? b->count : b->B;
    hb.bv.nv_u = b->nv_uniform;
    hb.bv.nr_u = b->nrows_uniform;
    hb.bv.nv = b->nv;
    hb.bv.nr = b->nrows;
    hb.bv.off_nn = b->off_nn;
    hb.bv.off_mn = b->off_mn;
    hb.bv.off_n = b->off_n;
    hb.bv.off_m = b->off_m;
    hb.bv.order = b->order;
    hb.bv.Bfull = b->B;
    hb.bv.nmax = hb.nmax;
    hb.bv.mmax = hb.mmax;
    hb.bv.tot_nn = hb.tot_nn;
    hb.bv.tot_mn = hb.tot_mn;
    hb.bv.tot_n = hb.tot_n;
    hb.bv.tot_m = hb.tot_m;
    return CS_OK;
}

// Packed lower triangles: sum_i n_i (n_i + 1) / 2 = (total_nn + total_n) / 2.
size_t factor_elems(const HostBatch &hb) { return (size_t)(hb.tot_nn + hb.tot_n) / 2; }

size_t state_bytes(const HostBatch &hb) {
    return align256(hb.s * factor_elems(hb)) + (size_t)hb.tot_m;
}

size_t tape_T_elems(const HostBatch &hb, int K) {
    return (size_t)K * (2 * (size_t)hb.tot_n + factor_elems(hb) + 2 * (size_t)hb.tot_m +
                        2 * (size_t)hb.B);
}

size_t tape_bytes(const HostBatch &hb, int K) {
    return align256(hb.s * tape_T_elems(hb, K)) + (size_t)K * 2 * (size_t)hb.tot_m;
}

int check_params(const cs_solver_params *p, bool unrolled = false) {
    if (!p) return CS_EINVAL;
    if (p->max_iter < 0 || p->max_iter > kMaxIterCap) return CS_EINVAL;
    if (unrolled ? (p->flags < 0 || p->flags > CS_UNROLLED_REPLAY)
                 : (p->flags != 0 && p->flags != CS_FORWARD_CG))
        return CS_EINVAL;
    if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) return CS_EINVAL;
    return CS_OK;
}

enum { FAM_TEAM = 0, FAM_SMALL = 1, FAM_CHUNK = 2, FAM_WAVE = 3 };

// Kernel family for this batch (FAM_*) or a negative error code.
int choose_family(const HostBatch &hb) {
    const bool small = cs::small_supported(hb.nmax, hb.mmax, (int)hb.s);
    const bool chunk = cs::chunk_supported(hb.nmax, hb.mmax, (int)hb.s);
    switch (hb.path) {
    case CS_PATH_SMALL: return small ? FAM_SMALL : CS_EUNSUPPORTED;
    case CS_PATH_CHUNK: return chunk ? FAM_CHUNK : CS_EUNSUPPORTED;
    case CS_PATH_WAVE:
        return cs::wave_supported(hb.nmax, hb.mmax, (int)hb.s) ? FAM_WAVE : CS_EUNSUPPORTED;
    case CS_PATH_TEAM: return FAM_TEAM;
    default:
        if (small) return FAM_SMALL;
        if (cs::wave_supported(hb.nmax, hb.mmax, (int)hb.s)) return FAM_WAVE;
        return chunk ? FAM_CHUNK : FAM_TEAM;
    }
}

// The VJP family for a batch whose forward ran on `fam`: the WAVE family
// has no VJP kernel of its own (the state layout is shared).
int vjp_family(const HostBatch &hb, int fam) {
    if (fam != FAM_WAVE) return fam;
    return cs::chunk_supported(hb.nmax, hb.mmax, (int)hb.s) ? FAM_CHUNK : FAM_TEAM;
}

int choose_family_unrolled(const HostBatch &hb) {
    const bool small = cs::small_unrolled_supported(hb.nmax, hb.mmax, (int)hb.s);
    switch (hb.path) {
    case CS_PATH_SMALL: return small ? FAM_SMALL : CS_EUNSUPPORTED;
    case CS_PATH_CHUNK:
    case CS_PATH_WAVE: return CS_EUNSUPPORTED;
    case CS_PATH_TEAM: return FAM_TEAM;
    default: return small ? FAM_SMALL : FAM_TEAM;
    }
}

// Generic family: team size by shape.
inline int generic_nt(const HostBatch &hb) {
    return (hb.nmax <= 32 && hb.mmax <= 32 * 64) ? 64 : 256;
}

template <typename K>
int prepare(K kernel, size_t lds) {
    if (lds > kLdsLimit) return CS_EUNSUPPORTED;
    return cs::ensure_lds(reinterpret_cast<const void *>(kernel), lds) ? CS_OK : CS_EHIP;
}

inline unsigned grid_for(int B) { return (unsigned)(B < (1 << 20) ? B : (1 << 20)); }

int launch_status() {
    return hipGetLastError() == hipSuccess ? CS_OK : CS_EHIP;
}

template <typename T>
int forward_launch(const HostBatch &hb, int fam, const cs_solver_params *p, const void *M,
                   const void *J, const void *a0, const void *aref, const void *D,
                   const void *a_init, void *a_out, T *fac, uint8_t *mask, int32_t *status,
                   int32_t *iters, hipStream_t stream);

template <typename T>
int forward_t(const HostBatch &hb, const cs_solver_params *p, const void *M, const void *J,
              const void *a0, const void *aref, const void *D, const void *a_init, void *a_out,
              void *state, int32_t *status, int32_t *iters, hipStream_t stream) {
    T *fac = static_cast<T *>(state);
    uint8_t *mask = static_cast<uint8_t *>(state) + align256(hb.s * factor_elems(hb));
    const int fam = choose_family(hb);
    if (fam < 0) return fam;
    if (p->flags == CS_FORWARD_CG) {
        // the conjugate-gradient forward exists in the SMALL family only
        if (fam != FAM_SMALL) return CS_EUNSUPPORTED;
        return cs::launch_small_forward_cg<T>(hb.bv, hb.nmax, hb.mmax, p->max_iter, (T)p->tol,
                                              (const T *)M, (const T *)J, (const T *)a0,
                                              (const T *)aref, (const T *)D, (const T *)a_init,
                                              (T *)a_out, fac, mask, status, iters, stream) == 0
                   ? CS_OK
                   : CS_EHIP;
    }
    const int rc = forward_launch<T>(hb, fam, p, M, J, a0, aref, D, a_init, a_out, fac, mask,
                                     status, iters, stream);
    if (rc != CS_OK) return rc;
    if constexpr (sizeof(T) == 4) {
        // FP32 team families: the final FP64-residual refinement of the
        // converged iterates (the SMALL family refines inside its kernel)
        if (fam != FAM_SMALL && cs::vjp_team_supported(hb.nmax, hb.mmax)) {
            const int rp = cs::launch_polish_team(hb.bv, hb.bv.B, hb.nmax, hb.mmax, status,
                                                  (float *)a_out, fac, mask, (const float *)M,
                                                  (const float *)J, (const float *)a0,
                                                  (const float *)aref, (const float *)D, stream);
            return rp == 0 ? CS_OK : CS_EHIP;
        }
    }
    return CS_OK;
}

template <typename T>
int forward_launch(const HostBatch &hb, int fam, const cs_solver_params *p, const void *M,
                   const void *J, const void *a0, const void *aref, const void *D,
                   const void *a_init, void *a_out, T *fac, uint8_t *mask, int32_t *status,
                   int32_t *iters, hipStream_t stream) {
    if constexpr (sizeof(T) == 4) {
        if (fam == FAM_WAVE) {
            const int rc = cs::launch_wave_forward(hb.bv, hb.bv.B, hb.nmax, hb.mmax, p->max_iter,
                                                   (float)p->tol, (const float *)M, (const float *)J,
                                                   (const float *)a0, (const float *)aref,
                                                   (const float *)D, (const float *)a_init,
                                                   (float *)a_out, fac, mask, status, iters, stream);
            return rc == 0 ? CS_OK : CS_EHIP;
        }
    }
    if (fam == FAM_CHUNK) {
        const int rc = cs::launch_chunk_forward<T>(hb.bv, hb.bv.B, hb.nmax, hb.mmax, p->max_iter,
                                                   (T)p->tol, (const T *)M, (const T *)J,
                                                   (const T *)a0, (const T *)aref, (const T *)D,
                                                   (const T *)a_init, (T *)a_out, fac, mask,
                                                   status, iters, stream);
        return rc == 0 ? CS_OK : CS_EHIP;
    }
    if (fam == FAM_SMALL) {
        return cs::launch_small_forward<T>(hb.bv, hb.nmax, hb.mmax, p->max_iter, (T)p->tol,
                                           (const T *)M, (const T *)J, (const T *)a0,
                                           (const T *)aref, (const T *)D, (const T *)a_init,
                                           (T *)a_out, fac, mask, status, iters, stream);
    }
    const int NT = generic_nt(hb);
    const size_t lds = cs::gen_lds_bytes(hb.nmax, hb.mmax, NT, hb.s);
    int rc;
    if (NT == 64) {
        auto k = cs::k_forward_generic<T, 64>;
        if ((rc = prepare(k, lds)) != CS_OK) return rc;
        hipLaunchKernelGGL(k, dim3(grid_for(hb.bv.B)), dim3(64), lds, stream, hb.bv, p->max_iter,
                           (T)p->tol, hb.nmax, hb.mmax, (const T *)M, (const T *)J,
                           (const T *)a0, (const T *)aref, (const T *)D, (const T *)a_init,
                           (T *)a_out, fac, mask, status, iters);
    } else {
        auto k = cs::k_forward_generic<T, 256>;
        if ((rc = prepare(k, lds)) != CS_OK) return rc;
        hipLaunchKernelGGL(k, dim3(grid_for(hb.bv.B)), dim3(256), lds, stream, hb.bv, p->max_iter,
                           (T)p->tol, hb.nmax, hb.mmax, (const T *)M, (const T *)J,
                           (const T *)a0, (const T *)aref, (const T *)D, (const T *)a_init,
                           (T *)a_out, fac, mask, status, iters);
    }
    return launch_status();
}

template <typename T>
int vjp_t(const HostBatch &hb, const void *state, const void *M, const void *J, const void *a0,
          const void *aref, const void *D, const void *a, const void *abar, void *a0bar,
          void *arefbar, void *Jbar, void *Dbar, void *Mbar, hipStream_t stream) {
    const T *fac = static_cast<const T *>(state);
    const uint8_t *mask =
        static_cast<const uint8_t *>(state) + align256(hb.s * factor_elems(hb));
    const int fam = vjp_family(hb, choose_family(hb));
    if (fam < 0) return fam;
    if constexpr (sizeof(T) == 4) {
        // FP32 team shapes: the FP64-arithmetic VJP
        if ((fam == FAM_CHUNK || fam == FAM_TEAM) && cs::vjp_team_supported(hb.nmax, hb.mmax)) {
            const int rc = cs::launch_vjp_team(hb.bv, hb.bv.B, hb.nmax, hb.mmax, fac, mask,
                                               (const float *)M, (const float *)J,
                                               (const float *)a0, (const float *)aref,
                                               (const float *)D, (const float *)a,
                                               (const float *)abar, (float *)a0bar,
                                               (float *)arefbar, (float *)Jbar, (float *)Dbar,
                                               (float *)Mbar, stream);
            return rc == 0 ? CS_OK : CS_EHIP;
        }
    }
    if (fam == FAM_CHUNK) {
        const int rc = cs::launch_chunk_vjp<T>(hb.bv, hb.bv.B, hb.nmax, hb.mmax, fac, mask,
                                               (const T *)M, (const T *)J, (const T *)a0,
                                               (const T *)aref, (const T *)D, (const T *)a,
                                               (const T *)abar, (T *)a0bar, (T *)arefbar,
                                               (T *)Jbar, (T *)Dbar, (T *)Mbar, stream);
        return rc == 0 ? CS_OK : CS_EHIP;
    }
    if (fam == FAM_SMALL) {
        return cs::launch_small_vjp<T>(hb.bv, hb.nmax, hb.mmax, fac, mask, (const T *)M,
                                       (const T *)J, (const T *)a0, (const T *)aref,
                                       (const T *)D, (const T *)a, (const T *)abar, (T *)a0bar,
                                       (T *)arefbar, (T *)Jbar, (T *)Dbar, (T *)Mbar, stream);
    }
    const int NT = generic_nt(hb);
    const size_t lds = cs::gen_lds_bytes(hb.nmax, hb.mmax, NT, hb.s);
    int rc;
    if (NT == 64) {
        auto k = cs::k_ift_vjp_generic<T, 64>;
        if ((rc = prepare(k, lds)) != CS_OK) return rc;
        hipLaunchKernelGGL(k, dim3(grid_for(hb.bv.B)), dim3(64), lds, stream, hb.bv, hb.nmax,
                           hb.mmax, fac, mask, (const T *)M, (const T *)J, (const T *)a0,
                           (const T *)aref, (const T *)D, (const T *)a, (const T *)abar,
                           (T *)a0bar, (T *)arefbar, (T *)Jbar, (T *)Dbar, (T *)Mbar);
    } else {
        auto k = cs::k_ift_vjp_generic<T, 256>;
        if ((rc = prepare(k, lds)) != CS_OK) return rc;
        hipLaunchKernelGGL(k, dim3(grid_for(hb.bv.B)), dim3(256), lds, stream, hb.bv, hb.nmax,
                           hb.mmax, fac, mask, (const T *)M, (const T *)J, (const T *)a0,
                           (const T *)aref, (const T *)D, (const T *)a, (const T *)abar,
                           (T *)a0bar, (T *)arefbar, (T *)Jbar, (T *)Dbar, (T *)Mbar);
    }
    return launch_status();
}

template <typename T>
int unrolled_t(const HostBatch &hb, const cs_solver_params *p, int mode, const void *M, const void *J,
               const void *a0, const void *aref, const void *D, const void *abar, void *a_out,
               void *a0bar, void *arefbar, void *Jbar, void *Dbar, void *Mbar, void *tape,
               int32_t *status, int32_t *iters, hipStream_t stream) {
    const int K = p->max_iter;
    T *tT = static_cast<T *>(tape);
    uint8_t *tB = static_cast<uint8_t *>(tape) + align256(hb.s * tape_T_elems(hb, K));
    const int fam = choose_family_unrolled(hb);
    if (fam < 0) return fam;
    if (fam == FAM_SMALL) {
        return cs::launch_small_unrolled<T>(hb.bv, hb.nmax, hb.mmax, K, mode, (T)p->tol, (const T *)M,
                                            (const T *)J, (const T *)a0, (const T *)aref,
                                            (const T *)D, (const T *)abar, (T *)a_out,
                                            (T *)a0bar, (T *)arefbar, (T *)Jbar, (T *)Dbar,
                                            (T *)Mbar, tT, tB, status, iters, stream);
    }
    const int NT = generic_nt(hb);
    const size_t lds = cs::gen_lds_bytes(hb.nmax, hb.mmax, NT, hb.s);
    int rc;
    if (NT == 64) {
        auto k = cs::k_unrolled_generic<T, 64>;
        if ((rc = prepare(k, lds)) != CS_OK) return rc;
        hipLaunchKernelGGL(k, dim3(grid_for(hb.bv.B)), dim3(64), lds, stream, hb.bv, K, mode,
                           (T)p->tol, hb.nmax, hb.mmax, (const T *)M, (const T *)J, (const T *)a0,
                           (const T *)aref, (const T *)D, (const T *)abar, (T *)a_out,
                           (T *)a0bar, (T *)arefbar, (T *)Jbar, (T *)Dbar, (T *)Mbar, tT, tB,
                           status, iters);
    } else {
        auto k = cs::k_unrolled_generic<T, 256>;
        if ((rc = prepare(k, lds)) != CS_OK) return rc;
        hipLaunchKernelGGL(k, dim3(grid_for(hb.bv.B)), dim3(256), lds, stream, hb.bv, K, mode,
                           (T)p->tol, hb.nmax, hb.mmax, (const T *)M, (const T *)J, (const T *)a0,
                           (const T *)aref, (const T *)D, (const T *)abar, (T *)a_out,
                           (T *)a0bar, (T *)arefbar, (T *)Jbar, (T *)Dbar, (T *)Mbar, tT, tB,
                           status, iters);
    }
    return launch_status();
}

int rollout_check(const HostBatch &hb, const cs_rollout_params *p) {
    if (!p) return CS_EINVAL;
    if (p->horizon < 1 || p->max_iter < 0 || p->max_iter > kMaxIterCap || p->reserved != 0)
        return CS_EINVAL;
    const int known = CS_ROLLOUT_FORWARD | CS_ROLLOUT_BACKWARD | CS_ROLLOUT_RECOMPUTE;
    if ((p->flags & ~known) || !(p->flags & (CS_ROLLOUT_FORWARD | CS_ROLLOUT_BACKWARD)))
        return CS_EINVAL;
    if (!(p->tol >= 0.0) || !std::isfinite(p->tol) || !std::isfinite(p->h) ||
        !std::isfinite(p->b_damp))
        return CS_EINVAL;
    (void)hb;
    return CS_OK;
}

size_t rollout_step_bytes(const HostBatch &hb, bool recompute, size_t *mask_off) {
    const size_t fac = recompute ? 0 : align256(hb.s * factor_elems(hb));
    if (mask_off) *mask_off = fac;
    return fac + align256((size_t)hb.tot_m);
}

template <typename T>
int rollout_t(const HostBatch &hb, const cs_rollout_params *p, const void *M, const void *J,
              const void *D, const void *c, const void *v0, const void *tau, const void *v_goal,
              const void *vbar_T, void *v_T, void *tau_bar, void *v0_bar, void *ws,
              int32_t *status, int32_t *iters, hipStream_t stream) {
    cs::RolloutArgs<T> g;
    g.M = (const T *)M;
    g.J = (const T *)J;
    g.D = (const T *)D;
    g.cref = (const T *)c;
    g.v0 = (const T *)v0;
    g.tau = (const T *)tau;
    g.vgoal = (const T *)v_goal;
    g.vbarT = (const T *)vbar_T;
    g.vT = (T *)v_T;
    g.taubar = (T *)tau_bar;
    g.v0bar = (T *)v0_bar;
    g.ws = (uint8_t *)ws;
    g.recompute = (p->flags & CS_ROLLOUT_RECOMPUTE) != 0;
    size_t moff = 0;
    g.ws_step = (int64_t)rollout_step_bytes(hb, g.recompute, &moff);
    g.mask_off = (int64_t)moff;
    g.status = status;
    g.iters = iters;
    g.tot_n = hb.tot_n;
    g.horizon = p->horizon;
    g.max_iter = p->max_iter;
    g.fwd = (p->flags & CS_ROLLOUT_FORWARD) != 0;
    g.bwd = (p->flags & CS_ROLLOUT_BACKWARD) != 0;
    g.tol = (T)p->tol;
    g.h = (T)p->h;
    g.bdamp = (T)p->b_damp;
    return cs::launch_rollout<T>(hb.bv, hb.bv.B, hb.nmax, hb.mmax, g, stream) == 0 ? CS_OK
                                                                                    : CS_EHIP;
}


}  // namespace

extern "C" {

int cs_version(void) { return kAbiVersion; }

const char *cs_strerror(int code) {
    switch (code) {
    case CS_OK: return "ok";
    case CS_EINVAL: return "invalid argument";
    case CS_ENOSPC: return "caller buffer too small";
    case CS_EHIP: return "HIP launch error";
    case CS_EUNSUPPORTED: return "unsupported shape";
    default: return "unknown error";
    }
}

size_t cs_state_bytes(const cs_batch *batch) {
    HostBatch hb;
    if (describe(batch, hb) != CS_OK) return 0;
    return state_bytes(hb);
}

size_t cs_unrolled_tape_bytes(const cs_batch *batch, int32_t K) {
    HostBatch hb;
    if (K < 0 || describe(batch, hb) != CS_OK) return 0;
    return tape_bytes(hb, K);
}

int cs_forward(const cs_batch *batch, const cs_solver_params *params, const void *M,
               const void *J, const void *a0, const void *aref, const void *D,
               const void *a_init, void *a_out, void *state, size_t state_bytes_given,
               int32_t *status, int32_t *iters, void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if ((rc = check_params(params)) != CS_OK) return rc;
    if (hb.B == 0) return CS_OK;
    if (!M || !a0 || !a_out || !state || !status) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !aref || !D)) return CS_EINVAL;
    if (state_bytes_given < state_bytes(hb)) return CS_ENOSPC;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hb.dtype == CS_F32)
        return forward_t<float>(hb, params, M, J, a0, aref, D, a_init, a_out, state, status,
                                iters, s);
    return forward_t<double>(hb, params, M, J, a0, aref, D, a_init, a_out, state, status, iters,
                             s);
}

int cs_ift_vjp(const cs_batch *batch, const void *state, size_t state_bytes_given, const void *M,
               const void *J, const void *a0, const void *aref, const void *D, const void *a,
               const void *abar, void *a0bar, void *arefbar, void *Jbar, void *Dbar, void *Mbar,
               void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if (hb.B == 0) return CS_OK;
    if (!state || !M || !a0 || !a || !abar) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !aref || !D)) return CS_EINVAL;
    if (state_bytes_given < state_bytes(hb)) return CS_ENOSPC;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hb.dtype == CS_F32)
        return vjp_t<float>(hb, state, M, J, a0, aref, D, a, abar, a0bar, arefbar, Jbar, Dbar,
                            Mbar, s);
    return vjp_t<double>(hb, state, M, J, a0, aref, D, a, abar, a0bar, arefbar, Jbar, Dbar, Mbar,
                         s);
}

int cs_ift_jvp(const cs_batch *batch, const void *state, size_t state_bytes_given, const void *M,
               const void *J, const void *D, int32_t k, const void *da0, const void *daref,
               void *da, void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if (k < 0) return CS_EINVAL;
    if (hb.B == 0 || k == 0) return CS_OK;
    if (!state || !M || !da) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !D)) return CS_EINVAL;
    if (state_bytes_given < state_bytes(hb)) return CS_ENOSPC;
    if (!cs::jvp_supported(hb.nmax, hb.mmax, (int)hb.s)) return CS_EUNSUPPORTED;
    const uint8_t *mask = static_cast<const uint8_t *>(state) + align256(hb.s * factor_elems(hb));
    hipStream_t s = static_cast<hipStream_t>(stream);
    int r;
    if (hb.dtype == CS_F32)
        r = cs::launch_ift_jvp<float>(hb.bv, hb.bv.B, hb.nmax, hb.mmax, k,
                                      static_cast<const float *>(state), mask,
                                      (const float *)M, (const float *)J, (const float *)D,
                                      (const float *)da0, (const float *)daref, (float *)da, s);
    else
        r = cs::launch_ift_jvp<double>(hb.bv, hb.bv.B, hb.nmax, hb.mmax, k,
                                       static_cast<const double *>(state), mask,
                                       (const double *)M, (const double *)J, (const double *)D,
                                       (const double *)da0, (const double *)daref, (double *)da, s);
    return r == 0 ? CS_OK : CS_EHIP;
}

int cs_forward_ell(const cs_batch *batch, const cs_solver_params *params, const void *M,
                   const void *J, const void *a0, const void *aref, const void *dn, const void *dt,
                   const void *mu, const void *a_init, void *a_out, void *state,
                   size_t state_bytes_given, int32_t *status, int32_t *iters, void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if ((rc = check_params(params)) != CS_OK) return rc;
    if (params->flags != 0) return CS_EINVAL;
    if (!hb.packed && batch->nrows_uniform % 3 != 0) return CS_EINVAL;
    if (hb.B == 0) return CS_OK;
    if (!M || !a0 || !a_out || !state || !status) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !aref || !dn || !dt || !mu)) return CS_EINVAL;
    if (state_bytes_given < state_bytes(hb)) return CS_ENOSPC;
    if (!cs::ell_supported(hb.nmax, hb.mmax, (int)hb.s)) return CS_EUNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *mask = static_cast<uint8_t *>(state) + align256(hb.s * factor_elems(hb));
    auto go = [&](auto tag) {
        typedef decltype(tag) T;
        cs::ElArgs<T> g = {};
        g.M = (const T *)M;
        g.J = (const T *)J;
        g.a0 = (const T *)a0;
        g.aref = (const T *)aref;
        g.dn = (const T *)dn;
        g.dt = (const T *)dt;
        g.mu = (const T *)mu;
        g.ainit = (const T *)a_init;
        g.aout = (T *)a_out;
        g.fac = (T *)state;
        g.mask = mask;
        g.status = status;
        g.iters = iters;
        g.max_iter = params->max_iter;
        g.tol = params->tol;
        return cs::launch_ell<T>(false, hb.bv, hb.bv.B, hb.nmax, hb.mmax, g, s);
    };
    const int r = hb.dtype == CS_F32 ? go(float()) : go(double());
    return r == 0 ? CS_OK : CS_EHIP;
}

int cs_ift_vjp_ell(const cs_batch *batch, const void *state, size_t state_bytes_given,
                   const void *M, const void *J, const void *a0, const void *aref, const void *dn,
                   const void *dt, const void *mu, const void *a, const void *abar, void *a0bar,
                   void *arefbar, void *Jbar, void *dnbar, void *dtbar, void *mubar, void *Mbar,
                   void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if (!hb.packed && batch->nrows_uniform % 3 != 0) return CS_EINVAL;
    if (hb.B == 0) return CS_OK;
    if (!state || !M || !a0 || !a || !abar) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !aref || !dn || !dt || !mu)) return CS_EINVAL;
    if (state_bytes_given < state_bytes(hb)) return CS_ENOSPC;
    if (!cs::ell_supported(hb.nmax, hb.mmax, (int)hb.s)) return CS_EUNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *mask = static_cast<uint8_t *>(const_cast<void *>(state)) +
                    align256(hb.s * factor_elems(hb));
    auto go = [&](auto tag) {
        typedef decltype(tag) T;
        cs::ElArgs<T> g = {};
        g.M = (const T *)M;
        g.J = (const T *)J;
        g.a0 = (const T *)a0;
        g.aref = (const T *)aref;
        g.dn = (const T *)dn;
        g.dt = (const T *)dt;
        g.mu = (const T *)mu;
        g.a = (const T *)a;
        g.abar = (const T *)abar;
        g.fac = (T *)const_cast<void *>(state);
        g.mask = mask;
        g.a0bar = (T *)a0bar;
        g.arefbar = (T *)arefbar;
        g.Jbar = (T *)Jbar;
        g.dnbar = (T *)dnbar;
        g.dtbar = (T *)dtbar;
        g.mubar = (T *)mubar;
        g.Mbar = (T *)Mbar;
        return cs::launch_ell<T>(true, hb.bv, hb.bv.B, hb.nmax, hb.mmax, g, s);
    };
    const int r = hb.dtype == CS_F32 ? go(float()) : go(double());
    return r == 0 ? CS_OK : CS_EHIP;
}

int cs_forward_rows(const cs_batch *batch, const cs_solver_params *params, const void *M,
                    const void *J, const void *a0, const void *aref, const void *D,
                    const uint8_t *kind, const void *floss, const void *a_init, void *a_out,
                    void *state, size_t state_bytes_given, int32_t *status, int32_t *iters,
                    void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if ((rc = check_params(params)) != CS_OK) return rc;
    if (params->flags != 0) return CS_EINVAL;
    if (hb.B == 0) return CS_OK;
    if (!M || !a0 || !a_out || !state || !status) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !aref || !D || !kind || !floss)) return CS_EINVAL;
    if (state_bytes_given < state_bytes(hb)) return CS_ENOSPC;
    if (!cs::rows_supported(hb.nmax, hb.mmax, (int)hb.s)) return CS_EUNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *mask = static_cast<uint8_t *>(state) + align256(hb.s * factor_elems(hb));
    auto go = [&](auto tag) {
        typedef decltype(tag) T;
        cs::RwArgs<T> g = {};
        g.M = (const T *)M;
        g.J = (const T *)J;
        g.a0 = (const T *)a0;
        g.aref = (const T *)aref;
        g.D = (const T *)D;
        g.fl = (const T *)floss;
        g.kind = kind;
        g.ainit = (const T *)a_init;
        g.aout = (T *)a_out;
        g.fac = (T *)state;
        g.mask = mask;
        g.status = status;
        g.iters = iters;
        g.max_iter = params->max_iter;
        g.tol = params->tol;
        return cs::launch_rows<T>(false, hb.bv, hb.bv.B, hb.nmax, hb.mmax, g, s);
    };
    const int r = hb.dtype == CS_F32 ? go(float()) : go(double());
    return r == 0 ? CS_OK : CS_EHIP;
}

int cs_ift_vjp_rows(const cs_batch *batch, const void *state, size_t state_bytes_given,
                    const void *M, const void *J, const void *a0, const void *aref, const void *D,
                    const uint8_t *kind, const void *floss, const void *a, const void *abar,
                    void *a0bar, void *arefbar, void *Jbar, void *Dbar, void *flossbar, void *Mbar,
                    void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if (hb.B == 0) return CS_OK;
    if (!state || !M || !a0 || !a || !abar) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !aref || !D || !kind || !floss)) return CS_EINVAL;
    if (state_bytes_given < state_bytes(hb)) return CS_ENOSPC;
    if (!cs::rows_supported(hb.nmax, hb.mmax, (int)hb.s)) return CS_EUNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *mask = static_cast<uint8_t *>(const_cast<void *>(state)) +
                    align256(hb.s * factor_elems(hb));
    auto go = [&](auto tag) {
        typedef decltype(tag) T;
        cs::RwArgs<T> g = {};
        g.M = (const T *)M;
        g.J = (const T *)J;
        g.a0 = (const T *)a0;
        g.aref = (const T *)aref;
        g.D = (const T *)D;
        g.fl = (const T *)floss;
        g.kind = kind;
        g.a = (const T *)a;
        g.abar = (const T *)abar;
        g.fac = (T *)const_cast<void *>(state);
        g.mask = mask;
        g.a0bar = (T *)a0bar;
        g.arefbar = (T *)arefbar;
        g.Jbar = (T *)Jbar;
        g.Dbar = (T *)Dbar;
        g.flbar = (T *)flossbar;
        g.Mbar = (T *)Mbar;
        return cs::launch_rows<T>(true, hb.bv, hb.bv.B, hb.nmax, hb.mmax, g, s);
    };
    const int r = hb.dtype == CS_F32 ? go(float()) : go(double());
    return r == 0 ? CS_OK : CS_EHIP;
}

size_t cs_rollout_workspace_bytes(const cs_batch *batch, const cs_rollout_params *params) {
    HostBatch hb;
    if (describe(batch, hb) != CS_OK || rollout_check(hb, params) != CS_OK) return 0;
    return (size_t)params->horizon *
           rollout_step_bytes(hb, (params->flags & CS_ROLLOUT_RECOMPUTE) != 0, nullptr);
}

int cs_rollout(const cs_batch *batch, const cs_rollout_params *params, const void *M,
               const void *J, const void *D, const void *c, const void *v0, const void *tau,
               const void *v_goal, const void *vbar_T, void *v_T, void *tau_bar, void *v0_bar,
               void *workspace, size_t workspace_bytes, int32_t *status, int32_t *iters,
               void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if ((rc = rollout_check(hb, params)) != CS_OK) return rc;
    if (hb.B == 0) return CS_OK;
    const bool fwd = params->flags & CS_ROLLOUT_FORWARD, bwd = params->flags & CS_ROLLOUT_BACKWARD;
    if (!M || !status || !workspace) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !D)) return CS_EINVAL;
    if (fwd && (!v0 || !tau || !v_T)) return CS_EINVAL;
    if (bwd && (!tau_bar || !v0_bar)) return CS_EINVAL;
    if (bwd && !vbar_T && !(fwd && v_goal)) return CS_EINVAL;
    if (workspace_bytes < cs_rollout_workspace_bytes(batch, params)) return CS_ENOSPC;
    if (!cs::rollout_supported(hb.nmax, hb.mmax, (int)hb.s)) return CS_EUNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hb.dtype == CS_F32)
        return rollout_t<float>(hb, params, M, J, D, c, v0, tau, v_goal, vbar_T, v_T, tau_bar,
                                v0_bar, workspace, status, iters, s);
    return rollout_t<double>(hb, params, M, J, D, c, v0, tau, v_goal, vbar_T, v_T, tau_bar, v0_bar,
                             workspace, status, iters, s);
}

int cs_unrolled_vjp(const cs_batch *batch, const cs_solver_params *params, const void *M,
                    const void *J, const void *a0, const void *aref, const void *D,
                    const void *abar, void *a_out, void *a0bar, void *arefbar, void *Jbar,
                    void *Dbar, void *Mbar, void *tape, size_t tape_bytes_given,
                    int32_t *status, int32_t *iters, void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if ((rc = check_params(params, true)) != CS_OK) return rc;
    if (hb.B == 0) return CS_OK;
    const int mode = params->flags;
    if (!M || !a0 || !status) return CS_EINVAL;
    if (hb.tot_m > 0 && (!J || !aref || !D)) return CS_EINVAL;
    if (mode != CS_UNROLLED_REPLAY && !a_out) return CS_EINVAL;
    if (mode == CS_UNROLLED_RECORD && !iters) return CS_EINVAL;
    if (mode == CS_UNROLLED_REPLAY && !iters) return CS_EINVAL;
    if (mode != CS_UNROLLED_RECORD) {
        if (!abar || !a0bar || !Mbar) return CS_EINVAL;
        if (hb.tot_m > 0 && (!arefbar || !Jbar || !Dbar)) return CS_EINVAL;
    }
    if (params->max_iter > 0 && !tape) return CS_EINVAL;
    if (tape_bytes_given < tape_bytes(hb, params->max_iter)) return CS_ENOSPC;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hb.dtype == CS_F32)
        return unrolled_t<float>(hb, params, mode, M, J, a0, aref, D, abar, a_out, a0bar, arefbar,
                                 Jbar, Dbar, Mbar, tape, status, iters, s);
    return unrolled_t<double>(hb, params, mode, M, J, a0, aref, D, abar, a_out, a0bar, arefbar, Jbar,
                              Dbar, Mbar, tape, status, iters, s);
}

int cs_unrolled_vjp_static(const cs_batch *batch, const cs_solver_params *params, const void *M,
                           const void *J, const void *a0, const void *aref, const void *D,
                           const void *abar, void *a_out, void *a0bar, void *arefbar, void *Jbar,
                           void *Dbar, void *Mbar, int32_t *status, int32_t *iters, void *stream) {
    HostBatch hb;
    int rc = describe(batch, hb);
    if (rc != CS_OK) return rc;
    if ((rc = check_params(params, true)) != CS_OK) return rc;
    if (params->flags != 0) return CS_EINVAL;
    if (tape_bytes(hb, params->max_iter) > CS_STATIC_TAPE_BYTES) return CS_ENOSPC;
    void *tape = nullptr;
    if ((rc = static_tape_ptr(&tape)) != CS_OK) return rc;
    return cs_unrolled_vjp(batch, params, M, J, a0, aref, D, abar, a_out, a0bar, arefbar, Jbar,
                           Dbar, Mbar, tape, CS_STATIC_TAPE_BYTES, status, iters, stream);
}

}  // extern "C"
