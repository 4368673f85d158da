// cs_serve.hip -- device steps of the MPC-window serving loop (include/cs_serve.h).
//
// One 256-lane workgroup per entry: every entry touches one slot only (a few
// thousand values at most), so a launch is latency-bound; four waves per slot
// cut the serial depth of each copy, and no barrier spans entries.  Copies
// issue a batch of loads before any of its stores (the slot and pool arrays
// reach the kernel through a struct, so the compiler cannot tell them apart
// and would otherwise wait for each load before the next), and all accesses
// walk the slot's live sizes lane-strided and coalesced.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cs.h"
#include "cs_serve.h"

namespace {

constexpr int NT = 256;  // lanes per entry
constexpr int CU = 4;    // loads in flight per lane in a copy

struct Geo {
    int S, W, nc, mc;
    int64_t ne;          // factor capacity per slot
};

__device__ inline Geo geo(const cs_serve_table &t) {
    return Geo{t.slots, t.window, t.n_cap, t.m_cap, (int64_t)t.n_cap * (t.n_cap + 1) / 2};
}

template <typename T> __device__ inline T *P(void *p) { return static_cast<T *>(p); }

// d[i] = s[i] for i < cnt by the workgroup's lanes: CU loads (indices clamped
// into the span) before the CU stores of each batch.
template <typename T>
__device__ inline void copy_span(T *__restrict__ d, const T *__restrict__ s, int64_t cnt, int l) {
    if (cnt <= 0) return;
    for (int64_t b = 0; b < cnt; b += (int64_t)NT * CU) {
        T x[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int64_t i = b + l + (int64_t)NT * u;
            x[u] = s[i < cnt ? i : cnt - 1];
        }
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int64_t i = b + l + (int64_t)NT * u;
            if (i < cnt) d[i] = x[u];
        }
    }
}

template <typename T> __device__ inline void fill_span(T *d, int64_t cnt, int l) {
    for (int64_t i = l; i < cnt; i += NT) d[i] = T(0);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_serve_admit(cs_serve_table t, cs_serve_table p,
                                                    const int32_t *__restrict__ pairs, int count) {
    const int e = blockIdx.x, l = threadIdx.x;
    if (e >= count) return;
    const Geo G = geo(t);
    const int s = pairs[2 * e], q = pairs[2 * e + 1];
    if (s < 0 || s >= G.S || q < 0 || q >= p.slots) return;
    const int n = p.nv[q], m = p.nrows[q];
    if (n < 1 || n > G.nc || m < 0 || m > G.mc) return;
    const int64_t nn = (int64_t)G.nc * G.nc, mn = (int64_t)G.mc * G.nc;
    copy_span(P<T>(t.M) + s * nn, P<T>(p.M) + q * nn, (int64_t)n * n, l);
    copy_span(P<T>(t.Minv) + s * nn, P<T>(p.Minv) + q * nn, (int64_t)n * n, l);
    copy_span(P<T>(t.J) + s * mn, P<T>(p.J) + q * mn, (int64_t)m * n, l);
    copy_span(P<T>(t.D) + (int64_t)s * G.mc, P<T>(p.D) + (int64_t)q * G.mc, m, l);
    copy_span(P<T>(t.pen) + (int64_t)s * G.mc, P<T>(p.pen) + (int64_t)q * G.mc, m, l);
    copy_span(P<T>(t.v) + (int64_t)s * G.nc, P<T>(p.v) + (int64_t)q * G.nc, G.nc, l);
    copy_span(P<T>(t.goal) + (int64_t)s * G.nc, P<T>(p.goal) + (int64_t)q * G.nc, G.nc, l);
    copy_span(P<T>(t.tau) + (int64_t)s * G.W * G.nc, P<T>(p.tau) + (int64_t)q * G.W * G.nc,
              (int64_t)G.W * G.nc, l);
    fill_span(P<T>(t.vbar) + (int64_t)s * G.nc, G.nc, l);
    fill_span(P<T>(t.taubar) + (int64_t)s * G.W * G.nc, (int64_t)G.W * G.nc, l);
    if (l == 0) {
        t.nv[s] = n;
        t.nrows[s] = m;
    }
}

// Entry decode shared by pre and post; false when the entry is out of range.
__device__ inline bool entry(const cs_serve_table &t, const Geo &G, const int32_t *ent, int e,
                             int &s, int &step, bool &fwd, int &n, int &m) {
    s = ent[2 * e];
    const int ph = ent[2 * e + 1];
    if (s < 0 || s >= G.S || ph < 0 || ph >= 2 * G.W) return false;
    fwd = ph < G.W;
    step = fwd ? ph : 2 * G.W - 1 - ph;
    n = t.nv[s];
    m = t.nrows[s];
    return n >= 1 && n <= G.nc && m >= 0 && m <= G.mc;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_serve_pre(cs_serve_table t, const int32_t *__restrict__ ent,
                                                  int count) {
    const int e = blockIdx.x, l = threadIdx.x;
    if (e >= count) return;
    const Geo G = geo(t);
    int s, st, n, m;
    bool fwd;
    if (!entry(t, G, ent, e, s, st, fwd, n, m)) return;
    const int64_t on = (int64_t)s * G.nc, om = (int64_t)s * G.mc;
    if (fwd) {
        // a0 = M^{-1} tau_t
        const T *Mi = P<T>(t.Minv) + (int64_t)s * G.nc * G.nc;
        const T *tau = P<T>(t.tau) + ((int64_t)s * G.W + st) * G.nc;
        for (int i = l; i < n; i += NT) {
            T acc = T(0);
            for (int j = 0; j < n; ++j) acc += Mi[i * n + j] * tau[j];
            P<T>(t.a0)[on + i] = acc;
        }
        // aref = -b J v - k pen
        const T *J = P<T>(t.J) + (int64_t)s * G.mc * G.nc;
        const T *v = P<T>(t.v) + on;
        const T b = T(t.b_damp), k = T(t.k_spring);
        for (int r = l; r < m; r += NT) {
            T acc = T(0);
#pragma unroll 6
            for (int j = 0; j < n; ++j) acc += J[(int64_t)r * n + j] * v[j];
            P<T>(t.aref)[om + r] = -b * acc - k * P<T>(t.pen)[om + r];
        }
    } else {
        const int64_t an = ((int64_t)st * G.S + s) * G.nc, am = ((int64_t)st * G.S + s) * G.mc;
        for (int i = l; i < n; i += NT) {
            P<T>(t.a)[on + i] = P<T>(t.arch_a)[an + i];
            P<T>(t.a0)[on + i] = P<T>(t.arch_a0)[an + i];
            P<T>(t.abar)[on + i] = T(t.h) * P<T>(t.vbar)[on + i];
        }
        copy_span(P<T>(t.aref) + om, P<T>(t.arch_aref) + am, m, l);
        copy_span(t.state + t.mask_offset + om, t.arch_mask + am, m, l);
        const int ne = n * (n + 1) / 2;
        const T *src = P<T>(t.arch_fac) + ((int64_t)st * G.S + s) * G.ne;
        T *dst = reinterpret_cast<T *>(t.state) + (int64_t)s * G.ne;
        copy_span(dst, src, ne, l);
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_serve_post(cs_serve_table t, const int32_t *__restrict__ ent,
                                                   int count) {
    __shared__ T part[NT];
    const int e = blockIdx.x, l = threadIdx.x;
    if (e >= count) return;
    const Geo G = geo(t);
    int s, st, n, m;
    bool fwd;
    if (!entry(t, G, ent, e, s, st, fwd, n, m)) return;
    const int64_t on = (int64_t)s * G.nc, om = (int64_t)s * G.mc;
    if (fwd) {
        const int64_t an = ((int64_t)st * G.S + s) * G.nc, am = ((int64_t)st * G.S + s) * G.mc;
        const T h = T(t.h);
        for (int i = l; i < n; i += NT) {
            const T a = P<T>(t.a)[on + i];
            P<T>(t.arch_a)[an + i] = a;
            P<T>(t.arch_a0)[an + i] = P<T>(t.a0)[on + i];
            const T vn = P<T>(t.v)[on + i] + h * a;
            P<T>(t.v)[on + i] = vn;
            if (st == G.W - 1) P<T>(t.vbar)[on + i] = T(2) * (vn - P<T>(t.goal)[on + i]);
        }
        copy_span(P<T>(t.arch_aref) + am, P<T>(t.aref) + om, m, l);
        copy_span(t.arch_mask + am, t.state + t.mask_offset + om, m, l);
        const int ne = n * (n + 1) / 2;
        copy_span(P<T>(t.arch_fac) + ((int64_t)st * G.S + s) * G.ne,
                  reinterpret_cast<const T *>(t.state) + (int64_t)s * G.ne, ne, l);
    } else {
        // taubar_t = M^{-T} a0bar
        const T *Mi = P<T>(t.Minv) + (int64_t)s * G.nc * G.nc;
        const T *a0b = P<T>(t.a0bar) + on;
        for (int i = l; i < n; i += NT) {
            T acc = T(0);
            for (int j = 0; j < n; ++j) acc += Mi[j * n + i] * a0b[j];
            P<T>(t.taubar)[((int64_t)s * G.W + st) * G.nc + i] = acc;
        }
        // vbar -= b J^T arefbar: lane (column c, part p) sums rows p, p + np, ...
        const T *J = P<T>(t.J) + (int64_t)s * G.mc * G.nc;
        const T *rb = P<T>(t.arefbar) + om;
        const int np = NT / n;          // n <= n_cap <= 64
        const int c = l % n, pp = l / n;
        T acc = T(0);
        if (pp < np) {
#pragma unroll 4
            for (int r = pp; r < m; r += np) acc += J[(int64_t)r * n + c] * rb[r];
        }
        part[l] = acc;
        __syncthreads();
        if (l < n) {
            T sum = T(0);
            for (int q = 0; q < np; ++q) sum += part[q * n + l];
            P<T>(t.vbar)[on + l] -= T(t.b_damp) * sum;
        }
    }
}

int check_table(const cs_serve_table *t, bool slots_table) {
    if (!t) return CS_EINVAL;
    if (t->dtype != CS_F32 && t->dtype != CS_F64) return CS_EINVAL;
    if (t->slots < 1 || t->window < 1 || t->n_cap < 1 || t->n_cap > 64 || t->m_cap < 0 ||
        t->m_cap > CS_NROWS_MAX)
        return CS_EINVAL;
    if (!t->M || !t->Minv || !t->v || !t->goal || !t->tau || !t->nv || !t->nrows) return CS_EINVAL;
    if (t->m_cap > 0 && (!t->J || !t->D || !t->pen)) return CS_EINVAL;
    if (slots_table) {
        if (!t->vbar || !t->taubar || !t->a0 || !t->abar || !t->a || !t->a0bar || !t->state ||
            !t->arch_a || !t->arch_a0 || !t->arch_fac)
            return CS_EINVAL;
        if (t->m_cap > 0 && (!t->aref || !t->arefbar || !t->arch_aref || !t->arch_mask))
            return CS_EINVAL;
    }
    return CS_OK;
}

template <typename K>
int launch(K kernel, int count, hipStream_t st, const cs_serve_table &a, const int32_t *list) {
    hipLaunchKernelGGL(kernel, dim3(count), dim3(NT), 0, st, a, list, count);
    return hipGetLastError() == hipSuccess ? CS_OK : CS_EHIP;
}

}  // namespace

extern "C" {

int cs_serve_admit(const cs_serve_table *table, const cs_serve_table *pool, const int32_t *pairs,
                   int32_t count, void *stream) {
    int rc = check_table(table, true);
    if (rc == CS_OK) rc = check_table(pool, false);
    if (rc != CS_OK) return rc;
    if (pool->dtype != table->dtype || pool->n_cap != table->n_cap ||
        pool->m_cap != table->m_cap || pool->window != table->window)
        return CS_EINVAL;
    if (count < 0 || (count > 0 && !pairs)) return CS_EINVAL;
    if (count == 0) return CS_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (table->dtype == CS_F32)
        hipLaunchKernelGGL(k_serve_admit<float>, dim3(count), dim3(NT), 0, st, *table, *pool, pairs,
                           count);
    else
        hipLaunchKernelGGL(k_serve_admit<double>, dim3(count), dim3(NT), 0, st, *table, *pool, pairs,
                           count);
    return hipGetLastError() == hipSuccess ? CS_OK : CS_EHIP;
}

int cs_serve_pre(const cs_serve_table *table, const int32_t *entries, int32_t count, void *stream) {
    const int rc = check_table(table, true);
    if (rc != CS_OK) return rc;
    if (count < 0 || (count > 0 && !entries)) return CS_EINVAL;
    if (count == 0) return CS_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    return table->dtype == CS_F32 ? launch(k_serve_pre<float>, count, st, *table, entries)
                                  : launch(k_serve_pre<double>, count, st, *table, entries);
}

int cs_serve_post(const cs_serve_table *table, const int32_t *entries, int32_t count, void *stream) {
    const int rc = check_table(table, true);
    if (rc != CS_OK) return rc;
    if (count < 0 || (count > 0 && !entries)) return CS_EINVAL;
    if (count == 0) return CS_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    return table->dtype == CS_F32 ? launch(k_serve_post<float>, count, st, *table, entries)
                                  : launch(k_serve_post<double>, count, st, *table, entries);
}

int cs_serve_tick(const cs_serve_table *table, const cs_serve_table *pool,
                  const cs_batch *classes, int32_t nclasses, const cs_solver_params *params,
                  size_t state_bytes, int32_t *status, int32_t *iters,
                  const int32_t *host_list, int32_t *dev_list, int32_t list_len,
                  int32_t n_admit, int32_t n_entries,
                  const cs_serve_launch *launches, int32_t nlaunch,
                  void *stream, void *side, void *ev_list, void *ev_fork, void *ev_join) {
    int rc = check_table(table, true);
    if (rc != CS_OK) return rc;
    if (!classes || nclasses < 1 || !params || list_len < 0 || n_admit < 0 || n_entries < 0 ||
        nlaunch < 0 || (nlaunch > 0 && !launches) || (list_len > 0 && (!host_list || !dev_list)))
        return CS_EINVAL;
    if (2 * (int64_t)n_admit + 2 * (int64_t)n_entries > list_len) return CS_EINVAL;
    if (n_admit > 0 && !pool) return CS_EINVAL;
    bool use_side = false;
    for (int i = 0; i < nlaunch; ++i) {
        const cs_serve_launch &L = launches[i];
        if (L.kind < 0 || L.kind > 1 || L.cls < 0 || L.cls >= nclasses || L.lane < 0 ||
            L.lane > 1 || L.count < 1 || L.order < 0 || (int64_t)L.order + L.count > list_len)
            return CS_EINVAL;
        use_side = use_side || L.lane == 1;
    }
    if (use_side && (!side || !ev_fork || !ev_join)) return CS_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream), sd = static_cast<hipStream_t>(side);
    if (list_len > 0 && hipMemcpyAsync(dev_list, host_list, sizeof(int32_t) * (size_t)list_len,
                                       hipMemcpyHostToDevice, st) != hipSuccess)
        return CS_EHIP;
    if (ev_list && hipEventRecord(static_cast<hipEvent_t>(ev_list), st) != hipSuccess) return CS_EHIP;
    if (n_admit > 0 && (rc = cs_serve_admit(table, pool, dev_list, n_admit, stream)) != CS_OK)
        return rc;
    const int32_t *ent = dev_list + 2 * (int64_t)n_admit;
    if ((rc = cs_serve_pre(table, ent, n_entries, stream)) != CS_OK) return rc;
    if (use_side && (hipEventRecord(static_cast<hipEvent_t>(ev_fork), st) != hipSuccess ||
                     hipStreamWaitEvent(sd, static_cast<hipEvent_t>(ev_fork), 0) != hipSuccess))
        return CS_EHIP;
    for (int i = 0; i < nlaunch && rc == CS_OK; ++i) {
        const cs_serve_launch &L = launches[i];
        cs_batch d = classes[L.cls];
        d.order = dev_list + L.order;
        d.count = L.count;
        void *ls = L.lane == 1 ? side : stream;
        if (L.kind == 0)
            rc = cs_forward(&d, params, table->M, table->J, table->a0, table->aref, table->D, nullptr,
                            table->a, table->state, state_bytes, status, iters, ls);
        else
            rc = cs_ift_vjp(&d, table->state, state_bytes, table->M, table->J, table->a0,
                            table->aref, table->D, table->a, table->abar, table->a0bar,
                            table->arefbar, nullptr, nullptr, nullptr, ls);
    }
    // the join is enqueued even after a failed launch, so the caller's stream
    // stays ordered after everything the side stream was given
    if (use_side && (hipEventRecord(static_cast<hipEvent_t>(ev_join), sd) != hipSuccess ||
                     hipStreamWaitEvent(st, static_cast<hipEvent_t>(ev_join), 0) != hipSuccess))
        return rc != CS_OK ? rc : CS_EHIP;
    if (rc != CS_OK) return rc;
    return cs_serve_post(table, ent, n_entries, stream);
}

}  // extern "C"
