/*
 * cs_serve.h -- device-side steps of the MPC-window serving loop (libcs.so).
 *
 * A request is a short receding-horizon window of W steps of the
 * semi-implicit rollout used by the paper's trajectory optimisation and its
 * short-horizon residual MPC (Sec. IV-A and Sec. V): per step t
 *
 *   a0_t   = M^{-1} tau_t                      (unconstrained acceleration)
 *   aref_t = -b J v_t - k pen                  (spring-damper reference, per row)
 *   a_t    = contact solve (cs_forward)
 *   v_{t+1} = v_t + h a_t,
 *
 * followed, in reverse, by the IFT VJP of every step (cs_ift_vjp, Sec.
 * III-C, eq. 17) for the gradient of ||v_W - v_goal||^2 w.r.t. every tau_t:
 *
 *   abar_t = h vbar_{t+1},  taubar_t = M^{-T} a0bar_t,
 *   vbar_t = vbar_{t+1} - b J^T arefbar_t,  vbar_W = 2 (v_W - v_goal).
 *
 * The caller keeps a table of S request slots in device memory.  Every
 * per-slot array has a fixed capacity (n_cap velocities, m_cap rows) and slot
 * s starts at s times that capacity; within a slot, matrices hold the
 * instance's n x n (M, Minv) or m x n (J) block tightly packed, row-major, at
 * the front, and vectors their n (or m) live entries at the front.  The
 * solver work arrays (a0, aref, a, abar, a0bar, arefbar, state) are the
 * arrays of a packed cs_batch whose instance s has capacity offsets
 * (off_nn = s n_cap^2, off_mn = s m_cap n_cap, off_n = s n_cap,
 * off_m = s m_cap) and live sizes nv[s], nrows[s]; so cs_forward /
 * cs_ift_vjp run directly on any subset of slots.  The state holds the
 * factor of slot s at element s n_cap (n_cap + 1) / 2 and its active-set
 * bytes at byte mask_offset + s m_cap.
 *
 * A W-deep archive keeps, per step and slot, the solution, a0, aref, factor
 * and active set between the forward and the backward phase, so the backward
 * step never refactors.
 *
 * Entry lists are device int32 arrays of pairs.  Calls are asynchronous on
 * `stream`, allocate nothing, and check arguments only (CS_EINVAL); the
 * kernels skip an entry whose slot, pool index, phase or sizes are out of
 * range.  Entries of one call must name distinct slots.
 */
#ifndef CS_SERVE_H
#define CS_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "cs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cs_serve_table {
    int32_t dtype;        /* CS_F32 or CS_F64 */
    int32_t slots;        /* S (rows of every per-slot array) */
    int32_t window;       /* W steps per request */
    int32_t n_cap;        /* 1 .. 64 */
    int32_t m_cap;        /* 0 .. CS_NROWS_MAX */
    int32_t reserved;
    double h;             /* time step */
    double b_damp;        /* reference damping b */
    double k_spring;      /* reference stiffness k */
    /* request payload */
    void *M;              /* [S, n_cap^2]   */
    void *Minv;           /* [S, n_cap^2]   M^{-1} */
    void *J;              /* [S, m_cap n_cap] */
    void *D;              /* [S, m_cap]     */
    void *pen;            /* [S, m_cap]     penetration of each row's contact */
    void *v;              /* [S, n_cap]     current velocity (initial velocity in a pool) */
    void *goal;           /* [S, n_cap]     v_goal */
    void *tau;            /* [S, W, n_cap]  actuation per step */
    int32_t *nv;          /* [S] live n */
    int32_t *nrows;       /* [S] live m */
    /* request state (slot tables only) */
    void *vbar;           /* [S, n_cap] */
    void *taubar;         /* [S, W, n_cap]  the request's result */
    /* solver work arrays (slot tables only) */
    void *a0, *abar, *a, *a0bar;      /* [S, n_cap] */
    void *aref, *arefbar;             /* [S, m_cap] */
    uint8_t *state;                   /* cs_forward state of the slot batch */
    uint64_t mask_offset;             /* byte offset of the active-set bytes in state */
    /* per-step archive (slot tables only) */
    void *arch_a, *arch_a0;           /* [W, S, n_cap] */
    void *arch_aref;                  /* [W, S, m_cap] */
    void *arch_fac;                   /* [W, S, n_cap (n_cap + 1) / 2] */
    uint8_t *arch_mask;               /* [W, S, m_cap] */
} cs_serve_table;

/* Copy request payloads into slots: pairs[2e] = slot, pairs[2e+1] = index
 * into `pool` (a table with only the payload fields set and `slots` = pool
 * size).  Sets nv/nrows, the payload and clears vbar and taubar of the slot. */
int cs_serve_admit(const cs_serve_table *table, const cs_serve_table *pool,
                   const int32_t *pairs, int32_t count, void *stream);

/* Inputs of one step for each entry (slot, phase).  Phase p < W: forward
 * step t = p, writes a0 and aref.  Phase W <= p < 2W: backward step
 * t = 2W - 1 - p, restores a, a0, aref, factor and active set of step t from
 * the archive and writes abar = h vbar. */
int cs_serve_pre(const cs_serve_table *table, const int32_t *entries, int32_t count,
                 void *stream);

/* Consume the step's solver outputs for each entry.  Forward: archive step
 * t, v += h a, and at t = W - 1 set vbar = 2 (v - goal).  Backward: write
 * taubar_t = M^{-T} a0bar and vbar -= b J^T arefbar. */
int cs_serve_post(const cs_serve_table *table, const int32_t *entries, int32_t count,
                  void *stream);

/* One solver launch of a tick: cs_forward (kind 0) or cs_ift_vjp (kind 1) of
 * the `count` slots whose indices sit in the tick's device list at element
 * `order`, with the batch description classes[cls] (its order and count
 * replaced), on `stream` (lane 0) or `side` (lane 1). */
typedef struct cs_serve_launch {
    int32_t kind;
    int32_t cls;
    int32_t lane;
    int32_t count;
    int32_t order;
} cs_serve_launch;

/* The device work of one serving tick in one call, in stream order:
 *   1. copy host_list[0 .. list_len) (pinned host memory) to dev_list and
 *      record ev_list on `stream` (the caller may reuse host_list once
 *      ev_list has completed);
 *   2. cs_serve_admit of the n_admit pairs at dev_list[0 ..), if n_admit > 0;
 *   3. cs_serve_pre of the n_entries (slot, phase) pairs that follow them;
 *   4. every launch of `launches` on its lane: when any launch is on lane 1,
 *      `side` first waits for ev_fork recorded on `stream` after step 3, and
 *      `stream` waits for ev_join recorded on `side` after its last launch;
 *      the launches of one tick must name disjoint slots;
 *   5. cs_serve_post of the same entries.
 * Forwards use table->M, J, a0, aref, D, a and state (state_bytes) and write
 * status / iters; VJPs read the same and abar and write a0bar and arefbar.
 * Streams and events are HIP handles (NULL stream: the null stream); side,
 * ev_fork and ev_join may be NULL when no launch is on lane 1.  Returns
 * CS_EINVAL for a bad argument before anything is enqueued (kind, lane,
 * class index, counts, list bounds), else the first error of the steps;
 * allocates nothing. */
int cs_serve_tick(const cs_serve_table *table, const cs_serve_table *pool,
                  const cs_batch *classes, int32_t nclasses, const cs_solver_params *params,
                  size_t state_bytes, int32_t *status, int32_t *iters,
                  const int32_t *host_list, int32_t *dev_list, int32_t list_len,
                  int32_t n_admit, int32_t n_entries,
                  const cs_serve_launch *launches, int32_t nlaunch,
                  void *stream, void *side, void *ev_list, void *ev_fork, void *ev_join);

#ifdef __cplusplus
}
#endif

#endif
