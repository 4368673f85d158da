"""Seeded synthetic contact-solve instances.

This module only draws inputs.  It holds none of the solver's arithmetic
and is shared by the FP64 oracle tests, the GPU parity tests and the
benchmark, so both sides of every comparison see the same numbers.

Instance recipe (one instance = one regularised contact block of the
reduced problem in Sec. III-A, eq. 5, with pyramidal friction rows):

* ``M = L L^T / n + I`` with ``L_ij ~ N(0, 1)``                (SPD mass matrix)
* per contact ``c``: ``J_n, J_t1, J_t2`` with entries ``~ N(0, 1/n)``
  (second argument of N is a variance), ``mu_c ~ U[0.5, 1]``,
  ``pen_c ~ U[0, 0.01]``; its four pyramid rows are, in this order,
  ``J_n + mu J_t1, J_n - mu J_t1, J_n + mu J_t2, J_n - mu J_t2``
* per row ``R_i ~ logU[1e-4, 1e-2]`` and ``D_i = 1 / R_i``
* ``v ~ N(0, 1)`` per instance and
  ``aref_i = -b (J_i . v) - k pen_c`` with ``b = 2 / timeconst`` and
  ``k = 1 / (timeconst^2 dampratio^2)``, ``timeconst = 0.02``,
  ``dampratio = 1`` (spring-damper reference acceleration)
* ``a0 ~ N(0, 10)`` and the output cotangent ``abar ~ N(0, 1)``.

Uniform batches draw every field for the whole batch at once from one
``PCG64`` stream in the fixed order L, J_n, J_t1, J_t2, mu, pen, R, v, a0,
abar.  Uneven (packed) batches draw instance ``i`` from its own stream
seeded with ``(seed, i)`` in the same field order, so an instance is the
same whatever batch it is placed in.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

TIMECONST = 0.02
DAMPRATIO = 1.0
B_DAMP = 2.0 / TIMECONST                               # 100
K_SPRING = 1.0 / (TIMECONST ** 2 * DAMPRATIO ** 2)      # 2500
ROWS_PER_CONTACT = 4

SEED_BASE = 20260724


def _pyramid_rows(Jn, Jt1, Jt2, mu):
    """Stack the four pyramid edge rows per contact along the row axis.

    Shapes: ``J* [..., nc, n]``, ``mu [..., nc]`` -> ``[..., 4 nc, n]``.
    """
    mu = mu[..., None]
    rows = np.stack([Jn + mu * Jt1, Jn - mu * Jt1, Jn + mu * Jt2, Jn - mu * Jt2],
                    axis=-2)                                # [..., nc, 4, n]
    return rows.reshape(*Jn.shape[:-2], Jn.shape[-2] * ROWS_PER_CONTACT, Jn.shape[-1])


def aref_from(J, v, pen):
    """Reference acceleration of the spring-damper rows: -b J v - k pen.

    ``J [..., m, n]``, ``v [..., n]``, ``pen [..., nc]`` (one per contact).
    """
    pen_rows = np.repeat(pen, ROWS_PER_CONTACT, axis=-1)
    return -B_DAMP * np.einsum("...ij,...j->...i", J, v) - K_SPRING * pen_rows


@dataclass
class UniformBatch:
    """``B`` instances of one shape, row-major ``[B, ...]`` arrays."""
    n: int
    nc: int
    M: np.ndarray
    J: np.ndarray
    a0: np.ndarray
    aref: np.ndarray
    D: np.ndarray
    abar: np.ndarray
    mu: np.ndarray
    pen: np.ndarray
    v: np.ndarray

    @property
    def B(self):
        return self.M.shape[0]

    @property
    def m(self):
        return self.nc * ROWS_PER_CONTACT

    def astype(self, dtype):
        """Copy with every array cast (FP32 configs round once, here)."""
        kw = {k: getattr(self, k).astype(dtype) for k in
              ("M", "J", "a0", "aref", "D", "abar", "mu", "pen", "v")}
        return UniformBatch(n=self.n, nc=self.nc, **kw)

    def rounded(self, dtype):
        """FP64 copy of the ``dtype``-rounded inputs (what the oracle sees)."""
        return self.astype(dtype).astype(np.float64)

    def subset(self, idx):
        kw = {k: np.ascontiguousarray(getattr(self, k)[idx]) for k in
              ("M", "J", "a0", "aref", "D", "abar", "mu", "pen", "v")}
        return UniformBatch(n=self.n, nc=self.nc, **kw)


def uniform_batch(B: int, n: int, nc: int, seed: int, a0_var: float = 10.0) -> UniformBatch:
    rng = np.random.Generator(np.random.PCG64(seed))
    L = rng.standard_normal((B, n, n))
    sd = math.sqrt(1.0 / n)
    Jn = rng.normal(0.0, sd, (B, nc, n))
    Jt1 = rng.normal(0.0, sd, (B, nc, n))
    Jt2 = rng.normal(0.0, sd, (B, nc, n))
    mu = rng.uniform(0.5, 1.0, (B, nc))
    pen = rng.uniform(0.0, 0.01, (B, nc))
    R = np.exp(rng.uniform(math.log(1e-4), math.log(1e-2), (B, nc * ROWS_PER_CONTACT)))
    v = rng.standard_normal((B, n))
    a0 = rng.normal(0.0, math.sqrt(a0_var), (B, n))
    abar = rng.standard_normal((B, n))
    M = np.einsum("bij,bkj->bik", L, L) / n + np.eye(n)[None]
    J = _pyramid_rows(Jn, Jt1, Jt2, mu)
    aref = aref_from(J, v, pen)
    return UniformBatch(n=n, nc=nc, M=np.ascontiguousarray(M), J=np.ascontiguousarray(J),
                        a0=a0, aref=np.ascontiguousarray(aref), D=1.0 / R, abar=abar,
                        mu=mu, pen=pen, v=v)


def instance(seed: int, index: int, n: int, nc: int, a0_var: float = 10.0) -> dict:
    """One instance from its own stream ``(seed, index)`` (FP64 arrays)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, index])))
    L = rng.standard_normal((n, n))
    sd = math.sqrt(1.0 / n)
    Jn = rng.normal(0.0, sd, (nc, n))
    Jt1 = rng.normal(0.0, sd, (nc, n))
    Jt2 = rng.normal(0.0, sd, (nc, n))
    mu = rng.uniform(0.5, 1.0, nc)
    pen = rng.uniform(0.0, 0.01, nc)
    R = np.exp(rng.uniform(math.log(1e-4), math.log(1e-2), nc * ROWS_PER_CONTACT))
    v = rng.standard_normal(n)
    a0 = rng.normal(0.0, math.sqrt(a0_var), n)
    abar = rng.standard_normal(n)
    M = L @ L.T / n + np.eye(n)
    J = _pyramid_rows(Jn, Jt1, Jt2, mu) if nc else np.zeros((0, n))
    aref = aref_from(J, v, pen) if nc else np.zeros(0)
    return dict(n=n, nc=nc, M=M, J=np.ascontiguousarray(J), a0=a0, aref=aref,
                D=1.0 / R, abar=abar, mu=mu, pen=pen, v=v)


@dataclass
class PackedBatch:
    """Instances of different ``(n, m)`` packed back to back.

    Flat arrays hold the instances in index order; ``off_*[i]`` is the
    element offset of instance ``i`` (``off_*[B]`` is the total).
    """
    nv: np.ndarray            # int32 [B]
    nrows: np.ndarray         # int32 [B]
    off_nn: np.ndarray        # int64 [B+1]
    off_mn: np.ndarray
    off_n: np.ndarray
    off_m: np.ndarray
    M: np.ndarray
    J: np.ndarray
    a0: np.ndarray
    aref: np.ndarray
    D: np.ndarray
    abar: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def B(self):
        return int(self.nv.shape[0])

    def get(self, i: int) -> dict:
        n, m = int(self.nv[i]), int(self.nrows[i])
        return dict(
            n=n, m=m,
            M=self.M[self.off_nn[i]:self.off_nn[i + 1]].reshape(n, n),
            J=self.J[self.off_mn[i]:self.off_mn[i + 1]].reshape(m, n),
            a0=self.a0[self.off_n[i]:self.off_n[i + 1]],
            aref=self.aref[self.off_m[i]:self.off_m[i + 1]],
            D=self.D[self.off_m[i]:self.off_m[i + 1]],
            abar=self.abar[self.off_n[i]:self.off_n[i + 1]],
        )

    def astype(self, dtype):
        kw = {k: getattr(self, k).astype(dtype) for k in ("M", "J", "a0", "aref", "D", "abar")}
        return PackedBatch(nv=self.nv, nrows=self.nrows, off_nn=self.off_nn, off_mn=self.off_mn,
                           off_n=self.off_n, off_m=self.off_m, extra=dict(self.extra), **kw)

    def rounded(self, dtype):
        return self.astype(dtype).astype(np.float64)


def offsets(sizes) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(np.asarray(sizes, dtype=np.int64), out=off[1:])
    return off


def pack(instances) -> PackedBatch:
    """Pack a list of instance dicts (``n``, ``M``, ``J``, ...) into flat arrays."""
    nv = np.array([d["n"] for d in instances], dtype=np.int32)
    nr = np.array([d["J"].shape[0] for d in instances], dtype=np.int32)
    cat = lambda k: (np.concatenate([np.asarray(d[k], dtype=np.float64).ravel() for d in instances])
                     if instances else np.zeros(0))
    return PackedBatch(
        nv=nv, nrows=nr,
        off_nn=offsets(nv.astype(np.int64) ** 2), off_mn=offsets(nv.astype(np.int64) * nr),
        off_n=offsets(nv), off_m=offsets(nr),
        M=cat("M"), J=cat("J"), a0=cat("a0"), aref=cat("aref"), D=cat("D"), abar=cat("abar"))


def uneven_batch(B: int, nv_choices, nc_max: int, seed: int, nc_min: int = 0) -> PackedBatch:
    """Mixed batch: ``n_i`` uniform over ``nv_choices``, ``nc_i ~ U{nc_min..nc_max}``.

    The shape draws come from the batch stream ``seed``; instance ``i``'s
    values come from ``instance(seed, i, ...)``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nv = rng.choice(np.asarray(nv_choices, dtype=np.int64), size=B)
    nc = rng.integers(nc_min, nc_max + 1, size=B)
    insts = [instance(seed, i, int(nv[i]), int(nc[i])) for i in range(B)]
    pb = pack(insts)
    pb.extra["nc"] = nc.astype(np.int32)
    return pb


# Named workloads (sizes as used by the parity tests and the benchmark).
CONFIGS = {
    # plain method, FP64, B=64, nv=6, 4 contacts x 4 pyramid rows
    "fp64_b64_n6_nc4": dict(B=64, n=6, nc=4, dtype="f64", tol=1e-10, max_iter=10),
    # uniform FP32 batch, B=4096, nv=9, 16 contacts (64 rows)
    "fp32_b4096_n9_nc16": dict(B=4096, n=9, nc=16, dtype="f32", tol=1e-5, max_iter=10),
    # uneven FP32 batch, B=8192, nv in {3,9,18,36,96}, nc ~ U{0..256}
    "fp32_uneven_b8192": dict(B=8192, nv_choices=(3, 9, 18, 36, 96), nc_max=256, dtype="f32",
                              tol=1e-5, max_iter=10),
    # differentiable rollout, B=1024, nv=18, 32 contacts, h=0.002, horizon 50
    "rollout_b1024_n18_nc32": dict(B=1024, n=18, nc=32, h=0.002, horizon=50),
    # serving: 6-step MPC windows, nv in {3,9,18}, nc ~ U{0..64}
    "serve_mpc6": dict(nv_choices=(3, 9, 18), nc_max=64, window=6),
}


# ------------------------------------------------------------------ round cone
#
# Elliptic-cone instances: per contact the three rows J_n, J_t1, J_t2 as drawn
# above (no pyramid edges), mu_c ~ U[0.5, 1], R_N ~ logU[1e-4, 1e-2] per
# contact with D_N = 1 / R_N and the tangential weight D_T = D_N (equal normal
# and frictional impedance), aref = -b J v - k pen on the normal row and -b J v
# on the tangential rows.  Same PCG64 stream order as uniform_batch with the
# per-contact R in place of the per-row one.

@dataclass
class EllipticBatch:
    n: int
    nc: int
    M: np.ndarray      # [B, n, n]
    J: np.ndarray      # [B, 3 nc, n]: rows (N, T1, T2) per contact
    a0: np.ndarray
    aref: np.ndarray   # [B, 3 nc]
    dn: np.ndarray     # [B, nc]
    dt: np.ndarray     # [B, nc]
    mu: np.ndarray     # [B, nc]
    abar: np.ndarray

    @property
    def B(self):
        return self.M.shape[0]

    @property
    def m(self):
        return 3 * self.nc

    def astype(self, dtype):
        kw = {k: getattr(self, k).astype(dtype) for k in
              ("M", "J", "a0", "aref", "dn", "dt", "mu", "abar")}
        return EllipticBatch(n=self.n, nc=self.nc, **kw)

    def rounded(self, dtype):
        return self.astype(dtype).astype(np.float64)


def elliptic_batch(B: int, n: int, nc: int, seed: int, a0_var: float = 10.0) -> EllipticBatch:
    rng = np.random.Generator(np.random.PCG64(seed))
    L = rng.standard_normal((B, n, n))
    sd = math.sqrt(1.0 / n)
    Jn = rng.normal(0.0, sd, (B, nc, n))
    Jt1 = rng.normal(0.0, sd, (B, nc, n))
    Jt2 = rng.normal(0.0, sd, (B, nc, n))
    mu = rng.uniform(0.5, 1.0, (B, nc))
    pen = rng.uniform(0.0, 0.01, (B, nc))
    R = np.exp(rng.uniform(math.log(1e-4), math.log(1e-2), (B, nc)))
    v = rng.standard_normal((B, n))
    a0 = rng.normal(0.0, math.sqrt(a0_var), (B, n))
    abar = rng.standard_normal((B, n))
    M = np.einsum("bij,bkj->bik", L, L) / n + np.eye(n)[None]
    J = np.stack([Jn, Jt1, Jt2], axis=-2).reshape(B, 3 * nc, n)
    pos = np.stack([pen, np.zeros_like(pen), np.zeros_like(pen)], axis=-1).reshape(B, 3 * nc)
    aref = -B_DAMP * np.einsum("bij,bj->bi", J, v) - K_SPRING * pos
    return EllipticBatch(n=n, nc=nc, M=np.ascontiguousarray(M), J=np.ascontiguousarray(J),
                         a0=a0, aref=np.ascontiguousarray(aref), dn=1.0 / R, dt=1.0 / R,
                         mu=mu, abar=abar)


# ------------------------------------------------------------------ mixed rows
#
# Pyramid contact rows followed by ne equality rows and nf friction-loss rows
# (row kinds 0, 1, 2).  Equality and friction-loss rows: J entries ~ N(0, 1/n),
# R ~ logU[1e-4, 1e-2] (D = 1/R), aref = -b J v (damping only; the equality rows
# also -k e with a violation e ~ N(0, 0.01^2)); the friction-loss bound
# f ~ U[0.1, 100] per row (0 on the other rows).  Drawn after the uniform
# batch's fields from the same stream order, per batch.

KIND_ONE_SIDED, KIND_EQUALITY, KIND_FRICTION_LOSS = 0, 1, 2


@dataclass
class MixedBatch:
    n: int
    M: np.ndarray
    J: np.ndarray
    a0: np.ndarray
    aref: np.ndarray
    D: np.ndarray
    kind: np.ndarray    # uint8 [B, m]
    floss: np.ndarray   # [B, m]
    abar: np.ndarray

    @property
    def B(self):
        return self.M.shape[0]

    @property
    def m(self):
        return self.J.shape[1]

    def astype(self, dtype):
        kw = {k: getattr(self, k).astype(dtype) for k in ("M", "J", "a0", "aref", "D", "floss", "abar")}
        return MixedBatch(n=self.n, kind=self.kind.copy(), **kw)

    def rounded(self, dtype):
        return self.astype(dtype).astype(np.float64)


def mixed_batch(B: int, n: int, nc: int, ne: int, nf: int, seed: int) -> MixedBatch:
    u = uniform_batch(B, n, nc, seed)
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    sd = math.sqrt(1.0 / n)
    k = ne + nf
    Jx = rng.normal(0.0, sd, (B, k, n))
    R = np.exp(rng.uniform(math.log(1e-4), math.log(1e-2), (B, k)))
    e = rng.normal(0.0, 0.01, (B, ne))
    f = rng.uniform(0.1, 100.0, (B, nf))
    arefx = -B_DAMP * np.einsum("bij,bj->bi", Jx, u.v)
    arefx[:, :ne] -= K_SPRING * e
    J = np.concatenate([u.J, Jx], axis=1)
    aref = np.concatenate([u.aref, arefx], axis=1)
    D = np.concatenate([u.D, 1.0 / R], axis=1)
    m = J.shape[1]
    kind = np.zeros((B, m), np.uint8)
    kind[:, u.m:u.m + ne] = KIND_EQUALITY
    kind[:, u.m + ne:] = KIND_FRICTION_LOSS
    floss = np.zeros((B, m))
    floss[:, u.m + ne:] = f
    return MixedBatch(n=n, M=u.M, J=np.ascontiguousarray(J), a0=u.a0, aref=np.ascontiguousarray(aref),
                      D=np.ascontiguousarray(D), kind=kind, floss=floss, abar=u.abar)
