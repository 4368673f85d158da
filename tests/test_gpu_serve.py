"""Continuous batching of MPC windows on the GPU.

* every request served by the engine (FP64, mixed shapes n in {3,9,18},
  0..64 contacts, queued behind a small slot table) returns the same final
  velocity and actuation gradient as an autograd rollout of that request
  alone through contact_solve;
* every served request (FP64 and FP32) against a window driven by the FP64
  oracle: oracle forwards step by step, then the adjoints in reverse with the
  oracle's IFT VJP (a-bar_t = h v-bar_{t+1}, tau-bar_t = M^-T a0-bar_t,
  v-bar_t = v-bar_{t+1} - b J^T aref-bar_t);
* a request gives the same result alone and inside a mix (FP32);
* admission never holds more requests than the HBM budget has slots, and the
  engine's device footprint stays within the budget;
* a Poisson stream completes and reports latency percentiles.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import serve, synth
from paper_2607_24959_amd.rollout import rollout

pytestmark = pytest.mark.gpu

N_CHOICES = (3, 9, 18)
NC_MAX = 64
W = 6


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pool(count, dtype, seed=5):
    return serve.RequestPool(count, N_CHOICES, NC_MAX, W, seed, 18, 4 * NC_MAX, dtype, "cuda")


def _serve_all(engine, pool, ids):
    engine.attach_pool(pool)
    engine.keep_results = True
    for k, i in enumerate(ids):
        engine.submit(serve.Request(rid=k, pool_index=int(i), n=int(pool.n[i]), m=int(pool.m[i])))
    ticks = 0
    while len(engine.finished) < len(ids):
        engine.tick(float("inf"))
        ticks += 1
        assert ticks <= 2 * W * len(ids) + 4
    torch.cuda.synchronize()
    return ticks


def _reference(pool, i, max_iter, tol):
    """Autograd rollout of one request alone (IFT backward)."""
    n, m = int(pool.n[i]), int(pool.m[i])
    M = pool.Mp[i, :n, :n].unsqueeze(0)
    J = pool.Jp[i, :m, :n].unsqueeze(0)
    D = pool.D[i, :m].unsqueeze(0)
    pen = pool.pen[i, :m:4].unsqueeze(0)
    v0 = pool.v0[i, :n].unsqueeze(0)
    goal = pool.goal[i, :n]
    tau = pool.tau[i, :, :n].unsqueeze(1).clone().requires_grad_(True)
    v = rollout(M, J, D, pen, v0, tau, h=0.002, max_iter=max_iter, tol=tol)
    ((v[0] - goal) ** 2).sum().backward()
    return v[0].detach(), tau.grad[:, 0].detach()


def test_engine_matches_per_request_rollout_fp64():
    _needs_gpu()
    pool = _pool(24, torch.float64)
    eng = serve.Engine(slots=5, window=W, max_iter=60, tol=1e-12, dtype=torch.float64)
    ids = np.arange(24)
    _serve_all(eng, pool, ids)
    assert eng.max_active <= 5
    errs = []
    for k, i in enumerate(ids):
        n = int(pool.n[i])
        out = eng.results[k]
        v_ref, g_ref = _reference(pool, i, 60, 1e-12)
        ev = (torch.linalg.norm(out[:n] - v_ref) / torch.linalg.norm(v_ref)).item()
        eg = (torch.linalg.norm(out[n:] - g_ref.reshape(-1)) / torch.linalg.norm(g_ref)).item()
        errs.append((max(ev, eg), int(i), n, int(pool.m[i])))
    errs.sort(reverse=True)
    print("worst", errs[:3])
    assert errs[0][0] <= 1e-9, errs[:3]


def _oracle_window(M, J, D, pen_rows, v0, goal, tau, max_iter, tol, h=0.002):
    """Final velocity and tau-bar of one MPC window, driven by the oracle."""
    v = v0.copy()
    steps = []
    for t in range(tau.shape[0]):
        a0 = np.linalg.solve(M, tau[t])
        aref = -synth.B_DAMP * (J @ v) - synth.K_SPRING * pen_rows
        res = oracle.forward(M, J, a0, aref, D, max_iter=max_iter, tol=tol)
        assert res["status"] == oracle.ST_CONVERGED
        steps.append((a0, aref, res["a"], res["active"]))
        v = v + h * res["a"]
    vbar = 2.0 * (v - goal)
    taubar = np.zeros_like(tau)
    for t in reversed(range(tau.shape[0])):
        a0, aref, a, act = steps[t]
        g = oracle.ift_vjp(M, J, a0, aref, D, a, h * vbar, active=act)
        taubar[t] = np.linalg.solve(M.T, g["a0"])
        vbar = vbar - synth.B_DAMP * (J.T @ g["aref"])
    return v, taubar


def _window_inputs(pool, i):
    n, m = int(pool.n[i]), int(pool.m[i])
    f = lambda x: x.detach().double().cpu().numpy()
    return (f(pool.Mp[i, :n, :n]), f(pool.Jp[i, :m, :n]), f(pool.D[i, :m]), f(pool.pen[i, :m]),
            f(pool.v0[i, :n]), f(pool.goal[i, :n]), f(pool.tau[i, :, :n]))


def _rel(x, y):
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_engine_matches_oracle_window(dtype):
    """Every served request against the oracle-driven window: FP64 within 1e-9;
    FP32 within 1e-4 (v_W) and 1e-3 (tau-bar), or, where the oracle's own
    result moves by more than that under a one-rounding-unit perturbation of
    the request's inputs, within 10 times that movement."""
    _needs_gpu()
    fp64 = dtype == torch.float64
    pool = _pool(32, dtype, seed=23)
    eng = serve.Engine(slots=12, window=W, max_iter=60, tol=1e-12 if fp64 else 1e-5, dtype=dtype)
    ids = np.arange(32)
    _serve_all(eng, pool, ids)
    rng = np.random.default_rng(7)
    worst = []
    n_ill = 0
    for k, i in enumerate(ids):
        n = int(pool.n[i])
        out = eng.results[k].double().cpu().numpy()
        inp = _window_inputs(pool, i)
        v_o, tb_o = _oracle_window(*inp, max_iter=60, tol=1e-12)
        ev, eg = _rel(out[:n], v_o), _rel(out[n:], tb_o.ravel())
        if fp64:
            bv, bg = 1e-9, 1e-9
        else:
            sv = sg = 0.0
            for _ in range(2):
                pert = [x * (1.0 + 2.0 ** -24 * rng.choice([-1.0, 1.0], size=x.shape)) for x in inp]
                vp, tp = _oracle_window(*pert, max_iter=60, tol=1e-12)
                sv, sg = max(sv, _rel(vp, v_o)), max(sg, _rel(tp.ravel(), tb_o.ravel()))
            bv, bg = max(1e-4, 10 * sv), max(1e-3, 10 * sg)
            n_ill += int(bv > 1e-4 or bg > 1e-3)
        worst.append((ev / bv, eg / bg, int(i), n, int(pool.m[i])))
        assert ev <= bv and eg <= bg, (int(i), n, int(pool.m[i]), ev, bv, eg, bg)
    worst.sort(reverse=True)
    print(str(dtype), "worst error / bound", worst[:3], "ill-conditioned", n_ill)


def test_alone_equals_in_mix_fp32():
    _needs_gpu()
    pool = _pool(40, torch.float32, seed=11)
    mix = serve.Engine(slots=16, window=W, max_iter=20, tol=1e-5)
    _serve_all(mix, pool, np.arange(40))
    n_bitwise = 0
    for i in (0, 3, 17, 39):
        alone = serve.Engine(slots=1, window=W, max_iter=20, tol=1e-5)
        _serve_all(alone, pool, [i])
        a, b = alone.results[0], mix.results[i]
        n_bitwise += int(torch.equal(a, b))
        e = (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()
        assert e <= 1e-6, (i, e)
    print("bitwise equal", n_bitwise, "of 4")


def test_admission_within_budget():
    _needs_gpu()
    pool = _pool(12, torch.float32, seed=13)
    per = serve.slot_bytes(18, 4 * NC_MAX, W, 4)
    budget = 3 * per + per // 2
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    eng = serve.Engine(budget_bytes=budget, window=W, max_iter=20, tol=1e-5)
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - base
    assert eng.S == 3
    # slot arrays plus the allocator's rounding of each tensor
    assert held <= budget + 64 * 1024, (held, budget)
    _serve_all(eng, pool, np.arange(12))
    assert eng.max_active == 3
    assert len(eng.finished) == 12
    with pytest.raises(ValueError):
        serve.Engine(budget_bytes=per - 1, window=W)


@pytest.mark.parametrize("rate", [2000.0, 20000.0])
def test_poisson_stream_reports_latency(rate):
    _needs_gpu()
    pool = _pool(64, torch.float32, seed=17)
    eng = serve.Engine(slots=1024, window=W, max_iter=10, tol=1e-5)
    eng.attach_pool(pool)
    res = serve.run_stream(eng, rate=rate, n_requests=1000, warmup=100, seed=1)
    print(res)
    assert res["requests"] == 1000
    assert 0 < res["p50_ms"] <= res["p99_ms"] < 1e4
    # every request took its 2W ticks: latency is at least that many tick times
    assert res["max_active"] <= 1024
