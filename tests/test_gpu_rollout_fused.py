"""The fused rollout (cs_rollout): a whole semi-implicit rollout through the
contact solve, and its backward through time, each in one launch.

* FP64 forward v_T against a rollout driven by the oracle, instance by
  instance (1e-9), every solve converged;
* FP64 gradient (tau-bar for every step, v-bar_0) of ||v_T - v_goal||^2
  against the oracle-driven adjoint (oracle forwards, then eq. 17 with the
  oracle's VJP in reverse), instance by instance (1e-9);
* one launch (forward + backward) equals a forward launch followed by a
  backward launch, and recomputing H_t in the backward equals keeping its
  factor -- both bit for bit;
* the autograd wrapper equals the layered rollout's autograd gradient;
* FP32 against the FP64 oracle-driven rollout on the FP32-rounded inputs,
  instance by instance, wherever the rollout takes the oracle's contact
  schedule and no step of the oracle's rollout has a row within 1e-7
  (relative) of the cone boundary;
* argument errors: workspace too small, n over the fused kernel's limit, a
  backward call without v-bar_T.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import rollout as R
from paper_2607_24959_amd import solver, synth
from paper_2607_24959_amd import _native as N

pytestmark = pytest.mark.gpu

H_STEP = 0.002


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_rollout(Pn, b, max_iter, tol, grad=True):
    """Instance b's rollout driven by the oracle: v_T, tau-bar [T, n], v-bar_0,
    every step's status and the smallest relative row margin of every step."""
    M, J, D = Pn["M"][b], Pn["J"][b], Pn["D"][b]
    c = -synth.K_SPRING * np.repeat(Pn["pen"][b], synth.ROWS_PER_CONTACT)
    v = Pn["v0"][b].copy()
    steps, margins = [], []
    for t in range(Pn["tau"].shape[0]):
        a0 = np.linalg.solve(M, Pn["tau"][t, b])
        aref = -synth.B_DAMP * (J @ v) + c
        res = oracle.forward(M, J, a0, aref, D, max_iter=max_iter, tol=tol)
        steps.append((a0, aref, res["a"], res["active"], res["status"]))
        r = J @ res["a"] - aref
        sc = np.abs(aref) + np.abs(J) @ np.abs(res["a"]) + 1e-300
        margins.append(float((np.abs(r) / sc).min()) if r.size else np.inf)
        v = v + H_STEP * res["a"]
    out = dict(v_T=v, status=[s[4] for s in steps], margin=min(margins),
               active=np.stack([s[3] for s in steps]))
    if grad:
        vbar = 2.0 * (v - Pn["v_goal"][b])
        taubar = np.zeros((len(steps), M.shape[0]))
        for t in reversed(range(len(steps))):
            a0, aref, a, act, _ = steps[t]
            g = oracle.ift_vjp(M, J, a0, aref, D, a, H_STEP * vbar, active=act)
            taubar[t] = np.linalg.solve(M.T, g["a0"])
            vbar = vbar - synth.B_DAMP * (J.T @ g["aref"])
        out.update(tau_bar=taubar, v0_bar=vbar)
    return out


def test_fused_forward_matches_oracle_rollout_fp64():
    _needs_gpu()
    P = R.make_rollout_problem(64, 18, 32, 10, seed=20260729)
    with torch.no_grad():
        vT, st = R.fused_rollout(P["M"], P["J"], P["D"], P["pen"], P["v0"], P["tau"], h=H_STEP,
                                 max_iter=60, tol=1e-12)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == N.ST_CONVERGED)
    Pn = {k: v.cpu().numpy() for k, v in P.items()}
    g = vT.cpu().numpy()
    for b in range(64):
        o = _oracle_rollout(Pn, b, 60, 1e-12, grad=False)
        assert all(s == oracle.ST_CONVERGED for s in o["status"]), b
        e = np.linalg.norm(g[b] - o["v_T"]) / np.linalg.norm(o["v_T"])
        assert e <= 1e-9, (b, e)


@pytest.mark.parametrize("recompute", [False, True])
def test_fused_gradient_matches_oracle_adjoint_fp64(recompute):
    """B=1024, nv=18, 32 contacts, horizon 50 (the rollout workload), FP64,
    one launch; the first 24 instances against the oracle-driven adjoint."""
    _needs_gpu()
    P = R.make_rollout_problem(1024, 18, 32, 50, seed=20260727)
    out = R.fused_loss_grad(P["M"], P["J"], P["D"], P["pen"], P["v0"], P["tau"], P["v_goal"],
                            h=H_STEP, max_iter=60, tol=1e-12, recompute=recompute)
    torch.cuda.synchronize()
    assert np.all(out["status"].cpu().numpy() == N.ST_CONVERGED)
    Pn = {k: v.cpu().numpy() for k, v in P.items()}
    tb = out["tau_bar"].cpu().numpy()
    vb = out["v0_bar"].cpu().numpy()
    worst = 0.0
    for b in range(24):
        o = _oracle_rollout(Pn, b, 60, 1e-12)
        e1 = np.linalg.norm(tb[:, b] - o["tau_bar"]) / np.linalg.norm(o["tau_bar"])
        e2 = np.linalg.norm(vb[b] - o["v0_bar"]) / np.linalg.norm(o["v0_bar"])
        worst = max(worst, e1, e2)
        assert e1 <= 1e-9 and e2 <= 1e-9, (b, e1, e2)
    print("fused rollout gradient vs oracle adjoint: max", worst, "Newton steps per solve",
          float(out["iters"].float().mean()) / 50, flush=True)


def test_one_launch_equals_two_and_recompute_equals_store():
    _needs_gpu()
    P = R.make_rollout_problem(256, 18, 32, 20, seed=20260731)
    args = (P["M"], P["J"], P["D"], P["pen"], P["v0"], P["tau"])
    one = R.fused_loss_grad(*args, P["v_goal"], h=H_STEP, max_iter=60, tol=1e-12)
    rec = R.fused_loss_grad(*args, P["v_goal"], h=H_STEP, max_iter=60, tol=1e-12, recompute=True)
    batch, Mc, Jc, Dc, c, v0c, tauc = R._fused_inputs(*args)
    f = R._fused_call(batch, N.ROLLOUT_FORWARD, 60, 1e-12, H_STEP, Mc, Jc, Dc, c, v0c, tauc)
    vbar = (2.0 * (f["v_T"] - P["v_goal"])).contiguous()
    b = R._fused_call(batch, N.ROLLOUT_BACKWARD, 60, 1e-12, H_STEP, Mc, Jc, Dc, c, None, tauc,
                      vbar_T=vbar, ws=f["ws"], status=f["status"])
    torch.cuda.synchronize()
    assert torch.equal(one["v_T"], f["v_T"])
    assert torch.equal(one["tau_bar"], b["tau_bar"]) and torch.equal(one["v0_bar"], b["v0_bar"])
    assert torch.equal(one["v_T"], rec["v_T"])
    assert torch.equal(one["tau_bar"], rec["tau_bar"]) and torch.equal(one["v0_bar"], rec["v0_bar"])
    ws_store = N.rollout_workspace_bytes(batch.desc, N.CsRolloutParams(20, 3, 60, 0, 1e-12, H_STEP, 1.0))
    ws_rec = N.rollout_workspace_bytes(batch.desc, N.CsRolloutParams(20, 7, 60, 0, 1e-12, H_STEP, 1.0))
    assert ws_rec < ws_store / 5, (ws_rec, ws_store)


def test_autograd_wrapper_matches_layered_rollout():
    _needs_gpu()
    P = R.make_rollout_problem(128, 18, 32, 20, seed=20260801)

    def grads(fn):
        tau = P["tau"].clone().requires_grad_(True)
        v0 = P["v0"].clone().requires_grad_(True)
        vT = fn(tau, v0)
        ((vT - P["v_goal"]) ** 2).sum().backward()
        return vT.detach(), tau.grad.detach(), v0.grad.detach()

    fused = grads(lambda tau, v0: R.fused_rollout(P["M"], P["J"], P["D"], P["pen"], v0, tau,
                                                  h=H_STEP, max_iter=60, tol=1e-12)[0])
    layered = grads(lambda tau, v0: R.rollout(P["M"], P["J"], P["D"], P["pen"], v0, tau, h=H_STEP,
                                              max_iter=60, tol=1e-12))
    for x, y, name in zip(fused, layered, ("v_T", "tau_bar", "v0_bar")):
        e = ((x - y).flatten(1).norm(dim=1) / y.flatten(1).norm(dim=1)).max().item() \
            if name != "tau_bar" else \
            ((x - y).transpose(0, 1).flatten(1).norm(dim=1) /
             y.transpose(0, 1).flatten(1).norm(dim=1)).max().item()
        assert e <= 1e-9, (name, e)


def test_fused_fp32_against_oracle():
    """FP32, B=256, nv=9, 16 contacts, horizon 5: v_T within 1e-4 and the
    gradient within 1e-3 of the FP64 oracle-driven rollout on the same
    FP32-rounded inputs, for every instance whose rollout takes the oracle's
    contact schedule (each step's active set, read from the workspace) and
    keeps each row at least 1e-7 (relative) from the cone boundary at every
    step of the oracle's rollout; at least 90 % of the instances qualify."""
    _needs_gpu()
    Bn, T_h = 256, 5
    P = {k: v.float() for k, v in R.make_rollout_problem(Bn, 9, 16, T_h, seed=20260802).items()}
    out = R.fused_loss_grad(P["M"], P["J"], P["D"], P["pen"], P["v0"], P["tau"], P["v_goal"],
                            h=H_STEP, max_iter=60, tol=1e-5, recompute=True)
    torch.cuda.synchronize()
    assert np.all(out["status"].cpu().numpy() & (N.ST_NONFINITE | N.ST_NOTSPD) == 0)
    m = P["J"].shape[1]
    step = (Bn * m + 255) // 256 * 256          # recomputing: each step holds the masks only
    act = out["ws"][:T_h * step].view(T_h, step)[:, :Bn * m].view(T_h, Bn, m).cpu().numpy() != 0
    Pn = {k: v.double().cpu().numpy() for k, v in P.items()}
    vT = out["v_T"].double().cpu().numpy()
    tb = out["tau_bar"].double().cpu().numpy()
    checked, worst_v, worst_g = 0, 0.0, 0.0
    for b in range(Bn):
        o = _oracle_rollout(Pn, b, 80, 1e-12)
        if o["margin"] < 1e-7 or not np.array_equal(act[:, b], o["active"]):
            continue
        checked += 1
        ev = np.linalg.norm(vT[b] - o["v_T"]) / np.linalg.norm(o["v_T"])
        eg = np.linalg.norm(tb[:, b] - o["tau_bar"]) / np.linalg.norm(o["tau_bar"])
        worst_v, worst_g = max(worst_v, ev), max(worst_g, eg)
        assert ev <= 1e-4, (b, ev)
        assert eg <= 1e-3, (b, eg)
    print("fused FP32 vs oracle: checked", checked / Bn, "v_T max", worst_v, "tau_bar max", worst_g,
          flush=True)
    assert checked / Bn >= 0.9


def test_fused_argument_errors():
    _needs_gpu()
    P = R.make_rollout_problem(8, 9, 4, 3, seed=1)
    batch, Mc, Jc, Dc, c, v0c, tauc = R._fused_inputs(P["M"], P["J"], P["D"], P["pen"], P["v0"],
                                                      P["tau"])
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(N.CsError) as e:
        R._fused_call(batch, N.ROLLOUT_FORWARD, 20, 1e-12, H_STEP, Mc, Jc, Dc, c, v0c, tauc, ws=small)
    assert e.value.code == N.CS_ENOSPC
    with pytest.raises(N.CsError) as e:
        R._fused_call(batch, N.ROLLOUT_BACKWARD, 20, 1e-12, H_STEP, Mc, Jc, Dc, c, None, tauc)
    assert e.value.code == N.CS_EINVAL
    Pb = R.make_rollout_problem(2, 36, 4, 2, seed=2)
    with pytest.raises(N.CsError) as e:
        R.fused_rollout(Pb["M"], Pb["J"], Pb["D"], Pb["pen"], Pb["v0"], Pb["tau"])
    assert e.value.code == N.CS_EUNSUPPORTED
