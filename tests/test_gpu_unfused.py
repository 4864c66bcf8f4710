"""The unfused projection (the plain baseline form) against the oracle and
against the fused kernel, called through the C ABI."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2309_08235_amd import workloads as W
from tests.parity import check_projection, oracle_problem, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t32(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32).to(DEV)


@pytest.fixture(scope="module")
def P(gpu_lib):
    from paper_2309_08235_amd import priest
    assert torch.cuda.is_available()
    return priest


@pytest.mark.parametrize("cfg,N,n_iter", [("c1", 64, 50), ("c2", 150, 40), ("c3", 40, 30)])
def test_unfused_matches_oracle(P, cfg, N, n_iter):
    wl = W.CONFIGS[cfg]
    say(f"unfused projection {cfg} N={N} iters={n_iter} vs oracle")
    prob = P.Problem.from_workload(wl)
    op = oracle_problem(wl)
    bc, obs = W.scene(wl, 0)
    xi = W.samples(wl, 9, n=N).astype(np.float32)
    xo, r, c1 = prob.project_unfused(t32(bc), t32(obs), t32(xi), n_iter)
    torch.cuda.synchronize()
    pr = O.project(op, bc, obs, xi.astype(np.float64), n_iter)
    check_projection(op, bc, obs, xi, xo.cpu().numpy().astype(np.float64), pr.xi_bar, n_iter,
                     label=f"unfused {cfg}")
    np.testing.assert_allclose(r.cpu().numpy(), pr.resid, atol=2e-3 * max(1.0, pr.resid.max()))
    c1_ref = O.smoothness_cost(op, pr.xi_bar)
    np.testing.assert_allclose(c1.cpu().numpy(), c1_ref, rtol=2e-3, atol=1e-3)
    prob.close()


def test_unfused_agrees_with_fused_and_aliases(P):
    say("unfused vs fused at the C2 shape, N=333, in-place output")
    wl = W.C2
    prob = P.Problem.from_workload(wl)
    bc, obs = W.scene(wl, 1)
    xi = t32(W.samples(wl, 2, n=333))
    xf, rf, cf = prob.project(t32(bc), t32(obs), xi, 60)
    ws = torch.empty(P.priest_project_unfused_workspace_size(prob.handle, 333), dtype=torch.uint8,
                     device=DEV)
    xu = xi.clone()
    ru = torch.empty(333, device=DEV)
    cu = torch.empty(333, device=DEV)
    P.priest_project_unfused(prob.handle, t32(bc), t32(obs), xu, 60, xu, ru, cu, ws)
    torch.cuda.synchronize()
    e = rel_err(xu.cpu().numpy(), xf.cpu().numpy())
    assert np.median(e) < 1e-5 and np.quantile(e, 0.99) < 1e-3, (np.median(e), e.max())
    prob.close()


def test_unfused_rejects_bf16_and_small_workspace(P):
    prob = P.Problem.from_workload(W.C1, precision=P.BF16_MIXED)
    xi = t32(W.samples(W.C1, 1, n=8))
    with pytest.raises(P.PriestError):
        prob.project_unfused(t32(W.scene(W.C1, 0)[0]), t32(W.scene(W.C1, 0)[1]), xi, 5)
    prob.close()
    prob = P.Problem.from_workload(W.C1)
    ws = torch.empty(16, dtype=torch.uint8, device=DEV)
    xo = torch.empty_like(xi)
    with pytest.raises(P.PriestError) as e:
        P.priest_project_unfused(prob.handle, t32(W.scene(W.C1, 0)[0]), t32(W.scene(W.C1, 0)[1]),
                                 xi, 5, xo, None, None, ws)
    assert e.value.code == P.PRIEST_ERR_NOMEM
    prob.close()


def test_unfused_odd_steps_against_oracle(P):
    """K = 51: rows of odd length, streamed in single-float loads."""
    wl = W.with_changes(W.C1, n_steps=51)
    say("unfused projection c1 with K=51, N=64, 30 iterations vs oracle")
    prob = P.Problem.from_workload(wl)
    op = oracle_problem(wl)
    bc, obs = W.scene(wl, 4)
    xi = W.samples(wl, 6, n=64).astype(np.float32)
    xo, r, _ = prob.project_unfused(t32(bc), t32(obs), t32(xi), 30)
    torch.cuda.synchronize()
    pr = O.project(op, bc, obs, xi.astype(np.float64), 30)
    check_projection(op, bc, obs, xi, xo.cpu().numpy().astype(np.float64), pr.xi_bar, 30,
                     label="unfused K=51")
    np.testing.assert_allclose(r.cpu().numpy(), pr.resid, atol=2e-3 * max(1.0, pr.resid.max()))
    prob.close()


def test_unfused_large_batch_against_fused_and_oracle(P):
    """N = 40000 in 2D: 80000 update rows, enough for one lane per row (small
    batches split each row over a group of lanes)."""
    wl = W.C2
    N, n_iter = 40000, 20
    say(f"unfused vs fused and an oracle sample, C2 shape, N={N}, {n_iter} iterations")
    prob = P.Problem.from_workload(wl)
    op = oracle_problem(wl)
    bc, obs = W.scene(wl, 3)
    xi_np = W.samples(wl, 5, n=N).astype(np.float32)
    xi = t32(xi_np)
    xf, _, _ = prob.project(t32(bc), t32(obs), xi, n_iter)
    xu, _, _ = prob.project_unfused(t32(bc), t32(obs), xi, n_iter)
    torch.cuda.synchronize()
    xu_np = xu.cpu().numpy()
    e = rel_err(xu_np, xf.cpu().numpy())
    assert np.median(e) < 1e-5 and np.quantile(e, 0.99) < 1e-3, (np.median(e), e.max())
    idx = np.sort(np.random.default_rng(0).choice(N, 48, replace=False))
    pr = O.project(op, bc, obs, xi_np[idx].astype(np.float64), n_iter)
    check_projection(op, bc, obs, xi_np[idx], xu_np[idx].astype(np.float64), pr.xi_bar, n_iter,
                     label="unfused N=40000 sample")
    prob.close()
