"""Navigation cost terms of c1 on the GPU (curvature, distance to the
start-goal segment, steering angle), computed in the projection's final pass,
against the oracle through one CEM step."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2309_08235_amd import workloads as W
from tests.parity import oracle_problem
from tests.test_gpu_parity import _cem, _check_cem_step

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t32(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32).to(DEV)


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def P(gpu_lib):
    from paper_2309_08235_amd import priest
    assert torch.cuda.is_available()
    return priest


CASES = [
    ("2d all terms", W.C1, dict(w_acc=0.5, w_curv=0.2, w_path=0.3, w_steer=0.8, wheelbase=2.5,
                                eps=0.01)),
    ("2d path only", W.with_changes(W.C2, n_samples=300, n_proj=W.default_n_proj(300), n_elite=30,
                                    n_proj_iters=40), dict(w_acc=0.0, w_path=1.0)),
    ("3d curvature and path", W.with_changes(W.C3, n_samples=128, n_proj=W.default_n_proj(128),
                                             n_elite=16, n_proj_iters=30),
     dict(w_acc=1.0, w_curv=0.4, w_path=0.2, eps=0.05)),
]


@pytest.mark.parametrize("label,wl,weights", CASES, ids=[c[0] for c in CASES])
def test_weighted_cost_step_matches_oracle(P, label, wl, weights):
    say(f"weighted cost, one CEM step: {label}")
    gp = P.Problem.from_workload(wl)
    op = oracle_problem(wl)
    bc, obs = W.scene(wl, 1)
    cost_g = P.Cost(kind=P.COST_WEIGHTED, **weights)
    cost_o = O.Cost(kind=1, **weights)
    cem = _cem(wl)
    cem.cost = cost_g
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    noise = W.standard_normals(12, (1, wl.n_samples, wl.D))
    mu, cov = t32(mu0), t32(cov0)
    out = gp.plan(t32(bc), t32(obs), cem, mu, cov, noise=t32(noise),
                  out=gp.plan_outputs(cem, 1, full=True))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, obs, wl, cem, mu0, cov0, noise[0], out, np64(mu), np64(cov),
                    label, cost=cost_o)
    gp.close()


def test_weighted_acceleration_only_is_the_smoothness_cost_bitwise(P):
    say("weighted cost with w_acc = 1 only equals the smoothness cost bit for bit")
    wl = W.with_changes(W.C1, n_proj_iters=20)
    gp = P.Problem.from_workload(wl)
    bc, obs = W.scene(wl, 0)
    res = []
    for cost in (None, P.Cost(kind=P.COST_WEIGHTED, w_acc=1.0)):
        cem = _cem(wl, n_cem=2)
        cem.cost = cost
        mu, cov = t32(W.initial_mean(wl)), t32(W.initial_cov(wl))
        out = gp.plan(t32(bc), t32(obs), cem, mu, cov, seed=4, out=gp.plan_outputs(cem, 1, full=True))
        torch.cuda.synchronize()
        res.append([out[k].cpu().numpy() for k in ("c1", "best_xi", "elite_idx")] + [mu.cpu().numpy()])
    for a, b in zip(*res):
        np.testing.assert_array_equal(a, b)
    gp.close()


def test_cost_validation(P):
    wl3 = W.C3
    gp = P.Problem.from_workload(wl3)
    bc, obs = W.scene(wl3, 0)
    mu, cov = t32(W.initial_mean(wl3)), t32(W.initial_cov(wl3))
    for bad in (P.Cost(kind=P.COST_WEIGHTED, w_steer=1.0), P.Cost(kind=P.COST_WEIGHTED, w_curv=-1.0),
                P.Cost(kind=P.COST_WEIGHTED, w_curv=1.0, eps=0.0), P.Cost(kind=7)):
        cem = _cem(wl3)
        cem.cost = bad
        with pytest.raises(P.PriestError):
            gp.plan(t32(bc), t32(obs), cem, mu, cov)
    gp.close()
