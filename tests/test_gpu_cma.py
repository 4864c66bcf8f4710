"""The CMA-ES-style covariance update on the GPU (the remark after eqs.
(9a)-(9c)), against the oracle through one and two CEM steps."""
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


@pytest.mark.parametrize("label,wl", [
    ("c1", W.C1),
    ("c2 shape N=300", W.with_changes(W.C2, n_samples=300, n_proj=W.default_n_proj(300), n_elite=30,
                                      n_proj_iters=40)),
    ("c3 shape N=128", W.with_changes(W.C3, n_samples=128, n_proj=W.default_n_proj(128), n_elite=16,
                                      n_proj_iters=30)),
], ids=["c1", "c2", "c3"])
def test_cma_two_steps_match_oracle(P, label, wl):
    say(f"CMA update, two CEM steps: {label}")
    gp = P.Problem.from_workload(wl)
    op = oracle_problem(wl)
    bc, obs = W.scene(wl, 3)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    noise = W.standard_normals(5, (2, wl.n_samples, wl.D))
    # step 1 alone
    cem1 = _cem(wl, n_cem=1, update=P.UPDATE_CMA)
    mu1, cov1 = t32(mu0), t32(cov0)
    out1 = gp.plan(t32(bc), t32(obs), cem1, mu1, cov1, noise=t32(noise[:1]),
                   out=gp.plan_outputs(cem1, 1, full=True))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, obs, wl, cem1, mu0, cov0, noise[0], out1, np64(mu1), np64(cov1),
                    f"{label} step 1")
    # the path after step 1, from the GPU's own elites
    xb1 = np64(out1["xi_bar"][0])
    el1 = out1["elite_idx"][0].cpu().numpy()
    caug1 = (out1["c1"][0].cpu().numpy() + out1["resid"][0].cpu().numpy()).astype(np.float64)
    _, _, pc1 = O.refit_cma(mu0, cov0, np.zeros(wl.D), xb1[el1], caug1[el1], cem1.sigma, cem1.gamma)
    # steps 1 and 2 in one plan: its first step is the run above, bit for bit
    cem2 = _cem(wl, n_cem=2, update=P.UPDATE_CMA)
    mu2, cov2 = t32(mu0), t32(cov0)
    out2 = gp.plan(t32(bc), t32(obs), cem2, mu2, cov2, noise=t32(noise),
                   out=gp.plan_outputs(cem2, 1, full=True))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, obs, wl, cem2, np64(mu1), np64(cov1), noise[1], out2, np64(mu2),
                    np64(cov2), f"{label} step 2", pc=pc1)
    gp.close()


def test_cma_rule_is_rejected_when_unknown_and_differs_from_mppi(P):
    wl = W.C1
    gp = P.Problem.from_workload(wl)
    bc, obs = W.scene(wl, 0)
    cem = _cem(wl, update=5)
    with pytest.raises(P.PriestError):
        gp.plan(t32(bc), t32(obs), cem, t32(W.initial_mean(wl)), t32(W.initial_cov(wl)))
    covs = []
    for rule in (P.UPDATE_MPPI, P.UPDATE_CMA):
        cem = _cem(wl, update=rule)
        mu, cov = t32(W.initial_mean(wl)), t32(W.initial_cov(wl))
        gp.plan(t32(bc), t32(obs), cem, mu, cov, seed=2)
        torch.cuda.synchronize()
        covs.append(np64(cov))
    assert np.abs(covs[0] - covs[1]).max() > 1e-3
    gp.close()
