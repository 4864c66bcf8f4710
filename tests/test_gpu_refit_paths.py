"""The refit kernel's two selection paths inside real plans.

A plan hands the ordered constraint-elite set (proj_idx) to its last CEM
iteration only; without it every iteration selects by radix selects and a
ranking by counting, with it by two stable radix sorts.  Both must give the
same plan bit for bit: the same elites in the same order, hence the same
refit, factor and draws.  The sorting path is checked against the oracle in
test_gpu_parity; here the two paths are checked against each other on
problems that reach each instantiation of the refit (D = 22, 24, 26, 32, 33,
48: factors padded to 24, 36 and 48 rows; 1..4 keys per thread), plus one
oracle check of a 48-coefficient refit."""
import sys

import numpy as np
import pytest
import torch

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
def priest(gpu_lib):
    from paper_2309_08235_amd import priest as P
    assert torch.cuda.is_available()
    return P


CASES = [
    # (label, base workload, changes)
    ("2d D=22 N=64", W.C1, dict(n_cem=3)),
    ("2d D=24 N=300", W.C1, dict(n_coeff=12, n_samples=300, n_proj=220, n_elite=30, n_cem=3)),
    ("2d D=26 N=1000", W.C1, dict(n_coeff=13, n_samples=1000, n_proj=727, n_elite=100, n_cem=2)),
    ("2d D=32 N=2048", W.C1, dict(n_coeff=16, n_samples=2048, n_proj=1500, n_elite=200, n_cem=2)),
    ("3d D=33 N=1500", W.C3, dict(n_obs=20, n_steps=50, n_samples=1500, n_proj=1100, n_elite=150,
                                  n_cem=2)),
    ("3d D=48 N=400", W.C3, dict(n_obs=20, n_steps=50, n_coeff=16, n_samples=400, n_proj=300,
                                 n_elite=40, n_cem=2)),
    ("2d n_elite=600 (sorting in every iteration)", W.C1,
     dict(n_samples=1000, n_proj=800, n_elite=600, n_cem=2)),
]


@pytest.mark.parametrize("label,base,chg", CASES, ids=[c[0] for c in CASES])
def test_plan_identical_with_and_without_ordered_set(priest, label, base, chg):
    say(f"refit paths: {label}")
    chg = dict(chg)
    n_cem = chg.pop("n_cem", 1)
    wl = W.with_changes(base, n_proj_iters=20, **chg)
    gp = priest.Problem.from_workload(wl)
    bc, obs = (t32(a) for a in W.scene(wl, 2))
    cem = _cem(wl, n_cem=n_cem)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    res = []
    for ordered in (True, False):
        mu, cov = t32(mu0), t32(cov0)
        out = gp.plan_outputs(cem)
        if not ordered:
            del out["proj_idx"]
        gp.plan(bc, obs, cem, mu, cov, seed=11, out=out)
        torch.cuda.synchronize()
        res.append((out, mu, cov))
    (a, mua, cova), (b, mub, covb) = res
    for k in ("best_xi", "best_cost", "elite_idx", "xi", "xi_bar", "resid", "c1", "status"):
        assert torch.equal(a[k], b[k]), (label, k)
    assert torch.equal(mua, mub) and torch.equal(cova, covb), label
    assert int(a["status"][0]) == 0
    gp.close()


def test_refit_48_coefficients_against_oracle(priest):
    """One CEM iteration with D = 48 (factor rows padded to 48) against the
    oracle's refit of the GPU's elites."""
    say("refit paths: 3d D=48 one CEM iteration against the oracle")
    wl = W.with_changes(W.C3, n_obs=20, n_steps=50, n_coeff=16, n_samples=200,
                        n_proj=W.default_n_proj(200), n_elite=30, n_proj_iters=30)
    gp = priest.Problem.from_workload(wl)
    op = oracle_problem(wl)
    bc = W.boundary_values(wl)
    obs = W.obstacles(wl, 3005)
    cem = _cem(wl)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    noise = W.standard_normals(37, (1, wl.n_samples, wl.D))
    mu, cov = t32(mu0), t32(cov0)
    out = gp.plan(t32(bc), t32(obs), cem, mu, cov, noise=t32(noise))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, obs, wl, cem, mu0, cov0, noise[0], out, np64(mu), np64(cov), "3d D=48")
    gp.close()
