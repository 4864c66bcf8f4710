"""priest_project_batch: several problems' projections in one launch equal
the single-problem projections bit for bit, and match the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2309_08235_amd import workloads as W
from tests.parity import check_projection, oracle_problem

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


@pytest.mark.parametrize("label,wl,N,paths", [
    ("2d", W.with_changes(W.C2, n_proj_iters=40), 173, False),
    ("3d", W.with_changes(W.C3, n_proj_iters=20), 45, False),
    ("2d paths", W.with_changes(W.C2, n_proj_iters=30), 60, True),
], ids=["2d", "3d", "2d paths"])
def test_project_batch_equals_single_projections(P, label, wl, N, paths):
    say(f"project_batch {label}: 3 problems, N={N}")
    nP = 3
    kw = dict(obs_model=P.OBS_PATH) if paths else {}
    gp = P.Problem.from_workload(wl, **kw)
    scenes = [W.scene(wl, q) for q in range(nP)]
    obs = [W.trajectory_obstacles(wl, s[1], swirl=1.0, seed=q) if paths else s[1]
           for q, s in enumerate(scenes)]
    bc = np.stack([s[0] for s in scenes])
    obs = np.stack(obs)
    xi = np.stack([W.samples(wl, 10 + q, n=N) for q in range(nP)]).astype(np.float32)
    xo, r, c1 = gp.project_batch(t32(bc), t32(obs), t32(xi), wl.n_proj_iters)
    torch.cuda.synchronize()
    for q in range(nP):
        x1, r1, c11 = gp.project(t32(bc[q]), t32(obs[q]), t32(xi[q]), wl.n_proj_iters)
        torch.cuda.synchronize()
        assert torch.equal(xo[q], x1) and torch.equal(r[q], r1) and torch.equal(c1[q], c11), q
    op = oracle_problem(wl, **({"obs_model": 1} if paths else {}))
    q = nP - 1
    idx = np.arange(min(N, 12))
    pr = O.project(op, bc[q], obs[q], xi[q][idx].astype(np.float64), wl.n_proj_iters)
    check_projection(op, bc[q], obs[q], xi[q][idx], xo[q].cpu().numpy()[idx].astype(np.float64),
                     pr.xi_bar, wl.n_proj_iters, label=label)
    gp.close()
