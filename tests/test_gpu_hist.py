"""Residual history of the projection (the per-iteration residual of Alg. 1's
projection, ||F xi_bar^k - e^{k+1}||) on the GPU against the oracle's."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2309_08235_amd import workloads as W
from tests.parity import oracle_problem

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


@pytest.mark.parametrize("cfg,N,n_iter,box", [("c1", 64, 50, None), ("c2", 150, 40, None),
                                              ("c3", 40, 30, None),
                                              ("c2", 77, 25, ((-0.3, -0.3), (10.3, 10.3)))],
                         ids=["c1", "c2", "c3", "c2 bounded"])
def test_residual_history_matches_oracle(P, cfg, N, n_iter, box):
    wl = W.CONFIGS[cfg]
    say(f"residual history {cfg} N={N} iters={n_iter} box={box is not None}")
    kw = {} if box is None else dict(s_min=box[0], s_max=box[1])
    gp = P.Problem.from_workload(wl, **kw)
    op = oracle_problem(wl, **kw)
    bc, obs = W.scene(wl, 0)
    xi = W.samples(wl, 6, n=N).astype(np.float32)
    xo, r, c1, h = gp.project_hist(t32(bc), t32(obs), t32(xi), n_iter)
    torch.cuda.synchronize()
    pr = O.project(op, bc, obs, xi.astype(np.float64), n_iter)
    hist = h.cpu().numpy().astype(np.float64)
    scale = max(1.0, float(pr.resid_hist.max()))
    np.testing.assert_allclose(hist, pr.resid_hist, atol=2e-3 * scale, rtol=2e-3)
    # the first entry is the residual of the input itself
    np.testing.assert_allclose(hist[0], O.residual(op, obs, xi.astype(np.float64)),
                               atol=1e-4 * scale, rtol=1e-4)
    # outputs equal priest_project's under the same (default) shape, bit for bit
    gp.set_tiling((4, 1, 0))
    xo2, r2, c12 = gp.project(t32(bc), t32(obs), t32(xi), n_iter)
    torch.cuda.synchronize()
    assert torch.equal(xo, xo2) and torch.equal(r, r2) and torch.equal(c1, c12)
    gp.close()


def test_residual_history_rejects_null(P):
    wl = W.C1
    gp = P.Problem.from_workload(wl)
    bc, obs = W.scene(wl, 0)
    xi = t32(W.samples(wl, 1, n=8))
    with pytest.raises(P.PriestError):
        P.priest_project_hist(gp.handle, t32(bc), t32(obs), xi, 5, torch.empty_like(xi), None, None,
                              None)
    gp.close()
