"""Edge cases of the HIP path against the oracle: coefficient counts around
the k-chunk boundary (n_coeff 4..16), the smallest and largest step counts,
obstacle counts that spill the candidate masks to LDS, the largest sample
count, and degenerate plans."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2309_08235_amd import workloads as W
from tests.parity import check_projection, oracle_problem
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


def _case(P, wl, N, n_iter, idx=None, seed=3, label=""):
    gp = P.Problem.from_workload(wl)
    op = oracle_problem(wl)
    bc, obs = W.scene(wl, 1)
    xi = W.samples(wl, seed, n=N).astype(np.float32)
    xo, r, _ = gp.project(t32(bc), t32(obs), t32(xi), n_iter)
    torch.cuda.synchronize()
    idx = np.arange(N) if idx is None else idx
    pr = O.project(op, bc, obs, xi[idx].astype(np.float64), n_iter)
    err = check_projection(op, bc, obs, xi[idx], np64(xo)[idx], pr.xi_bar, n_iter, label=label)
    np.testing.assert_allclose(np64(r)[idx], pr.resid, atol=2e-3 * max(1.0, pr.resid.max()))
    gp.close()
    return err


@pytest.mark.parametrize("dims,nc", [(2, 5), (2, 8), (2, 12), (2, 13), (2, 16), (3, 16)])
def test_coefficient_counts(P, dims, nc):
    say(f"edges: dims={dims} n_coeff={nc}")
    base = W.with_changes(W.C1, bc_mask=W.BC_DEFAULT) if dims == 2 else W.with_changes(W.C3, n_obs=16)
    wl = W.with_changes(base, n_coeff=nc, n_steps=40)
    err = _case(P, wl, 21, 30, label=f"n_coeff {nc}")
    assert np.median(err) < 1e-4


def test_coefficient_count_16_identical_across_tilings(P):
    say("edges: n_coeff=16 under every tile shape")
    wl = W.with_changes(W.C2, n_coeff=16, n_steps=60)
    gp = P.Problem.from_workload(wl)
    bc, obs = W.scene(wl, 0)
    xi = t32(W.samples(wl, 2, n=50))
    ref = None
    for c in gp.tiling_candidates():
        gp.set_tiling(c)
        out = [np64(v) for v in gp.project(t32(bc), t32(obs), xi, 15)]
        if ref is None:
            ref = out
        for got, want in zip(out, ref):
            np.testing.assert_array_equal(got, want, err_msg=str(c))
    gp.close()


@pytest.mark.parametrize("K", [2, 17, 256])
def test_step_counts(P, K):
    say(f"edges: n_steps={K}")
    wl = W.with_changes(W.C1, n_steps=K, horizon=10.0 if K > 2 else 3.0)
    _case(P, wl, 9, 20, label=f"K {K}")


@pytest.mark.parametrize("dims,M", [(2, 300), (3, 200)])
def test_obstacle_masks_beyond_registers(P, dims, M):
    """More than 128 obstacles: the candidate masks of groups 2.. live in LDS."""
    say(f"edges: dims={dims} n_obs={M}")
    base = W.C2 if dims == 2 else W.C3
    wl = W.with_changes(base, n_obs=M, n_steps=50)
    err = _case(P, wl, 40, 25, label=f"M {M}")
    assert np.median(err) < 1e-4


def test_largest_sample_count_sampled(P):
    say("edges: N = 65536 (sampled against the oracle)")
    wl = W.with_changes(W.C2, n_steps=40, n_obs=20)
    idx = np.random.default_rng(5).choice(65536, 12, replace=False)
    _case(P, wl, 65536, 15, idx=idx, label="N 65536")


@pytest.mark.parametrize("N,n_proj,n_elite", [(1, 1, 1), (7, 3, 1), (64, 64, 64)])
def test_degenerate_plans(P, N, n_proj, n_elite):
    say(f"edges: plan N={N} n_proj={n_proj} n_elite={n_elite}")
    wl = W.with_changes(W.C1, n_samples=N, n_proj=n_proj, n_elite=n_elite, n_proj_iters=20)
    gp = P.Problem.from_workload(wl)
    op = oracle_problem(wl)
    bc, obs = W.scene(wl, 0)
    cem = _cem(wl)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    noise = W.standard_normals(9, (1, N, wl.D))
    mu, cov = t32(mu0), t32(cov0)
    out = gp.plan(t32(bc), t32(obs), cem, mu, cov, noise=t32(noise),
                  out=gp.plan_outputs(cem, 1, full=True))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, obs, wl, cem, mu0, cov0, noise[0], out, np64(mu), np64(cov),
                    f"N {N}")
    gp.close()
