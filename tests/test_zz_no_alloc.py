"""priest_plan_static, the plan entry point that allocates nothing (its
workspace is the library's static device array), against priest_plan with a
caller workspace: the same kernels on the same tile shape, so every output
must agree bit for bit.  Two static calls in a row, the second one smaller,
so that the second runs on what the first left in the shared array."""
import sys

import numpy as np
import pytest
import torch

from paper_2309_08235_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t32(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32).to(DEV)


def test_plan_static_matches_plan(gpu_lib):
    from paper_2309_08235_amd import priest as P
    assert torch.cuda.is_available()
    base = W.with_changes(W.C2, n_proj_iters=30)
    bc, obs = W.scene(W.C2, 0)
    cases = [(1000, 3, True, 11), (300, 2, False, 12)]     # (N, n_cem, supplied noise, seed)
    for N, n_cem, use_noise, seed in cases:
        wl = W.with_changes(base, n_samples=N, n_proj=W.default_n_proj(N), n_elite=max(4, N // 10))
        say(f"priest_plan_static vs priest_plan, C2 scene, N={N}, n_cem={n_cem}, "
            f"noise={'supplied' if use_noise else 'philox'}")
        prob = P.Problem.from_workload(wl)
        prob.set_tiling((4, 1, 0))
        cem = P.Cem(n_samples=N, n_cem=n_cem, n_proj_iters=wl.n_proj_iters, n_proj=wl.n_proj,
                    n_elite=wl.n_elite, sigma=wl.sigma, gamma=wl.gamma, cov_jitter=wl.cov_jitter)
        noise = t32(W.standard_normals(seed, (n_cem, N, wl.D))) if use_noise else None
        mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
        mu_r, cov_r = t32(mu0), t32(cov0)
        ref = prob.plan(t32(bc), t32(obs), cem, mu_r, cov_r, seed=seed, stream_id=3, noise=noise)
        mu_s, cov_s = t32(mu0), t32(cov0)
        got = prob.plan_outputs(cem)
        P.priest_plan_static(prob.handle, t32(bc), t32(obs), cem.c(), mu_s, cov_s, seed, 3, noise,
                             got)
        torch.cuda.synchronize()
        assert int(got["status"][0]) == 0 and int(ref["status"][0]) == 0
        for k in ("best_xi", "best_cost", "elite_idx", "proj_idx", "xi", "xi_bar", "resid", "c1"):
            assert torch.equal(got[k], ref[k]), (N, k)
        assert torch.equal(mu_s, mu_r) and torch.equal(cov_s, cov_r), N
        assert np.isfinite(float(got["best_cost"][0]))
        prob.close()
