"""The profiling hooks used by the benchmark: launch timing and the count of
evaluated (sample, step, obstacle) pairs, checked on scenes where the count
is known exactly."""
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


@pytest.fixture(scope="module")
def P(gpu_lib):
    from paper_2309_08235_amd import priest
    assert torch.cuda.is_available()
    return priest


def _count(P, prob, bc, obs, xi, n_iter):
    P.priest_profile_count_pairs(True)
    prob.project(t32(bc), t32(obs), t32(xi), n_iter)
    n = P.priest_profile_read_pairs()
    P.priest_profile_count_pairs(False)
    return n


@pytest.mark.parametrize("wl,N", [(W.C1, 37), (W.with_changes(W.C2, n_obs=2), 100),
                                  (W.with_changes(W.C3, n_obs=2), 21)],
                         ids=["2d k50", "2d k100", "3d k100"])
def test_pair_count_exact_when_obstacles_cover_or_avoid_everything(P, wl, N):
    say(f"pair counter: {wl.name} N={N}")
    n_iter = 7
    bc, obs = W.scene(wl, 0)
    xi = W.samples(wl, 2, n=N)
    # far away: never a candidate
    far = obs.copy()
    far[:, :3] = 1e4
    far[:, 3:6] = 0.0
    far[:, 6:8] = 0.5
    prob = P.Problem.from_workload(wl)
    assert _count(P, prob, bc, far, xi, n_iter) == 0
    # huge, with its surface about 20 m beyond the scene: never touched (no
    # push-out moves the items) but always within the candidate radius
    big = far.copy()
    big[:, :3] = 5.0
    big[:, 0] = 1025.0
    big[:, 6:8] = 1e3
    per_pass = N * wl.n_steps * wl.n_obs
    want = per_pass * (n_iter + 1)
    for c in prob.tiling_candidates():
        prob.set_tiling(c)
        n = _count(P, prob, bc, big, xi, n_iter)
        if c[1] != 0:
            # time-split shapes evaluate every candidate pair on every pass
            assert n == want, c
        else:
            # the whole-horizon shape evaluates a block's positions on the
            # first pass, the final pass, and when its position budget (the
            # items' clearance to the candidates, here about 15 m) runs out;
            # every evaluation covers all M candidates of the block's items
            assert 2 * per_pass <= n <= want and n % wl.n_obs == 0, (c, n, want)
    # bounded by the brute-force count on the real scene (which may cull
    # every pair); off means no count
    prob.set_tiling(None)
    n = _count(P, prob, bc, obs, xi, n_iter)
    assert 0 <= n <= want
    prob.project(t32(bc), t32(obs), t32(xi), n_iter)
    torch.cuda.synchronize()
    assert P.priest_profile_read_pairs() == 0
    prob.close()


def test_profile_timing_counts_launches(P):
    say("profile timing: launches of one plan")
    wl = W.with_changes(W.C1, n_proj_iters=10)
    prob = P.Problem.from_workload(wl)
    bc, obs = W.scene(wl, 0)
    cem = P.Cem(wl.n_samples, 4, wl.n_proj_iters, wl.n_proj, wl.n_elite)
    mu, cov = t32(W.initial_mean(wl)), t32(W.initial_cov(wl))
    prob.plan(t32(bc), t32(obs), cem, mu, cov)        # tunes outside the profiled region
    torch.cuda.synchronize()
    P.priest_profile_read()
    P.priest_profile_enable(True)
    prob.plan(t32(bc), t32(obs), cem, mu, cov)
    P.priest_profile_enable(False)
    n, ms = P.priest_profile_read()
    assert n == 4 and ms > 0.0
    prob.close()
