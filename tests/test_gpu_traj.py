"""Obstacles given by their paths (positions at every time stamp, the stacked
obstacle positions of eq. (13)) on the GPU, against the oracle."""
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


CASES = [
    ("2d velocity paths", W.with_changes(W.C2, n_proj_iters=60), 0.0, 300),
    ("2d curved paths", W.with_changes(W.C2, n_proj_iters=60), 1.2, 300),
    ("3d curved paths", W.with_changes(W.C3, n_obs=40, n_proj_iters=30), 1.0, 60),
]


@pytest.mark.parametrize("label,wl,swirl,N", CASES, ids=[c[0] for c in CASES])
def test_path_projection_matches_oracle(P, label, wl, swirl, N):
    say(f"obstacle paths: projection {label} N={N}")
    gp = P.Problem.from_workload(wl, obs_model=P.OBS_PATH)
    op = oracle_problem(wl, obs_model=1)
    bc, obs = W.scene(wl, 0)
    if wl.dims == 3:
        obs[:, 3:6] = np.random.default_rng(2).uniform(-0.3, 0.3, (wl.n_obs, 3))
    path = W.trajectory_obstacles(wl, obs, swirl=swirl, seed=5)
    xi = W.samples(wl, 7, n=N).astype(np.float32)
    xo, r, c1 = gp.project(t32(bc), t32(path), t32(xi), wl.n_proj_iters)
    torch.cuda.synchronize()
    idx = np.random.default_rng(3).choice(N, min(N, 40), replace=False)
    pr = O.project(op, bc, path, xi[idx].astype(np.float64), wl.n_proj_iters)
    err = check_projection(op, bc, path, xi[idx], np64(xo)[idx], pr.xi_bar, wl.n_proj_iters,
                           label=label)
    assert np.median(err) < 1e-4
    np.testing.assert_allclose(np64(r)[idx], pr.resid, atol=2e-3 * max(1.0, pr.resid.max()))
    assert gp.last_tiling()[0] == (4, 1, 0)
    gp.close()


def test_velocity_paths_agree_with_the_velocity_model(P):
    say("obstacle paths from constant velocities vs the velocity rows")
    wl = W.with_changes(W.C2, n_proj_iters=40)
    bc, obs = W.scene(wl, 1)
    path = W.trajectory_obstacles(wl, obs)
    xi = t32(W.samples(wl, 8, n=200))
    gv = P.Problem.from_workload(wl)
    gt = P.Problem.from_workload(wl, obs_model=P.OBS_PATH)
    gv.set_tiling((4, 1, 0))
    xv, rv, _ = gv.project(t32(bc), t32(obs), xi, wl.n_proj_iters)
    xt_, rt_, _ = gt.project(t32(bc), t32(path), xi, wl.n_proj_iters)
    torch.cuda.synchronize()
    scale = max(1.0, float(xv.abs().max()))
    np.testing.assert_allclose(np64(xt_), np64(xv), atol=2e-3 * scale)
    np.testing.assert_allclose(np64(rt_), np64(rv), atol=2e-3 * max(1.0, float(rv.max())))
    gv.close()
    gt.close()


def test_path_offsets_and_plan_step_match_oracle(P):
    say("obstacle paths: push-out offsets and one CEM step")
    wl = W.with_changes(W.C1, n_obs=4)
    gp = P.Problem.from_workload(wl, obs_model=P.OBS_PATH)
    op = oracle_problem(wl, obs_model=1)
    bc, obs = W.scene(wl, 2)
    obs[:, 3:5] = np.random.default_rng(4).uniform(-0.3, 0.3, (wl.n_obs, 2))
    path = W.trajectory_obstacles(wl, obs, swirl=0.8, seed=2)
    xi = W.samples(wl, 11, n=6).astype(np.float32)
    got = np64(gp.offsets(t32(bc), t32(path), t32(xi)))
    xi64 = xi.astype(np.float64)
    want = O.targets(op, path, xi64) - xi64 @ op.F().T
    want = want.reshape(6, wl.dims, wl.n_obs + 2, wl.n_steps).transpose(0, 2, 3, 1)
    np.testing.assert_allclose(got, want, atol=2e-4 * max(1.0, np.abs(want).max()))
    cem = _cem(wl)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    noise = W.standard_normals(13, (1, wl.n_samples, wl.D))
    mu, cov = t32(mu0), t32(cov0)
    out = gp.plan(t32(bc), t32(path), cem, mu, cov, noise=t32(noise),
                  out=gp.plan_outputs(cem, 1, full=True))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, path, wl, cem, mu0, cov0, noise[0], out, np64(mu), np64(cov),
                    "paths c1")
    gp.close()


def test_path_problems_keep_the_default_shape_and_skip_the_unfused_form(P):
    wl = W.C1
    gp = P.Problem.from_workload(wl, obs_model=P.OBS_PATH)
    with pytest.raises(P.PriestError):
        gp.set_tiling((2, 1, 0))
    gp.set_tiling((4, 1, 0))
    bc, obs = W.scene(wl, 0)
    path = W.trajectory_obstacles(wl, obs)
    with pytest.raises(P.PriestError):
        gp.project_unfused(t32(bc), t32(path), t32(W.samples(wl, 1, n=4)), 5)
    gp.close()
