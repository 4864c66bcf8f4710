"""Workspace bounds (Appendix, G xi <= tau) on the GPU through the C ABI:
fused and unfused projections and one CEM step against the oracle, and
bit-identity of the fused kernel across tile shapes."""
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

BOXES = {
    "c1": ((-0.2, -0.2), (10.2, 10.2)),
    "c2": ((-0.3, -0.3), (10.3, 10.3)),
    "c3": ((3.5, 3.5, 3.5), (16.5, 16.5, 16.5)),
}


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


def _pair(P, wl, cfg, **kw):
    lo, hi = BOXES[cfg]
    return (P.Problem.from_workload(wl, s_min=lo, s_max=hi, **kw),
            oracle_problem(wl, s_min=lo, s_max=hi))


def _positions(op, xb):
    N = xb.shape[0]
    return np.einsum('kc,nac->nak', op.P, xb.reshape(N, op.dims, op.n_coeff))


@pytest.mark.parametrize("cfg,N,n_iter,sampled", [("c1", 64, 50, None), ("c2", 1000, 100, 30),
                                                  ("c3", 200, 40, 12)])
def test_bounded_projection_matches_oracle(P, cfg, N, n_iter, sampled):
    wl = W.CONFIGS[cfg]
    say(f"bounded projection {cfg} N={N} iters={n_iter}")
    gp, op = _pair(P, wl, cfg)
    bc, obs = W.scene(wl, 0)
    xi = W.samples(wl, 9, n=N).astype(np.float32)
    xo, r, c1 = gp.project(t32(bc), t32(obs), t32(xi), n_iter)
    torch.cuda.synchronize()
    idx = np.arange(N) if sampled is None else np.random.default_rng(4).choice(N, sampled, replace=False)
    pr = O.project(op, bc, obs, xi[idx].astype(np.float64), n_iter)
    got = np64(xo)[idx]
    err = check_projection(op, bc, obs, xi[idx], got, pr.xi_bar, n_iter, label=f"bounded {cfg}")
    assert np.median(err) < 1e-4
    np.testing.assert_allclose(np64(r)[idx], pr.resid, atol=2e-3 * max(1.0, pr.resid.max()))
    # the box is really used: the same samples projected without it differ
    free = O.project(oracle_problem(wl), bc, obs, xi[idx[:4]].astype(np.float64), n_iter).xi_bar
    assert np.abs(free - pr.xi_bar[:4]).max() > 1e-2
    gp.close()


def test_bounded_unfused_matches_fused_and_oracle(P):
    say("bounded unfused projection c2 N=150 vs oracle and fused")
    wl = W.C2
    gp, op = _pair(P, wl, "c2")
    bc, obs = W.scene(wl, 1)
    xi = W.samples(wl, 3, n=150).astype(np.float32)
    xu, ru, cu = gp.project_unfused(t32(bc), t32(obs), t32(xi), 40)
    xf, rf, cf = gp.project(t32(bc), t32(obs), t32(xi), 40)
    torch.cuda.synchronize()
    pr = O.project(op, bc, obs, xi.astype(np.float64), 40)
    check_projection(op, bc, obs, xi, np64(xu), pr.xi_bar, 40, label="bounded unfused")
    np.testing.assert_allclose(np64(ru), pr.resid, atol=2e-3 * max(1.0, pr.resid.max()))
    np.testing.assert_allclose(np64(xu), np64(xf), atol=2e-3 * max(1.0, np.abs(pr.xi_bar).max()))
    gp.close()


@pytest.mark.parametrize("cfg,N", [("c2", 301), ("c3", 61)])
def test_bounded_projection_identical_across_tilings(P, cfg, N):
    wl = W.CONFIGS[cfg]
    say(f"bounded projection {cfg} N={N}: every tile shape")
    gp, _ = _pair(P, wl, cfg)
    bc, obs = W.scene(wl, 2)
    xi = t32(W.samples(wl, 5, n=N))
    ref = None
    for c in gp.tiling_candidates():
        gp.set_tiling(c)
        out = [np64(v) for v in gp.project(t32(bc), t32(obs), xi, 25)]
        if ref is None:
            ref = out
        for got, want in zip(out, ref):
            np.testing.assert_array_equal(got, want, err_msg=str(c))
    gp.close()


def test_bounded_projection_reaches_the_box(P):
    """Bounds only (no obstacles, no velocity/acceleration limits): after
    enough iterations every position is inside the box up to FP32 rounding."""
    say("bounded projection, box only, 400 iterations")
    wl = W.with_changes(W.C1, n_obs=0, v_max=np.inf, a_max=np.inf)
    gp, op = _pair(P, wl, "c1")
    bc, obs = W.scene(wl, 0)
    obs = obs[:0]
    xi = W.samples(wl, 8, n=64).astype(np.float32)
    xo, r, _ = gp.project(t32(bc), t32(np.zeros((1, 8))), t32(xi), 400)
    torch.cuda.synchronize()
    p = _positions(op, np64(xo))
    lo, hi = BOXES["c1"]
    assert p.min(axis=(0, 2))[0] >= lo[0] - 1e-3 and p.max(axis=(0, 2))[0] <= hi[0] + 1e-3
    assert p.min(axis=(0, 2))[1] >= lo[1] - 1e-3 and p.max(axis=(0, 2))[1] <= hi[1] + 1e-3
    assert np64(r).max() < 1e-2
    gp.close()


def test_bounded_plan_step_matches_oracle(P):
    say("bounded plan c1, one CEM iteration, supplied noise")
    wl = W.C1
    gp, op = _pair(P, wl, "c1")
    bc, obs = W.scene(wl, 0)
    cem = _cem(wl)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    noise = W.standard_normals(31, (1, wl.n_samples, wl.D))
    mu, cov = t32(mu0), t32(cov0)
    out = gp.plan(t32(bc), t32(obs), cem, mu, cov, noise=t32(noise))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, obs, wl, cem, mu0, cov0, noise[0], out, np64(mu), np64(cov),
                    "bounded c1")
    gp.close()
