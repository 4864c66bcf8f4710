"""Every tile shape of the projection kernel (MFMA column packing, time blocks
per wave, persistent grid or sample groups drawn per wave) computes the same
arithmetic per sample, so results
must be bit-identical across shapes; the autotuner's pick is one of them.
The default shape is pinned to the oracle by test_gpu_parity.py; one shape
is also compared with the oracle here."""
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


CASES = [
    # (label, workload, changes, N)
    ("2d k100 m50", W.C2, {}, 301),
    ("2d k200 m20", W.C2, dict(n_steps=200, n_obs=20, horizon=20.0), 45),
    ("2d k10 m4", W.C1, dict(n_steps=10), 19),
    ("3d k100 m128", W.C3, {}, 101),
    ("3d k40 m0", W.C3, dict(n_steps=40, n_obs=0), 13),
    ("2d k50 m8 n1", W.C1, dict(n_obs=8), 1),
]


@pytest.mark.parametrize("label,wl,changes,N", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_projection_identical_across_tilings(P, label, wl, changes, N, precision):
    w = W.with_changes(wl, **changes)
    say(f"tilings: projection {label}, N={N}, precision={precision}")
    prob = P.Problem.from_workload(w, precision=precision, n_refine_fp32=3)
    bc, obs = W.scene(w, 0)
    xi = t32(W.samples(w, 11, n=N))
    bc_t, obs_t = t32(bc), t32(obs)
    cands = prob.tiling_candidates()
    assert cands[0] == (4, 1, 0)
    assert ((2, 1, 0) in cands) == (w.dims == 2)
    assert (8, 1, 0) in cands and (8, 1, 1) in cands
    outs = {}
    for c in cands:
        prob.set_tiling(c)
        xo, r, c1 = prob.project(bc_t, obs_t, xi, 12)
        torch.cuda.synchronize()
        assert prob.last_tiling() == (c, False)
        outs[c] = (xo.cpu().numpy(), r.cpu().numpy(), c1.cpu().numpy())
    ref = outs[cands[0]]
    for c, o in outs.items():
        for got, want in zip(o, ref):
            np.testing.assert_array_equal(got, want, err_msg=f"tiling {c}")
    prob.close()


NONFINITE = [
    # (label, workload, N, index of the sample made non-finite)
    ("3d k100 m128", W.C3, 37, 5),
    ("2d k100 m50", W.C2, 45, 9),
]


@pytest.mark.parametrize("label,wl,N,bad", NONFINITE, ids=[c[0] for c in NONFINITE])
def test_nonfinite_sample_leaves_the_others_unchanged(P, label, wl, N, bad):
    """A NaN coefficient in one sample: the samples that share its wave and
    tile get the same results, bit for bit, as without it (each sample's
    projection is independent of the others; with a NaN in the wave every
    skipping budget is NaN, so nothing is skipped, while the finite run
    skips), in every tile shape; the NaN sample's own result is not finite."""
    say(f"tilings: non-finite sample {bad} of {N}, {label}")
    prob = P.Problem.from_workload(wl)
    bc, obs = W.scene(wl, 0)
    xi = W.samples(wl, 13, n=N).astype(np.float32)
    xin = xi.copy()
    xin[bad, 3] = np.nan
    keep = np.arange(N) != bad
    for c in prob.tiling_candidates():
        prob.set_tiling(c)
        a = prob.project(t32(bc), t32(obs), t32(xi), 20)
        b = prob.project(t32(bc), t32(obs), t32(xin), 20)
        torch.cuda.synchronize()
        for want, got in zip(a, b):
            want, got = want.cpu().numpy(), got.cpu().numpy()
            np.testing.assert_array_equal(got[keep], want[keep], err_msg=f"tiling {c}")
        assert not np.all(np.isfinite(b[0].cpu().numpy()[bad])), f"tiling {c}"
    prob.close()


def test_packed_2d_tiling_matches_oracle(P):
    say("tilings: 8-samples-per-block shape vs the oracle (C2 scene, N=77)")
    w = W.C2
    prob = P.Problem.from_workload(w)
    op = oracle_problem(w)
    bc, obs = W.scene(w, 0)
    xi = W.samples(w, 3, n=77).astype(np.float32)
    prob.set_tiling((2, 2, 1))
    xo, _, _ = prob.project(t32(bc), t32(obs), t32(xi), 30)
    torch.cuda.synchronize()
    want = O.project(op, bc, obs, xi.astype(np.float64), 30).xi_bar
    check_projection(op, bc, obs, xi, xo.cpu().numpy().astype(np.float64), want, 30,
                     label="packed 2d")
    prob.close()


def test_plan_batch_identical_across_tilings_and_graphs(P):
    say("tilings: plan_batch of 3 problems under every shape, with graph replays")
    w = W.with_changes(W.C2, n_samples=150, n_proj=W.default_n_proj(150), n_elite=20,
                       n_proj_iters=15, n_cem=3)
    prob = P.Problem.from_workload(w)
    nP = 3
    scenes = [W.scene(W.C2, q) for q in range(nP)]
    bc = t32(np.stack([s[0] for s in scenes]))
    obs = t32(np.stack([s[1] for s in scenes]))
    mu0 = t32(np.stack([W.initial_mean(w)] * nP))
    cov0 = t32(np.stack([W.initial_cov(w)] * nP))
    cem = P.Cem(w.n_samples, w.n_cem, w.n_proj_iters, w.n_proj, w.n_elite)
    s = torch.cuda.Stream()
    results = {}
    for c in prob.tiling_candidates():
        prob.set_tiling(c)
        for graph in (False, True):
            for rep in range(2 if graph else 1):
                mu, cov = mu0.clone(), cov0.clone()
                with torch.cuda.stream(s):
                    out = prob.plan_batch(nP, bc, obs, cem, mu, cov, seed=5, use_graph=graph,
                                          stream=s)
                s.synchronize()
                results[(c, graph, rep)] = (out["best_xi"].cpu().numpy(),
                                            out["xi_bar"].cpu().numpy(), mu.cpu().numpy(),
                                            cov.cpu().numpy(), out["elite_idx"].cpu().numpy())
    ref = results[((4, 1, 0), False, 0)]
    for key, val in results.items():
        for got, want in zip(val, ref):
            np.testing.assert_array_equal(got, want, err_msg=str(key))
    prob.close()


def test_plan_with_noise_identical_across_tilings(P):
    """Supplied normals (the sampler's other input), 3D, a ragged last group
    of samples: every shape, including the whole-horizon ones whose waves
    draw and stage their own sample groups, gives the same plan bit for bit."""
    say("tilings: 3D plan with supplied normals under every shape")
    w = W.with_changes(W.C3, n_obs=24, n_steps=50, n_samples=150, n_proj=W.default_n_proj(150),
                       n_elite=20, n_proj_iters=12, n_cem=2)
    prob = P.Problem.from_workload(w)
    bc, obs = W.scene(w, 0)
    noise = t32(W.standard_normals(17, (w.n_cem, w.n_samples, w.D)))
    cem = P.Cem(w.n_samples, w.n_cem, w.n_proj_iters, w.n_proj, w.n_elite)
    results = {}
    for c in prob.tiling_candidates():
        prob.set_tiling(c)
        mu, cov = t32(W.initial_mean(w)), t32(W.initial_cov(w))
        out = prob.plan(t32(bc), t32(obs), cem, mu, cov, noise=noise)
        torch.cuda.synchronize()
        results[c] = (out["best_xi"].cpu().numpy(), out["xi_bar"].cpu().numpy(),
                      mu.cpu().numpy(), cov.cpu().numpy())
    ref = results[(4, 1, 0)]
    for c, val in results.items():
        for got, want in zip(val, ref):
            np.testing.assert_array_equal(got, want, err_msg=f"tiling {c}")
    prob.close()


def test_autotuner_picks_a_candidate_and_keeps_results(P):
    say("tilings: autotuned projection equals the default shape")
    w = W.C2
    prob = P.Problem.from_workload(w)
    bc, obs = W.scene(w, 0)
    xi = t32(W.samples(w, 4, n=500))
    prob.set_tiling((4, 1, 0))
    ref = prob.project(t32(bc), t32(obs), xi, 20)[0].cpu().numpy()
    prob.set_tiling(None)
    xo = prob.project(t32(bc), t32(obs), xi, 20)[0]
    torch.cuda.synchronize()
    shape, tuned = prob.last_tiling()
    assert tuned and shape in prob.tiling_candidates()
    np.testing.assert_array_equal(xo.cpu().numpy(), ref)
    # the second call reuses the cached pick
    xo2 = prob.project(t32(bc), t32(obs), xi, 20)[0]
    torch.cuda.synchronize()
    assert prob.last_tiling() == (shape, True)
    np.testing.assert_array_equal(xo2.cpu().numpy(), ref)
    # in-place projection (xi_in aliases xi_out) on a fresh shape key
    xi2 = t32(W.samples(w, 4, n=333))
    want = prob.project(t32(bc), t32(obs), xi2.clone(), 20)[0].cpu().numpy()
    P.priest_project(prob.handle, t32(bc), t32(obs), xi2, 20, xi2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(xi2.cpu().numpy(), want)
    prob.close()


def test_set_tiling_rejects_non_candidates(P):
    prob = P.Problem.from_workload(W.C3)
    for bad in [(2, 1, 0), (3, 1, 0), (4, 3, 0), (4, 1, 2), (8, 2, 0), (16, 1, 0), (2, 0, 0),
                (8, 0, 0), (4, -1, 0)]:
        with pytest.raises(P.PriestError):
            prob.set_tiling(bad)
    assert (4, 0, 0) in prob.tiling_candidates() and (4, 0, 1) in prob.tiling_candidates()
    prob.close()
    # the whole-horizon shape holds at most 8 time blocks (n_steps <= 128)
    long = P.Problem.from_workload(W.with_changes(W.C2, n_steps=129, horizon=20.0))
    assert all(c[1] != 0 for c in long.tiling_candidates())
    with pytest.raises(P.PriestError):
        long.set_tiling((2, 0, 0))
    long.close()


def test_whole_horizon_shape_matches_oracle(P):
    """The whole-horizon shape (one wave per sample group over every time
    block) against the oracle directly, 3D and 2D, with a ragged last group."""
    for wl, n, shape in ((W.with_changes(W.C3, n_obs=40), 37, (4, 0, 0)),
                         (W.C2, 45, (2, 0, 1))):
        say(f"tilings: whole-horizon shape {shape} vs the oracle ({wl.name}, N={n})")
        prob = P.Problem.from_workload(wl)
        op = oracle_problem(wl)
        bc, obs = W.scene(wl, 0)
        xi = W.samples(wl, 8, n=n).astype(np.float32)
        prob.set_tiling(shape)
        xo, r, c1 = prob.project(t32(bc), t32(obs), t32(xi), 25)
        torch.cuda.synchronize()
        assert prob.last_tiling() == (shape, False)
        pr = O.project(op, bc, obs, xi.astype(np.float64), 25)
        check_projection(op, bc, obs, xi, xo.cpu().numpy().astype(np.float64), pr.xi_bar, 25,
                         label=f"whole horizon {wl.name}")
        np.testing.assert_allclose(r.cpu().numpy(), pr.resid, atol=2e-3 * max(1, pr.resid.max()))
        prob.close()
