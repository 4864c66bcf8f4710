"""GPU-vs-oracle parity of the HIP path, called through the C ABI.

Each case prints (and flushes) what it runs before touching the GPU."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2309_08235_amd import workloads as W
from tests.parity import check_projection, check_selection, oracle_problem, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t32(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(DEV)


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def priest(gpu_lib):
    from paper_2309_08235_amd import priest as P
    assert torch.cuda.is_available()
    return P


def make(priest, wl, **kw):
    return priest.Problem.from_workload(wl, **kw), oracle_problem(wl, **kw)


# ---------------------------------------------------------------------------
# one-time FP64 KKT factorisation and basis rows
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cfg", ["c1", "c2", "c3"])
def test_kkt_constants_match_fp64_inverse(priest, cfg):
    wl = W.CONFIGS[cfg]
    say(f"kkt constants {cfg}")
    gp, op = make(priest, wl)
    c = gp.constants()
    P, Pd, Pdd = op.P, op.Pd, op.Pdd
    Q = np.eye(wl.n_coeff) + op.rho * (op.n_obs * P.T @ P + Pd.T @ Pd + Pdd.T @ Pdd)
    A = op.A_axis()
    E = A.shape[0]
    kkt = np.block([[Q, A.T], [A, np.zeros((E, E))]])
    inv = np.linalg.inv(kkt)
    M11 = inv[:wl.n_coeff, :wl.n_coeff]
    M12 = inv[:wl.n_coeff, wl.n_coeff:]
    np.testing.assert_allclose(c["M11"], M11, rtol=1e-5, atol=1e-6 * np.abs(M11).max())
    np.testing.assert_allclose(c["Pi"], M11 @ Q, rtol=1e-5, atol=1e-6 * np.abs(M11 @ Q).max())
    M12full = np.zeros((wl.n_coeff, 6))
    M12full[:, op.boundary_rows()] = M12
    np.testing.assert_allclose(c["M12"], M12full, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(c["W"][:, 0], P, atol=1e-6)
    np.testing.assert_allclose(c["W"][:, 1], Pd, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(c["W"][:, 2], Pdd, rtol=1e-5, atol=1e-5)
    gp.close()


def test_singular_boundary_rows_rejected(priest):
    say("singular boundary rows")
    with pytest.raises(priest.PriestError) as ei:
        priest.Problem(dims=2, n_coeff=3, n_steps=10, horizon=2.0, n_obs=1,
                       bc_mask=priest.BC_DEFAULT)
    assert ei.value.code == priest.PRIEST_ERR_SINGULAR


# ---------------------------------------------------------------------------
# closed-form alpha / beta / d step, per row
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cfg", ["c1", "c2", "c3"])
def test_offsets_match_oracle_targets(priest, cfg):
    wl = W.CONFIGS[cfg]
    say(f"offsets {cfg}")
    gp, op = make(priest, wl)
    bc, obs = W.scene(wl, 4)
    xi = W.samples(wl, 11, n=6).astype(np.float32)
    got = np64(gp.offsets(t32(bc), t32(obs), t32(xi)))            # [N][M+2][K][dims]
    xi64 = xi.astype(np.float64)
    want = O.targets(op, obs, xi64) - xi64 @ op.F().T              # [N][dims*(M+2)*K]
    want = want.reshape(6, wl.dims, wl.n_obs + 2, wl.n_steps).transpose(0, 2, 3, 1)
    np.testing.assert_allclose(got, want, atol=2e-4 * max(1.0, np.abs(want).max()))
    gp.close()


def test_offsets_zero_offset_canonical_direction(priest):
    say("offsets zero offset")
    for dims in (2, 3):
        wl = W.with_changes(W.C1, dims=dims, n_obs=1, n_steps=5, start=(0.0, 0.0, 0.0),
                            goal=(5.0, 5.0, 5.0), bc_mask=W.BC_DEFAULT)
        gp, op = make(priest, wl)
        obs = np.zeros((1, 8)); obs[0, :dims] = 1.5; obs[0, 6] = 0.4; obs[0, 7] = 0.7
        xi = np.zeros((1, dims, 11), np.float32); xi[0, :, :] = 1.5    # p(t0) == centre exactly
        got = np64(gp.offsets(t32(W.boundary_values(wl)), t32(obs), t32(xi.reshape(1, -1))))
        want = np.zeros(dims); want[0 if dims == 2 else 2] = 0.4 if dims == 2 else 0.7
        np.testing.assert_allclose(got[0, 0, 0], want, atol=1e-7)
        gp.close()


@pytest.mark.parametrize("dims", [2, 3])
def test_projection_zero_offset(priest, dims):
    """An item exactly at an obstacle's centre (step 0) gets the canonical
    push-out of the full semi-axis inside the fused projection too (not only
    in the offsets kernel), as in the oracle: a push-out that came out short
    moves one projection step by about 10% here."""
    say(f"projection with an exactly zero offset, {dims}D")
    wl = W.with_changes(W.C1, dims=dims, n_obs=1, n_steps=5, start=(0.0, 0.0, 0.0),
                        goal=(5.0, 5.0, 5.0), bc_mask=W.BC_DEFAULT)
    gp, op = make(priest, wl)
    obs = np.zeros((1, 8)); obs[0, :dims] = 1.5; obs[0, 6] = 0.4; obs[0, 7] = 0.7
    xi = np.full((1, dims * 11), 1.5, np.float32)                  # p(t0) == centre exactly
    bc = W.boundary_values(wl)
    for n_iter in (1, 5):
        xo, _, _ = gp.project(t32(bc), t32(obs), t32(xi), n_iter)
        want = O.project(op, bc, obs, xi.astype(np.float64), n_iter).xi_bar
        err = rel_err(np64(xo), want)
        assert err.max() < 1e-3, (n_iter, err)
    gp.close()


@pytest.mark.parametrize("dims", [2, 3])
def test_residual_zero_offset_every_step(priest, dims):
    """n_iter = 0 on the zero trajectory with an obstacle centred at the
    origin: every step's offset is exactly zero (all coefficients are zero,
    so every product and sum is an exact zero; a constant trajectory at 1.5
    would leave rounding residues of the partition of unity instead), so the
    final pass takes the canonical push-out at all K steps and
    r = sqrt(K) * (canonical semi-axis): a in 2D (+x), b in 3D (+z), as in the
    oracle.  No velocity or acceleration violation (v = a = 0)."""
    say(f"residual of a trajectory at an obstacle's centre, n_iter = 0, {dims}D")
    K = 7
    wl = W.with_changes(W.C1, dims=dims, n_obs=1, n_steps=K, start=(0.0, 0.0, 0.0),
                        goal=(5.0, 5.0, 5.0), bc_mask=W.BC_DEFAULT)
    gp, op = make(priest, wl)
    obs = np.zeros((1, 8)); obs[0, 6] = 0.4; obs[0, 7] = 0.7
    xi = np.zeros((3, dims * 11), np.float32)
    bc = W.boundary_values(wl)
    xo, r, _ = gp.project(t32(bc), t32(obs), t32(xi), 0)
    torch.cuda.synchronize()
    semi = 0.4 if dims == 2 else 0.7
    want = O.residual(op, obs, xi.astype(np.float64))
    np.testing.assert_allclose(want, semi * math.sqrt(K), rtol=1e-12)
    np.testing.assert_allclose(np64(r), want, rtol=2e-6)
    np.testing.assert_array_equal(np64(xo), xi.astype(np.float64))
    gp.close()


# ---------------------------------------------------------------------------
# counter-based draws
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,stream,it,n,D", [(0, 0, 0, 300, 22), (2 ** 40 + 17, 5, 19, 257, 33)])
def test_normals_match_oracle(priest, seed, stream, it, n, D):
    say(f"normals seed={seed} stream={stream}")
    z = torch.empty((n, D), device=DEV)
    priest.priest_debug_normals(seed, stream, it, z)
    want = O.normals(seed, stream, it, n, D)
    np.testing.assert_allclose(np64(z), want, atol=3e-5, rtol=1e-5)


# ---------------------------------------------------------------------------
# projection
# ---------------------------------------------------------------------------
def _project_case(priest, wl, n_gpu, idx, seed=5, n_iter=None, scene=0, **kw):
    gp, op = make(priest, wl, **kw)
    bc, obs = W.scene(wl, scene)
    n_iter = wl.n_proj_iters if n_iter is None else n_iter
    xi = W.samples(wl, seed, n=n_gpu).astype(np.float32)
    xo, r, c1 = gp.project(t32(bc), t32(obs), t32(xi), n_iter)
    torch.cuda.synchronize()
    got, gr, gc = np64(xo), np64(r), np64(c1)
    pr = O.project(op, bc, obs, xi[idx].astype(np.float64), n_iter)
    err = check_projection(op, bc, obs, xi[idx], got[idx], pr.xi_bar, n_iter, label=wl.name)
    want_c1 = O.smoothness_cost(op, pr.xi_bar)
    gp.close()
    return err, got, gr, gc, pr, want_c1


def test_project_c1_full(priest):
    say("project c1 full batch (64 samples, 50 iterations)")
    idx = np.arange(64)
    err, got, gr, gc, pr, want_c1 = _project_case(priest, W.C1, 64, idx)
    assert np.median(err) < 1e-4
    np.testing.assert_allclose(gr, pr.resid, atol=2e-3 * max(1, pr.resid.max()))
    np.testing.assert_allclose(gc, want_c1, rtol=2e-3, atol=1e-3)


def test_project_c2_full_size_sampled(priest):
    """Paper-scale shape (N=1000, M=50 incl. moving obstacles, K=100, 100
    iterations) in the launch configuration of the benchmark; the oracle
    checks a sampled subset, element by element."""
    say("project c2 N=1000, oracle on 40 sampled samples")
    idx = np.random.default_rng(1).choice(1000, 40, replace=False)
    err, got, gr, gc, pr, want_c1 = _project_case(priest, W.C2, 1000, idx)
    assert np.median(err) < 1e-4
    np.testing.assert_allclose(gr[idx], pr.resid, atol=2e-3 * max(1, pr.resid.max()))
    np.testing.assert_allclose(gc[idx], want_c1, rtol=2e-3, atol=1e-3)
    assert np.all(np.isfinite(got))


def test_project_c3_shape_sampled(priest):
    say("project c3 3D N=2000 M=128, oracle on 16 sampled samples")
    idx = np.random.default_rng(2).choice(2000, 16, replace=False)
    err, got, gr, gc, pr, want_c1 = _project_case(priest, W.C3, 2000, idx, n_iter=60)
    assert np.median(err) < 1e-4
    np.testing.assert_allclose(gr[idx], pr.resid, atol=2e-3 * max(1, pr.resid.max()))


def test_project_c3_full_batch_100_iterations(priest):
    """The 3D batched workload at its configured size: 64 problems (distinct
    scenes) x 2000 samples, M = 128 spheres, K = 100, 100 projection
    iterations, in one priest_project_batch launch with the autotuned tile
    shape (the launch the benchmark's batched plans make); the oracle checks
    16 samples from each of 4 problems spread over the batch, element by
    element, with their residual and smoothness cost."""
    wl = W.C3
    P_, N = wl.n_problems, wl.n_samples
    say(f"project_batch c3 {P_} problems x {N} samples, 100 iterations, oracle on 4 x 16 samples")
    gp, op = make(priest, wl)
    scenes = [W.scene(wl, q) for q in range(P_)]
    bc = np.stack([s[0] for s in scenes])
    obs = np.stack([s[1] for s in scenes])
    xi = np.stack([W.samples(wl, 500 + q, n=N) for q in range(P_)]).astype(np.float32)
    xo, r, c1 = gp.project_batch(t32(bc), t32(obs), t32(xi), wl.n_proj_iters)
    torch.cuda.synchronize()
    got, gr, gc = np64(xo), np64(r), np64(c1)
    assert np.all(np.isfinite(got)) and np.all(np.isfinite(gr)) and np.all(np.isfinite(gc))
    counts = {}
    rng = np.random.default_rng(3)
    for q in (0, 21, 42, 63):
        idx = rng.choice(N, 16, replace=False)
        pr = O.project(op, bc[q], obs[q], xi[q, idx].astype(np.float64), wl.n_proj_iters)
        err = check_projection(op, bc[q], obs[q], xi[q, idx], got[q, idx], pr.xi_bar,
                               wl.n_proj_iters, label=f"c3 batch problem {q}", counts=counts)
        assert np.median(err) < 1e-4, (q, np.median(err))
        np.testing.assert_allclose(gr[q, idx], pr.resid, atol=2e-3 * max(1, pr.resid.max()))
        want_c1 = O.smoothness_cost(op, pr.xi_bar)
        np.testing.assert_allclose(gc[q, idx], want_c1, rtol=2e-3, atol=1e-3)
    say(f"c3 batch: {counts['sensitive']} of {counts['checked']} checked samples above the "
        f"tolerance (each shown sensitive)")
    gp.close()


def test_plan_batch_c3_shared_counter_against_oracle(priest):
    """The benchmark's batched plans at their configured size (64 problems x
    2000 samples, M = 128, K = 100, 100 projection iterations), one CEM
    iteration through priest_plan_batch with the whole-horizon shape whose
    waves draw (problem, group) pairs from one counter for the whole launch
    (obstacle records read from the plan workspace): the oracle projects 16
    of the drawn samples of each of 4 problems, and the plan's projected
    samples, residuals and costs must match them."""
    wl = W.C3
    P_, N = wl.n_problems, wl.n_samples
    say(f"plan_batch c3 {P_} x {N}, shared counter, oracle on 4 x 16 samples")
    gp, op = make(priest, wl)
    gp.set_tiling((4, 0, 1))
    scenes = [W.scene(wl, q) for q in range(P_)]
    bc = np.stack([s[0] for s in scenes])
    obs = np.stack([s[1] for s in scenes])
    cem = priest.Cem(n_samples=N, n_cem=1, n_proj_iters=wl.n_proj_iters, n_proj=wl.n_proj,
                     n_elite=wl.n_elite, sigma=wl.sigma, gamma=wl.gamma, cov_jitter=wl.cov_jitter)
    mu = t32(np.stack([W.initial_mean(wl)] * P_))
    cov = t32(np.stack([W.initial_cov(wl)] * P_))
    out = gp.plan_batch(P_, t32(bc), t32(obs), cem, mu, cov, seed=11,
                        out=gp.plan_outputs(cem, P_, full=True))
    torch.cuda.synchronize()
    assert gp.last_tiling()[0] == (4, 0, 1)
    xi, got, gr, gc = (np64(out[k]) for k in ("xi", "xi_bar", "resid", "c1"))
    counts = {}
    rng = np.random.default_rng(4)
    for q in (0, 21, 42, 63):
        idx = rng.choice(N, 16, replace=False)
        pr = O.project(op, bc[q], obs[q], xi[q, idx], wl.n_proj_iters)
        err = check_projection(op, bc[q], obs[q], xi[q, idx].astype(np.float32), got[q, idx],
                               pr.xi_bar, wl.n_proj_iters, label=f"c3 plan problem {q}",
                               counts=counts)
        assert np.median(err) < 1e-4, (q, np.median(err))
        np.testing.assert_allclose(gr[q, idx], pr.resid, atol=2e-3 * max(1, pr.resid.max()))
        np.testing.assert_allclose(gc[q, idx], O.smoothness_cost(op, pr.xi_bar), rtol=2e-3,
                                   atol=1e-3)
    gp.close()


@pytest.mark.parametrize("n", [1, 3, 37])
def test_project_ragged_batches(priest, n):
    say(f"project ragged N={n}")
    wl = W.with_changes(W.C1, n_steps=23)
    idx = np.arange(n)
    _project_case(priest, wl, n, idx, n_iter=30)


def test_project_zero_iterations_and_no_obstacles(priest):
    say("project n_iter=0 and n_obs=0")
    wl = W.C1
    gp, op = make(priest, wl)
    bc, obs = W.scene(wl, 0)
    xi = W.samples(wl, 3, n=10).astype(np.float32)
    xo, r, c1 = gp.project(t32(bc), t32(obs), t32(xi), 0)
    np.testing.assert_array_equal(np64(xo), xi.astype(np.float64))
    np.testing.assert_allclose(np64(r), O.residual(op, obs, xi.astype(np.float64)), rtol=1e-4, atol=1e-4)
    gp.close()
    wl0 = W.with_changes(W.C1, n_obs=0, v_max=math.inf, a_max=math.inf)
    _project_case(priest, wl0, 10, np.arange(10), n_iter=40)


def test_project_3d_ellipsoids_and_moving(priest):
    say("project 3D ellipsoids a != b, moving")
    wl = W.with_changes(W.C3, n_obs=12, n_steps=40, n_samples=50)
    gp, op = make(priest, wl)
    bc = W.boundary_values(wl)
    rng = np.random.default_rng(3)
    obs = np.zeros((12, 8))
    obs[:, :3] = rng.uniform(6, 14, (12, 3))
    obs[:, 3:6] = rng.uniform(-0.2, 0.2, (12, 3))
    obs[:, 6] = rng.uniform(0.5, 1.5, 12)
    obs[:, 7] = rng.uniform(0.5, 1.5, 12)
    xi = W.samples(wl, 4, n=50).astype(np.float32)
    xo, r, c1 = gp.project(t32(bc), t32(obs), t32(xi), 40)
    pr = O.project(op, bc, obs, xi.astype(np.float64), 40)
    check_projection(op, bc, obs, xi, np64(xo), pr.xi_bar, 40, label="ellipsoids")
    gp.close()


def test_project_deterministic_and_alias(priest):
    say("project determinism and in-place")
    wl = W.C1
    gp, _ = make(priest, wl)
    bc, obs = W.scene(wl, 0)
    xi = t32(W.samples(wl, 5))
    a = gp.project(t32(bc), t32(obs), xi, 50)
    b = gp.project(t32(bc), t32(obs), xi, 50)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    inplace = xi.clone()
    priest.priest_project(gp.handle, t32(bc), t32(obs), inplace, 50, inplace)
    assert torch.equal(inplace, a[0])
    gp.close()


def test_project_equality_constraints_hold(priest):
    say("project A xi_bar = b in FP32")
    wl = W.C2
    gp, op = make(priest, wl)
    bc, obs = W.scene(wl, 0)
    xi = W.samples(wl, 7, n=500).astype(np.float32)
    xo, _, _ = gp.project(t32(bc), t32(obs), t32(xi), 100)
    xb = np64(xo)
    viol = np.abs(xb @ op.A().T - op.b_eq(bc)).max(1)
    assert viol.max() < 1e-4 * max(1.0, np.abs(xb).max())
    gp.close()


# ---------------------------------------------------------------------------
# sampling loop
# ---------------------------------------------------------------------------
def _cem(wl, n_cem=1, **kw):
    from paper_2309_08235_amd.priest import Cem
    d = dict(n_samples=wl.n_samples, n_cem=n_cem, n_proj_iters=wl.n_proj_iters,
             n_proj=wl.n_proj, n_elite=wl.n_elite, sigma=wl.sigma, gamma=wl.gamma,
             cov_jitter=wl.cov_jitter)
    d.update(kw)
    return Cem(**d)


def _check_cem_step(op, bc, obs, wl, cem, mu, cov, noise, out, mu_gpu, cov_gpu, label, cost=None,
                    pc=None):
    """One CEM iteration of the GPU against the oracle; ``cost`` is the
    oracle's Cost matching cem.cost (None: the smoothness cost); ``pc`` the
    evolution path entering the step when cem.update is the CMA rule."""
    update = "cma" if getattr(cem, "update", 0) == 1 else "mppi"
    prm = O.CemParams(n_samples=cem.n_samples, n_proj_iters=cem.n_proj_iters, n_proj=cem.n_proj,
                      n_elite=cem.n_elite, sigma=cem.sigma, gamma=cem.gamma,
                      cov_jitter=cem.cov_jitter, cost=cost, update=update)
    st = O.cem_iteration(op, bc, obs, mu, cov, noise, prm, pc)
    xi_g = np64(out["xi"][0])
    np.testing.assert_allclose(xi_g, st.xi, atol=2e-5 * max(1, np.abs(st.xi).max()))
    # projection of the GPU's own draws, compared element by element
    pr = O.project(op, bc, obs, xi_g, cem.n_proj_iters)
    xb_g = np64(out["xi_bar"][0])
    check_projection(op, bc, obs, out["xi"][0].cpu().numpy(), xb_g, pr.xi_bar, cem.n_proj_iters,
                     label=label)
    r_g, c1_g = np64(out["resid"][0]), np64(out["c1"][0])
    np.testing.assert_allclose(r_g, pr.resid, atol=2e-3 * max(1, pr.resid.max()))
    # selection: exact on the GPU's own keys, tie-band rule against the oracle's
    proj = out["proj_idx"][0].cpu().numpy()
    elite = out["elite_idx"][0].cpu().numpy()
    np.testing.assert_array_equal(proj, O.select_lowest(r_g.astype(np.float32), cem.n_proj))
    caug_g = (c1_g.astype(np.float32) + r_g.astype(np.float32)).astype(np.float64)
    np.testing.assert_array_equal(elite, proj[O.select_lowest(caug_g[proj], cem.n_elite)])
    check_selection(pr.resid, proj, cem.n_proj, label=f"{label} proj")
    c_aug = O.trajectory_cost(op, bc, pr.xi_bar, cost) + pr.resid
    # EliteSet against the oracle's c_aug: among the GPU's constraint-elite
    # set, the elites must be the n_elite lowest oracle keys wherever those
    # are separated by more than the tie band
    pos = {int(s): i for i, s in enumerate(proj)}
    assert all(int(e) in pos for e in elite), f"{label}: an elite outside the constraint-elite set"
    check_selection(c_aug[proj], [pos[int(e)] for e in elite], cem.n_elite, label=f"{label} elite")
    # c1 of the GPU's own projected samples
    c1_o = O.trajectory_cost(op, bc, xb_g, cost)
    np.testing.assert_allclose(c1_g, c1_o, rtol=2e-3, atol=2e-3 * max(1.0, np.abs(c1_o).mean()))
    # refit of the GPU's elites with the oracle's arithmetic
    if update == "cma":
        pc0 = np.zeros(op.D) if pc is None else pc
        mu2, S2, _ = O.refit_cma(mu, cov, pc0, xb_g[elite], caug_g[elite], cem.sigma, cem.gamma)
    else:
        mu2, S2, _ = O.refit(mu, cov, xb_g[elite], caug_g[elite], cem.sigma, cem.gamma)
    np.testing.assert_allclose(mu_gpu, mu2, atol=1e-4 * max(1, np.abs(mu2).max()))
    np.testing.assert_allclose(cov_gpu, S2, atol=2e-4 * max(1, np.abs(S2).max()))
    np.testing.assert_allclose(np64(out["best_xi"][0]), xb_g[elite[0]], atol=0)
    assert abs(float(out["best_cost"][0]) - caug_g[elite[0]]) <= 1e-5 * max(1, caug_g[elite[0]])
    assert int(out["status"][0]) == 0
    return st, c_aug


def test_plan_one_iteration_c1(priest):
    say("plan c1 one CEM iteration, supplied noise")
    wl = W.C1
    gp, op = make(priest, wl)
    bc, obs = W.scene(wl, 0)
    cem = _cem(wl)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    noise = W.standard_normals(21, (1, wl.n_samples, wl.D))
    mu, cov = t32(mu0), t32(cov0)
    out = gp.plan(t32(bc), t32(obs), cem, mu, cov, noise=t32(noise))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, obs, wl, cem, mu0, cov0, noise[0], out, np64(mu), np64(cov), "c1")
    gp.close()


def test_plan_chained_iterations_c2_shape(priest):
    """Three CEM iterations at the paper-scale shape (N=1000, M=50, K=100),
    each checked from the state the GPU carried in."""
    say("plan c2 shape, 3 chained CEM iterations (oracle on every step)")
    wl = W.with_changes(W.C2, n_samples=300, n_proj=W.default_n_proj(300), n_elite=30,
                        n_proj_iters=40)
    gp, op = make(priest, wl)
    bc, obs = W.scene(W.C2, 0)
    cem = _cem(wl)
    mu_h, cov_h = W.initial_mean(wl), W.initial_cov(wl)
    mu, cov = t32(mu_h), t32(cov_h)
    for l in range(3):
        noise = W.standard_normals(100 + l, (1, wl.n_samples, wl.D))
        mu_in, cov_in = np64(mu), np64(cov)
        out = gp.plan(t32(bc), t32(obs), cem, mu, cov, noise=t32(noise))
        torch.cuda.synchronize()
        _check_cem_step(op, bc, obs, wl, cem, mu_in, cov_in, noise[0], out, np64(mu), np64(cov),
                        f"c2 iter {l}")
    gp.close()


def test_plan_philox_draws_match_oracle(priest):
    say("plan with on-device Philox draws")
    wl = W.C1
    gp, op = make(priest, wl)
    bc, obs = W.scene(wl, 1)
    cem = _cem(wl, n_proj_iters=10)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    out = gp.plan(t32(bc), t32(obs), cem, t32(mu0), t32(cov0), seed=1234, stream_id=7)
    torch.cuda.synchronize()
    z = O.normals(1234, 7, 0, wl.n_samples, wl.D)
    L = O.jittered_cholesky(cov0, cem.cov_jitter)
    np.testing.assert_allclose(np64(out["xi"][0]), mu0 + z @ L.T, atol=1e-4)
    gp.close()


def test_plan_batch_matches_single_and_graph_replays(priest):
    say("plan_batch of 4 problems vs single plans; graph replays")
    wl = W.with_changes(W.C1, n_proj_iters=20)
    gp, _ = make(priest, wl)
    P = 4
    cem = _cem(wl, n_cem=3)
    scenes = [W.scene(wl, q) for q in range(P)]
    bc = t32(np.stack([s[0] for s in scenes]))
    obs = t32(np.stack([s[1] for s in scenes]))
    mu0 = np.stack([W.initial_mean(wl)] * P)
    cov0 = np.stack([W.initial_cov(wl)] * P)
    mu, cov = t32(mu0), t32(cov0)
    out = gp.plan_batch(P, bc, obs, cem, mu, cov, seed=5, stream_base=100)
    torch.cuda.synchronize()
    for q in range(P):
        m1, c1_ = t32(mu0[q]), t32(cov0[q])
        o1 = gp.plan(bc[q], obs[q], cem, m1, c1_, seed=5, stream_id=100 + q)
        torch.cuda.synchronize()
        np.testing.assert_allclose(np64(o1["best_xi"][0]), np64(out["best_xi"][q]), atol=1e-6)
        np.testing.assert_allclose(np64(m1), np64(mu[q]), atol=1e-6)
        np.testing.assert_array_equal(o1["elite_idx"][0].cpu().numpy(), out["elite_idx"][q].cpu().numpy())
    # graph: capture once, replay several times with eager work in between
    s = torch.cuda.Stream()
    mu_g, cov_g = t32(mu0), t32(cov0)
    outg = gp.plan_outputs(cem, P)
    ws = gp.workspace(cem, P)
    for rep in range(3):
        mu_g.copy_(t32(mu0)); cov_g.copy_(t32(cov0))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            gp.plan_batch(P, bc, obs, cem, mu_g, cov_g, seed=5, stream_base=100, out=outg,
                          workspace=ws, use_graph=True, stream=s)
        s.synchronize()
        assert torch.equal(outg["best_xi"], out["best_xi"]), f"replay {rep}"
        assert torch.equal(mu_g, mu), f"replay {rep}"
        assert torch.equal(cov_g, cov), f"replay {rep}"
        _ = torch.randn(1000, device=DEV).sum().item()   # eager work between replays
    gp.close()


def test_plan_nonfinite_mean_isolated(priest):
    say("plan batch with a NaN mean in one problem")
    wl = W.with_changes(W.C1, n_proj_iters=10)
    gp, _ = make(priest, wl)
    P = 3
    cem = _cem(wl, n_cem=2)
    bc = t32(np.stack([W.scene(wl, q)[0] for q in range(P)]))
    obs = t32(np.stack([W.scene(wl, q)[1] for q in range(P)]))
    mu0 = np.stack([W.initial_mean(wl)] * P)
    mu0[1, 3] = np.nan
    cov0 = np.stack([W.initial_cov(wl)] * P)
    out = gp.plan_batch(P, bc, obs, cem, t32(mu0), t32(cov0), seed=1)
    ref = gp.plan_batch(P, bc, obs, cem, t32(np.nan_to_num(mu0)), t32(cov0), seed=1)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert st[1] == priest.PRIEST_ERR_NONFINITE and st[0] == 0 and st[2] == 0
    for q in (0, 2):
        assert torch.equal(out["best_xi"][q], ref["best_xi"][q])
    gp.close()


def test_plan_one_iteration_3d(priest):
    """3D (D = 33): covariance entries beyond one per thread and a 33 x 33
    Cholesky, against the oracle's refit of the GPU's elites."""
    say("plan 3D one CEM iteration, supplied noise")
    wl = W.with_changes(W.C3, n_obs=20, n_steps=50, n_samples=160, n_proj=W.default_n_proj(160),
                        n_elite=24, n_proj_iters=30)
    gp, op = make(priest, wl)
    bc = W.boundary_values(wl)
    obs = W.obstacles(wl, 3003)
    cem = _cem(wl)
    mu0, cov0 = W.initial_mean(wl), W.initial_cov(wl)
    noise = W.standard_normals(31, (1, wl.n_samples, wl.D))
    mu, cov = t32(mu0), t32(cov0)
    out = gp.plan(t32(bc), t32(obs), cem, mu, cov, noise=t32(noise))
    torch.cuda.synchronize()
    _check_cem_step(op, bc, obs, wl, cem, mu0, cov0, noise[0], out, np64(mu), np64(cov), "3d")
    L = np.linalg.cholesky(np64(cov) + cem.cov_jitter * np.trace(np64(cov)) / wl.D * np.eye(wl.D))
    assert np.all(np.isfinite(L))
    gp.close()


# ---------------------------------------------------------------------------
# mixed precision: BF16 MFMA operands for the right-hand side and a BF16
# hi/lo split of the KKT product, FP32 accumulation, FP32 refinement tail
# ---------------------------------------------------------------------------
def test_bf16_mixed_error_against_oracle(priest):
    """Error of the mixed-precision projection against the FP64 oracle is
    reported per coefficient and per constraint residual, and bounded."""
    say("project c2 BF16 mixed precision, oracle on 40 sampled samples")
    wl = W.C2
    idx = np.random.default_rng(11).choice(1000, 40, replace=False)
    bc, obs = W.scene(wl, 0)
    xi = W.samples(wl, 5, n=1000).astype(np.float32)
    gp32 = priest.Problem.from_workload(wl)
    gpbf = priest.Problem.from_workload(wl, precision=priest.BF16_MIXED, n_refine_fp32=10)
    x32, r32, _ = gp32.project(t32(bc), t32(obs), t32(xi), wl.n_proj_iters)
    xbf, rbf, _ = gpbf.project(t32(bc), t32(obs), t32(xi), wl.n_proj_iters)
    torch.cuda.synchronize()
    op = oracle_problem(wl)
    pr = O.project(op, bc, obs, xi[idx].astype(np.float64), wl.n_proj_iters)
    e32 = rel_err(np64(x32)[idx], pr.xi_bar)
    ebf = rel_err(np64(xbf)[idx], pr.xi_bar)
    res_err = np.abs(np64(rbf)[idx] - pr.resid)
    eq = np.abs(np64(xbf) @ op.A().T - op.b_eq(bc)).max()
    print(f"[bf16] coefficient rel err median {np.median(ebf):.2e} p99 {np.quantile(ebf, .99):.2e} "
          f"max {ebf.max():.2e} (fp32: median {np.median(e32):.2e}); residual abs err "
          f"median {np.median(res_err):.2e} max {res_err.max():.2e}; max |A xi - b| {eq:.2e}",
          flush=True)
    assert np.median(ebf) < 3e-3
    assert np.quantile(ebf, 0.9) < 3e-2
    assert np.median(res_err) < 2e-2
    assert eq < 1e-3
    gp32.close(); gpbf.close()


def test_bf16_mode_with_full_refinement_is_fp32(priest):
    """With n_refine_fp32 >= n_iter no iteration runs in BF16: the result is
    bitwise the FP32 one."""
    say("BF16 mode with full FP32 refinement")
    wl = W.C1
    bc, obs = W.scene(wl, 0)
    xi = t32(W.samples(wl, 5))
    a = priest.Problem.from_workload(wl).project(t32(bc), t32(obs), xi, 50)
    b = priest.Problem.from_workload(wl, precision=priest.BF16_MIXED, n_refine_fp32=50).project(
        t32(bc), t32(obs), xi, 50)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
