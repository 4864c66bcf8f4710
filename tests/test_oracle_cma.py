"""Pins of the oracle's CMA-ES-style covariance update (the remark after
eqs. (9a)-(9c) that Alg. 1 is agnostic to the update rule)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2309_08235_amd import workloads as W


def _case(rng, D=6, M=9):
    mu = rng.normal(0, 1, D)
    B = rng.normal(0, 1, (D, D))
    Sigma = B @ B.T + 0.5 * np.eye(D)
    pc = rng.normal(0, 0.3, D)
    el = mu + rng.normal(0, 1.2, (M, D))
    c = rng.uniform(0.0, 3.0, M)
    return mu, Sigma, pc, el, c


def test_affine_equivariance():
    """CMA-ES is affine invariant: mapping samples, mean and path by x -> A x + b
    (and Sigma -> A Sigma A^T) maps the update the same way.  A transposed
    product or a mean taken about the wrong point breaks it."""
    rng = np.random.default_rng(0)
    mu, S, pc, el, c = _case(rng)
    A = rng.normal(0, 1, (6, 6)) + 2 * np.eye(6)
    b = rng.normal(0, 1, 6)
    m1, S1, p1 = O.refit_cma(mu, S, pc, el, c, 0.6, 0.8)
    m2, S2, p2 = O.refit_cma(A @ mu + b, A @ S @ A.T, A @ pc, el @ A.T + b, c, 0.6, 0.8)
    np.testing.assert_allclose(m2, A @ m1 + b, atol=1e-10)
    np.testing.assert_allclose(p2, A @ p1, atol=1e-10)
    np.testing.assert_allclose(S2, A @ S1 @ A.T, atol=1e-9)


def test_rates_and_equal_weights():
    """Equal costs give equal weights, mu_eff = N_elite, and the tutorial's
    default rates for that selection mass."""
    rng = np.random.default_rng(1)
    mu, S, pc, el, _ = _case(rng, D=4, M=5)
    c = np.full(5, 2.0)
    cc, c1, cmu = O.cma_rates(4, 5.0)
    assert cc == pytest.approx((4 + 5 / 4) / (4 + 4 + 10 / 4))
    assert c1 == pytest.approx(2 / (5.3 ** 2 + 5))
    assert cmu == pytest.approx(min(1 - c1, 2 * (5 - 2 + 0.2) / (36 + 5)))
    m1, S1, p1 = O.refit_cma(mu, S, np.zeros(4), el, c, 1.0, 1.0)
    np.testing.assert_allclose(m1, el.mean(axis=0), atol=1e-12)
    yw = el.mean(axis=0) - mu
    np.testing.assert_allclose(p1, math.sqrt(cc * (2 - cc) * 5) * yw, atol=1e-12)
    y = el - mu
    want = (1 - c1 - cmu) * S + c1 * np.outer(p1, p1) + cmu * (y.T @ y) / 5
    np.testing.assert_allclose(S1, want, atol=1e-12)
    # rank-mu term against numpy.cov about the old mean (aweights, bias=True form)
    np.testing.assert_allclose((y.T @ y) / 5, np.cov(el.T, bias=True, aweights=np.ones(5))
                               + np.outer(el.mean(0) - mu, el.mean(0) - mu), atol=1e-12)


def test_single_elite_and_positive_definite():
    rng = np.random.default_rng(2)
    mu, S, pc, el, c = _case(rng, D=5, M=1)
    m1, S1, p1 = O.refit_cma(mu, S, pc, el, c, 0.5, 1.0)
    cc, c1, cmu = O.cma_rates(5, 1.0)
    assert cmu == 0.0            # mu_eff = 1: no rank-mu term
    np.testing.assert_allclose(S1, (1 - c1) * S + c1 * np.outer(p1, p1), atol=1e-12)
    for seed in range(5):
        mu, S, pc, el, c = _case(np.random.default_rng(10 + seed))
        _, S1, _ = O.refit_cma(mu, S, pc, el, c, 0.5, 1.0)
        np.testing.assert_allclose(S1, S1.T, atol=1e-12)
        assert np.all(np.linalg.eigvalsh(S1) > 0)


def test_plan_with_cma_update_improves_and_carries_the_path():
    wl = W.with_changes(W.C1, v_max=3.0, a_max=3.0, bc_mask=W.BC_DEFAULT)
    bc, obs = W.scene(W.C1, 2)
    prob = O.Problem(wl.dims, wl.n_coeff, wl.n_steps, wl.horizon, wl.n_obs, wl.rho,
                     wl.v_max, wl.a_max, wl.bc_mask)
    prm = O.CemParams(n_samples=64, n_proj_iters=20, n_proj=47, n_elite=12, update="cma")
    steps = O.plan(prob, bc, obs, W.initial_mean(wl), W.initial_cov(wl), prm, n_cem=5, seed=99)
    assert steps[-1].best_cost < steps[0].best_cost
    # the second step starts from the first step's path
    st0, st1 = steps[0], steps[1]
    w = np.exp(-(st1.c_aug[st1.elite_idx] - st1.c_aug[st1.elite_idx].min()))
    again = O.refit_cma(st0.mu, st0.Sigma, st0.pc, st1.xi_bar[st1.elite_idx],
                        st1.c_aug[st1.elite_idx], prm.sigma, prm.gamma)
    np.testing.assert_allclose(again[2], st1.pc, atol=1e-12)
    np.testing.assert_allclose(again[1], st1.Sigma, atol=1e-12)


def test_rates_asymptotics():
    """The default rates pinned by their limits rather than by retyping them:
    c_c ~ 4/n, c_1 ~ 2/n^2 and c_mu ~ 2 (mu_eff - 2 + 1/mu_eff)/n^2 for large
    n; c_1 + c_mu <= 1 always, tending to 1 as mu_eff grows (the rank-mu
    update then replaces the old covariance).  A dropped square, a swapped
    rate or a missing min() fails one of these."""
    for mu_eff in (1.0, 3.0, 12.5):
        n = 1e6
        cc, c1, cmu = O.cma_rates(n, mu_eff)
        assert cc * n == pytest.approx(4.0, rel=1e-4)
        assert c1 * n * n == pytest.approx(2.0, rel=1e-4)
        assert cmu * n * n == pytest.approx(2.0 * (mu_eff - 2.0 + 1.0 / mu_eff), rel=1e-4, abs=1e-9)
    for n in (2, 6, 22, 33):
        for mu_eff in (1.0, 2.0, 7.3, 50.0, 1e3):
            cc, c1, cmu = O.cma_rates(n, mu_eff)
            assert 0.0 < cc < 1.0 and 0.0 < c1 < 1.0 and 0.0 <= cmu
            assert c1 + cmu <= 1.0 + 1e-15
        _, c1, cmu = O.cma_rates(n, 1e9)
        assert c1 + cmu == pytest.approx(1.0, abs=1e-6)


def test_evolution_path_is_stationary_under_random_selection():
    """With elites drawn from N(mu, Sigma) independently of their costs (no
    selection pressure) the path's normalisation sqrt(c_c (2 - c_c) mu_eff)
    keeps it distributed as N(0, Sigma): the stationary covariance of
    p' = (1 - c_c) p + sqrt(c_c (2 - c_c) mu_eff) y_w is exactly Sigma."""
    rng = np.random.default_rng(7)
    D, M = 3, 6
    B = np.array([[1.0, 0.0, 0.0], [0.4, 0.8, 0.0], [-0.3, 0.2, 0.5]])
    S = B @ B.T
    mu = np.array([1.0, -2.0, 0.5])
    pc = np.zeros(D)
    acc = np.zeros((D, D))
    n_burn, n_keep = 200, 6000
    for it in range(n_burn + n_keep):
        el = mu + rng.normal(0.0, 1.0, (M, D)) @ B.T
        _, _, pc = O.refit_cma(mu, S, pc, el, np.zeros(M), 0.0, 1.0)
        if it >= n_burn:
            acc += np.outer(pc, pc)
    emp = acc / n_keep
    # successive paths are correlated (1 - c_c ~ 0.5 here): a loose bound
    np.testing.assert_allclose(emp, S, atol=0.12)
    # a path normalised by sqrt(mu_eff) only (c_c dropped) would be off by ~1.4x
    cc, _, _ = O.cma_rates(D, float(M))
    assert abs(cc * (2 - cc) - 1.0) > 0.2
