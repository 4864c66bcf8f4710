"""Pins of the oracle's workspace bounds (Appendix: G xi <= tau with a slack
variable, G = [-P; P] per axis, tau from s_min and s_max)."""
import numpy as np
import pytest

import oracle as O


def _prob(dims=2, n_obs=0, v=np.inf, a=np.inf, lo=(0.0, 0.0, 0.0), hi=(10.0, 10.0, 10.0), **kw):
    d = dict(dims=dims, n_coeff=kw.pop("n_coeff", 11), n_steps=kw.pop("n_steps", 40),
             horizon=kw.pop("horizon", 8.0), n_obs=n_obs, v_max=v, a_max=a,
             s_min=tuple(lo[:dims]), s_max=tuple(hi[:dims]))
    d.update(kw)
    return O.Problem(**d)


def _obs(rng, M, dims):
    obs = np.zeros((M, 8))
    obs[:, :dims] = rng.uniform(2, 8, (M, dims))
    obs[:, 3:3 + dims] = rng.uniform(-0.3, 0.3, (M, dims))
    obs[:, 6] = rng.uniform(0.4, 0.9, M)
    obs[:, 7] = obs[:, 6] if dims == 2 else rng.uniform(0.4, 0.9, M)
    return obs


@pytest.mark.parametrize("dims", [2, 3])
def test_residual_dense_equals_violation_form_with_bounds(dims):
    rng = np.random.default_rng(5)
    prob = _prob(dims, n_obs=4, v=1.3, a=0.9, lo=(1, 2, 1.5), hi=(8, 7, 9))
    obs = _obs(rng, 4, dims)
    xi = rng.normal(5.0, 4.0, (16, prob.D))     # wanders well outside the box
    r_dense = O.residual_dense(prob, obs, xi)
    r_viol = O.residual(prob, obs, xi)
    np.testing.assert_allclose(r_dense, r_viol, rtol=1e-12, atol=1e-12)
    # the bound rows alone: the distance of every position to the box
    p = np.einsum('kc,nac->nak', prob.P, xi.reshape(16, dims, 11))
    lo = np.array([1, 2, 1.5])[:dims][None, :, None]
    hi = np.array([8, 7, 9])[:dims][None, :, None]
    only = O.residual(_prob(dims, lo=(1, 2, 1.5), hi=(8, 7, 9)), np.zeros((0, 8)), xi)
    free = O.residual(O.Problem(dims=dims, n_coeff=11, n_steps=40, horizon=8.0, n_obs=0), np.zeros((0, 8)), xi)
    assert np.all(free == 0.0)
    np.testing.assert_allclose(only, np.sqrt(((np.clip(p, lo, hi) - p) ** 2).sum(axis=(1, 2))),
                               rtol=1e-12)


def test_slack_step_minimises_the_lagrangian_over_nonnegative_slack():
    """The slack of the Appendix's AM step is the minimiser over s >= 0 of
    ||G xi_bar - tau + s||^2: random feasible perturbations never do better."""
    rng = np.random.default_rng(1)
    prob = _prob(2, lo=(1, 1), hi=(9, 9), n_steps=12)
    xi = rng.normal(5.0, 5.0, (1, prob.D))
    e = O.targets(prob, np.zeros((0, 8)), xi)
    F = prob.F()
    K = prob.n_steps
    R = prob.n_rows_axis
    y = (xi @ F.T).reshape(2, R)
    eg = e.reshape(2, R)[:, 2 * K:]
    for ax in range(2):
        tau = prob.tau(ax)
        g = y[ax, 2 * K:]
        s_star = tau - eg[ax]
        assert np.all(s_star >= 0)
        best = np.sum((g - tau + s_star) ** 2)
        for _ in range(200):
            s = np.maximum(0.0, s_star + rng.normal(0, 0.5, s_star.shape))
            assert np.sum((g - tau + s) ** 2) >= best - 1e-12


def test_feasible_sample_is_a_fixed_point():
    """A trajectory inside the box that meets A xi = b is its own projection:
    every target equals F xi, so the iterate never moves."""
    prob = _prob(2, lo=(-1, -1), hi=(11, 11), n_steps=30)
    bc = np.array([[0, 0, 0, 10, 0, 0], [0, 0, 0, 10, 0, 0]], float)
    # straight line from (0,0) at rest to (10,10): Bernstein coefficients of a
    # monotone ramp stay inside the box
    w = np.array([0, 0, 0, 1, 2, 3, 4, 5, 6, 8, 10], float) * 1.0
    A = prob.A()
    b = prob.b_eq(bc)
    xi = np.concatenate([w, w])[None]
    assert np.max(np.abs(xi @ A.T - b)) < 1e-12
    pr = O.project(prob, bc, np.zeros((0, 8)), xi, 25)
    np.testing.assert_allclose(pr.xi_bar, xi, atol=1e-9)
    assert pr.resid[0] < 1e-9


def _rows(prob, z):
    """Values of G z - tau for every axis (positive = violated)."""
    P, nc = prob.P, prob.n_coeff
    out = []
    for ax in range(prob.dims):
        p = P @ z[ax * nc:(ax + 1) * nc]
        out += [prob.s_min[ax] - p, p - prob.s_max[ax]]
    return np.concatenate(out)


@pytest.mark.parametrize("dims,seed", [(2, s) for s in range(6)] + [(3, s) for s in range(3)])
def test_bounds_only_iteration_ends_feasible(dims, seed):
    """With the box as the only constraint besides A z = b, the iteration
    reaches a point inside the box (r = 0, every row of G z <= tau holds).
    As stated, the slack step carries no multiplier of its own, so this
    fixed point is a feasible point near the Euclidean projection, not
    necessarily the projection itself."""
    rng = np.random.default_rng(seed)
    lo, hi = (0.5, 1.0, -2.0), (7.0, 8.0, 3.0)
    prob = _prob(dims, lo=lo, hi=hi, n_coeff=6, n_steps=12, horizon=4.0, rho=1.0)
    bc = np.zeros((dims, 6))
    bc[:, 0] = [1, 2, 0][:dims]
    bc[:, 3] = [6, 7, 1][:dims]
    xi = rng.normal(4.0, 6.0, (1, prob.D))
    assert np.any(_rows(prob, xi[0]) > 0.1)           # the sample starts outside
    pr = O.project(prob, bc, np.zeros((0, 8)), xi, 1500)
    got = pr.xi_bar[0]
    assert pr.resid[0] < 1e-9
    assert np.all(_rows(prob, got) <= 1e-9)
    assert np.max(np.abs(prob.A() @ got - prob.b_eq(bc))) < 1e-9


def test_mirrored_box_gives_the_mirrored_trajectory():
    """x -> -x maps the box [lo, hi] to [-hi, -lo]: lower and upper rows of G
    trade places, so the projected trajectory must mirror exactly."""
    rng = np.random.default_rng(4)
    n_obs = 2
    obs = _obs(rng, n_obs, 2)
    prob = _prob(2, n_obs=n_obs, v=2.0, a=1.5, lo=(0.5, 1.0), hi=(7.0, 8.0), n_steps=20)
    mprob = _prob(2, n_obs=n_obs, v=2.0, a=1.5, lo=(-7.0, 1.0), hi=(-0.5, 8.0), n_steps=20)
    bc = np.array([[1, 0, 0, 6, 0, 0], [2, 0, 0, 7, 0, 0]], float)
    xi = rng.normal(4.0, 4.0, (3, prob.D))
    flip = np.concatenate([-np.ones(11), np.ones(11)])
    mobs = obs.copy()
    mobs[:, 0] *= -1
    mobs[:, 3] *= -1
    a = O.project(prob, bc, obs, xi, 30)
    b = O.project(mprob, bc * np.array([[-1.0], [1.0]]), mobs, xi * flip, 30)
    np.testing.assert_allclose(b.xi_bar, a.xi_bar * flip, atol=1e-10)
    np.testing.assert_allclose(b.resid, a.resid, atol=1e-10)


def test_far_bounds_reach_the_unbounded_fixed_point():
    """Bounds that never bind leave the fixed point unchanged (they only
    change the path through I + rho F^T F)."""
    rng = np.random.default_rng(3)
    base = dict(dims=2, n_coeff=6, n_steps=12, horizon=4.0, n_obs=0, v_max=np.inf, a_max=np.inf)
    bc = np.array([[1, 0, 0, 6, 0, 0], [2, 0, 0, 7, 0, 0]], float)
    xi = rng.normal(4.0, 1.0, (2, 12))
    prob = O.Problem(**base)
    A, b = prob.A(), prob.b_eq(bc)
    least_norm = xi - np.linalg.solve(A @ A.T, (xi @ A.T - b).T).T @ A
    got = O.project(O.Problem(**base, s_min=(-1e3, -1e3), s_max=(1e3, 1e3)), bc, np.zeros((0, 8)),
                    xi, 3000).xi_bar
    np.testing.assert_allclose(got, least_norm, atol=1e-9)
