"""Pins of the oracle's closed-form alpha/beta/d targets (Appendix, eqs. (10),
(11), (15a)-(15c)) and of the residual r, by brute-force search on tiny inputs."""
import math

import numpy as np
import pytest

import oracle as O


def _prob(dims, n_obs=1, v_max=math.inf, a_max=math.inf):
    return O.Problem(dims=dims, n_coeff=3, n_steps=2, horizon=1.0, n_obs=n_obs,
                     v_max=v_max, a_max=a_max)


def _xi_with_positions(prob, p0, p1):
    """Coefficients whose grid positions (K = 2, degree 2) are p0 and p1."""
    xi = np.zeros((prob.dims, prob.n_coeff))
    xi[:, 0] = p0
    xi[:, -1] = p1
    xi[:, 1] = 0.5 * (np.asarray(p0) + np.asarray(p1))
    return xi.reshape(1, -1)


def _obstacle_target(prob, obs, p):
    """Target of obstacle 0 at the first grid point for robot position p."""
    xi = _xi_with_positions(prob, p, p)
    e = O.targets(prob, obs, xi)
    K = prob.n_steps
    R = (prob.n_obs + 2) * K
    return np.array([e[0, ax * R + 0] for ax in range(prob.dims)])


def _sphere_points(n):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


@pytest.mark.parametrize("seed", range(20))
def test_circle_target_is_nearest_feasible_point(seed):
    rng = np.random.default_rng(seed)
    prob = _prob(2)
    a = rng.uniform(0.2, 2.0)
    o = rng.uniform(-3, 3, 2)
    p = o + rng.uniform(-2.5 * a, 2.5 * a, 2)
    obs = np.zeros((1, 8)); obs[0, :2] = o; obs[0, 6] = obs[0, 7] = a
    tgt = _obstacle_target(prob, obs, p)
    # brute force: dense boundary samples plus p itself when p is feasible
    th = np.linspace(0, 2 * np.pi, 200001)
    cand = o[None, :] + a * np.stack([np.cos(th), np.sin(th)], 1)
    if np.linalg.norm(p - o) >= a:
        cand = np.vstack([cand, p])
    best = np.min(np.linalg.norm(cand - p, axis=1))
    assert np.linalg.norm(tgt - o) >= a * (1 - 1e-12)          # feasible
    assert np.linalg.norm(tgt - p) <= best + a * 2 * np.pi / 200000 + 1e-12


@pytest.mark.parametrize("seed", range(10))
def test_sphere_target_is_nearest_feasible_point(seed):
    rng = np.random.default_rng(100 + seed)
    prob = _prob(3)
    a = rng.uniform(0.2, 2.0)
    o = rng.uniform(-3, 3, 3)
    p = o + rng.uniform(-2 * a, 2 * a, 3)
    obs = np.zeros((1, 8)); obs[0, :3] = o; obs[0, 6] = obs[0, 7] = a
    tgt = _obstacle_target(prob, obs, p)
    cand = o[None, :] + a * _sphere_points(200000)
    if np.linalg.norm(p - o) >= a:
        cand = np.vstack([cand, p])
    best = np.min(np.linalg.norm(cand - p, axis=1))
    assert np.linalg.norm(tgt - o) >= a * (1 - 1e-12)
    # Fibonacci lattice spacing ~ sqrt(4 pi / n) a
    assert np.linalg.norm(tgt - p) <= best + 0.01 * a


@pytest.mark.parametrize("seed", range(10))
def test_ellipsoid_target_is_feasible_and_radial(seed):
    """a != b: the scaled closed form lands on or outside the ellipsoid, on the
    ray from the centre through the robot (radial projection)."""
    rng = np.random.default_rng(200 + seed)
    prob = _prob(3)
    a, b = rng.uniform(0.3, 1.5, 2)
    o = rng.uniform(-3, 3, 3)
    p = o + rng.uniform(-1.5, 1.5, 3) * np.array([a, a, b])
    obs = np.zeros((1, 8)); obs[0, :3] = o; obs[0, 6] = a; obs[0, 7] = b
    tgt = _obstacle_target(prob, obs, p)
    u = tgt - o
    q = (u[0] ** 2 + u[1] ** 2) / a ** 2 + u[2] ** 2 / b ** 2
    assert q >= 1 - 1e-12
    dp = p - o
    np.testing.assert_allclose(np.cross(u, dp), 0.0, atol=1e-12)
    assert np.dot(u, dp) > 0
    qp = (dp[0] ** 2 + dp[1] ** 2) / a ** 2 + dp[2] ** 2 / b ** 2
    if qp >= 1:
        np.testing.assert_allclose(tgt, p, atol=1e-12)


def test_zero_offset_uses_canonical_direction():
    for dims, want in ((2, [0.7, 0.0]), (3, [0.0, 0.0, 0.9])):
        prob = _prob(dims)
        obs = np.zeros((1, 8)); obs[0, :dims] = 1.25; obs[0, 6] = 0.7; obs[0, 7] = 0.9 if dims == 3 else 0.7
        tgt = _obstacle_target(prob, obs, np.full(dims, 1.25))
        np.testing.assert_allclose(tgt - 1.25, want, atol=1e-15)


@pytest.mark.parametrize("dims", [2, 3])
def test_velocity_target_is_nearest_point_of_ball(dims):
    rng = np.random.default_rng(dims)
    vmax = 1.3
    prob = O.Problem(dims=dims, n_coeff=2, n_steps=2, horizon=1.0, n_obs=0, v_max=vmax)
    for _ in range(20):
        v = rng.uniform(-3, 3, dims)
        # degree-1 polynomial with velocity v everywhere: c1 - c0 = v T
        xi = np.zeros((dims, 2)); xi[:, 1] = v
        e = O.targets(prob, np.zeros((0, 8)), xi.reshape(1, -1))
        R = 2 * 2
        tgt = np.array([e[0, ax * R + 0] for ax in range(dims)])
        # brute force over a polar grid of the ball
        if dims == 2:
            r = np.linspace(0, vmax, 801)[:, None]
            th = np.linspace(0, 2 * np.pi, 4001)[None, :]
            grid = np.stack([(r * np.cos(th)).ravel(), (r * np.sin(th)).ravel()], 1)
            tol = vmax * 2 * np.pi / 4000 + 1e-12
        else:
            grid = np.concatenate([s * _sphere_points(20000) for s in np.linspace(0, vmax, 201)])
            tol = 0.03 * vmax
        best = np.min(np.linalg.norm(grid - v, axis=1))
        assert np.linalg.norm(tgt) <= vmax * (1 + 1e-12)
        assert np.linalg.norm(tgt - v) <= best + tol


@pytest.mark.parametrize("seed", range(8))
def test_am_steps_minimise_lagrangian_term(seed):
    """Eqs. (15a)-(15c) for a = b: with the other two polar variables held
    fixed, the closed form of each one is the minimiser of the obstacle term of
    eq. (14), checked against a dense grid."""
    rng = np.random.default_rng(300 + seed)
    a = rng.uniform(0.3, 1.5)
    dlt = rng.uniform(-2, 2, 3)

    def term(al, be, d):
        al, be, d = np.broadcast_arrays(np.asarray(al, float), np.asarray(be, float),
                                        np.asarray(d, float))
        u = np.stack([np.cos(al) * np.sin(be), np.sin(al) * np.sin(be), np.cos(be)], -1)
        return np.sum((dlt - a * d[..., None] * u) ** 2, -1)

    prob = _prob(3)
    obs = np.zeros((1, 8)); obs[0, 6] = obs[0, 7] = a
    alpha, beta, d = O.polar_obstacle(prob, dlt.reshape(1, 3, 1), np.zeros((1, 1, 3)), obs)
    alpha, beta, d = alpha.item(), beta.item(), d.item()
    g = np.linspace(-np.pi, np.pi, 100001)
    b0, d0 = rng.uniform(0.2, 3.0), rng.uniform(1, 3)
    assert term(alpha, b0, d0) <= term(g, b0, d0).min() + 1e-8
    g = np.linspace(0, np.pi, 100001)
    assert term(alpha, beta, d0) <= term(alpha, g, d0).min() + 1e-8
    g = np.linspace(1, 10, 100001)
    assert term(alpha, beta, d) <= term(alpha, beta, g).min() + 1e-8


@pytest.mark.parametrize("dims", [2, 3])
def test_residual_dense_equals_violation_form(dims):
    rng = np.random.default_rng(7 + dims)
    prob = O.Problem(dims=dims, n_coeff=11, n_steps=40, horizon=8.0, n_obs=6, v_max=1.2, a_max=0.8)
    obs = np.zeros((6, 8))
    obs[:, :dims] = rng.uniform(1, 7, (6, dims))
    obs[:, 3:3 + dims] = rng.uniform(-0.3, 0.3, (6, dims))
    obs[:, 6] = rng.uniform(0.5, 1.5, 6)
    obs[:, 7] = obs[:, 6] if dims == 2 else rng.uniform(0.5, 1.5, 6)
    xi = np.linspace(0, 8, 11)[None, None, :] + rng.normal(0, 1.5, (30, dims, 11))
    xi = xi.reshape(30, -1)
    np.testing.assert_allclose(O.residual(prob, obs, xi), O.residual_dense(prob, obs, xi),
                               rtol=1e-12, atol=1e-12)


def test_residual_zero_iff_feasible_on_grid():
    rng = np.random.default_rng(11)
    prob = O.Problem(dims=2, n_coeff=11, n_steps=60, horizon=10.0, n_obs=3, v_max=5.0, a_max=5.0)
    obs = np.zeros((3, 8)); obs[:, :2] = [[3, 3], [6, 5], [4, 8]]; obs[:, 6] = obs[:, 7] = 0.8
    xi = np.linspace(0, 10, 11)[None, None, :] + rng.normal(0, 1.0, (200, 2, 11))
    xi = xi.reshape(200, -1)
    r = O.residual(prob, obs, xi)
    C = xi.reshape(200, 2, 11)
    p = np.einsum('kc,nac->nak', prob.P, C)
    clear = np.min(np.stack([np.linalg.norm(p - obs[j, :2][None, :, None], axis=1) - 0.8
                             for j in range(3)]), axis=(0, 2))
    v = np.linalg.norm(np.einsum('kc,nac->nak', prob.Pd, C), axis=1).max(1)
    acc = np.linalg.norm(np.einsum('kc,nac->nak', prob.Pdd, C), axis=1).max(1)
    feas = (clear >= 0) & (v <= 5.0) & (acc <= 5.0)
    assert feas.any() and (~feas).any()
    np.testing.assert_array_equal(r == 0, feas)
