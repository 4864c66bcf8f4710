"""Pins of the oracle's trajectory obstacle model (obstacle positions given at
every time stamp, the stacked x_o, y_o, z_o of eq. (13))."""
import numpy as np
import pytest

import oracle as O
from paper_2309_08235_amd import workloads as W


def _probs(wl, **kw):
    base = dict(dims=wl.dims, n_coeff=wl.n_coeff, n_steps=wl.n_steps, horizon=wl.horizon,
                n_obs=wl.n_obs, rho=wl.rho, v_max=wl.v_max, a_max=wl.a_max, bc_mask=wl.bc_mask)
    base.update(kw)
    return O.Problem(**base), O.Problem(**base, obs_model=1)


@pytest.mark.parametrize("wl", [W.with_changes(W.C2, n_steps=40), W.with_changes(W.C3, n_steps=30,
                                                                                  n_obs=12)],
                         ids=["2d moving", "3d"])
def test_constant_velocity_trajectories_reproduce_the_velocity_model(wl):
    """Positions c + v t_k at every step give the same targets, residuals and
    projection as the (centre, velocity) rows."""
    prob_v, prob_t = _probs(wl)
    bc, obs = W.scene(wl, 0)
    if wl.dims == 3:
        obs[:, 3:6] = np.random.default_rng(1).uniform(-0.4, 0.4, (wl.n_obs, 3))
    traj = W.trajectory_obstacles(wl, obs)
    xi = W.samples(wl, 2, n=12)
    np.testing.assert_allclose(O.obstacle_positions(prob_t, traj), O.obstacle_positions(prob_v, obs),
                               atol=1e-12)
    np.testing.assert_allclose(O.targets(prob_t, traj, xi), O.targets(prob_v, obs, xi), atol=1e-10)
    np.testing.assert_allclose(O.residual(prob_t, traj, xi), O.residual(prob_v, obs, xi), atol=1e-10)
    a = O.project(prob_v, bc, obs, xi, 15)
    b = O.project(prob_t, bc, traj, xi, 15)
    np.testing.assert_allclose(b.xi_bar, a.xi_bar, atol=1e-9)
    np.testing.assert_allclose(b.resid_hist, a.resid_hist, atol=1e-9)


def test_trajectory_residual_dense_equals_violation_form():
    wl = W.with_changes(W.C2, n_steps=30, n_obs=6)
    _, prob = _probs(wl)
    _, obs = W.scene(wl, 1)
    traj = W.trajectory_obstacles(wl, obs, swirl=1.5, seed=3)
    xi = W.samples(wl, 4, n=10)
    np.testing.assert_allclose(O.residual_dense(prob, traj, xi), O.residual(prob, traj, xi),
                               rtol=1e-12, atol=1e-12)


def test_each_step_uses_its_own_position():
    """An obstacle that jumps half-way: at every step the target of its rows
    is the nearest point outside the circle at that step's position."""
    wl = W.with_changes(W.C1, n_steps=20, n_obs=1)
    _, prob = _probs(wl)
    K = wl.n_steps
    pos = np.zeros((K, 2))
    pos[: K // 2] = [3.0, 3.0]
    pos[K // 2:] = [7.0, 6.0]
    traj = np.concatenate([pos.reshape(-1), [1.5, 1.5]])[None]
    xi = W.samples(wl, 5, n=6)
    e = O.targets(prob, traj, xi).reshape(6, 2, -1)[:, :, :K]          # obstacle rows
    p = np.einsum('kc,nac->nak', prob.P, xi.reshape(6, 2, wl.n_coeff))
    for k in range(K):
        d = p[:, :, k] - pos[k]
        nrm = np.linalg.norm(d, axis=1, keepdims=True)
        want = np.where(nrm < 1.5, pos[k] + 1.5 * d / nrm, p[:, :, k])
        np.testing.assert_allclose(e[:, :, k], want, atol=1e-12)


def test_trajectory_obstacles_permute():
    wl = W.with_changes(W.C2, n_steps=25, n_obs=5)
    _, prob = _probs(wl)
    bc, obs = W.scene(wl, 2)
    traj = W.trajectory_obstacles(wl, obs, swirl=1.0, seed=1)
    xi = W.samples(wl, 1, n=5)
    perm = np.array([3, 0, 4, 1, 2])
    a = O.project(prob, bc, traj, xi, 10)
    b = O.project(prob, bc, traj[perm], xi, 10)
    np.testing.assert_allclose(b.xi_bar, a.xi_bar, atol=1e-10)
