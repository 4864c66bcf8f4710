"""Pins of the oracle's D-PRIEST (Sec. III-C): several Gaussians, each refitted
only on its own samples, and the lowest final cost over them returned."""
import numpy as np
import pytest

import oracle as O
from paper_2309_08235_amd import workloads as W


def _setup(n_samples=32, iters=8):
    wl = W.with_changes(W.C1, v_max=3.0, a_max=3.0, bc_mask=W.BC_DEFAULT)
    bc, obs = W.scene(W.C1, 3)
    prob = O.Problem(wl.dims, wl.n_coeff, wl.n_steps, wl.horizon, wl.n_obs, wl.rho,
                     wl.v_max, wl.a_max, wl.bc_mask)
    prm = O.CemParams(n_samples=n_samples, n_proj_iters=iters, n_proj=24, n_elite=8)
    return wl, bc, obs, prob, prm


def test_pick_group_orders_nan_last_and_ties_first():
    assert O.pick_group([3.0, 1.0, 2.0]) == 1
    assert O.pick_group([np.nan, 5.0, 5.0]) == 1
    assert O.pick_group([np.nan, np.nan]) == 0
    assert O.pick_group([2.0, -np.inf, np.nan]) == 1
    assert O.pick_group([0.5]) == 0


def test_single_group_is_alg1():
    wl, bc, obs, prob, prm = _setup()
    mu, S = W.initial_mean(wl), W.initial_cov(wl)
    res = O.dpriest(prob, bc, obs, [mu], [S], prm, n_cem=2, seed=7, stream_base=5)
    ref = O.plan(prob, bc, obs, mu, S, prm, n_cem=2, seed=7, stream=5)
    assert res.best_group == 0
    np.testing.assert_array_equal(res.best_xi, ref[-1].best_xi)
    assert res.best_cost == ref[-1].best_cost


def test_groups_are_independent_and_the_pick_is_the_minimum():
    wl, bc, obs, prob, prm = _setup()
    G = 3
    mus = W.dpriest_means(wl, G)
    Ss = [W.initial_cov(wl)] * G
    res = O.dpriest(prob, bc, obs, mus, Ss, prm, n_cem=2, seed=11, stream_base=2)
    # a group's run depends only on its own distribution and stream: dropping
    # the other groups (or reordering them) leaves it unchanged
    alone = O.dpriest(prob, bc, obs, [mus[2]], [Ss[2]], prm, n_cem=2, seed=11, stream_base=4)
    np.testing.assert_array_equal(alone.groups[0][-1].mu, res.groups[2][-1].mu)
    np.testing.assert_array_equal(alone.best_xi, res.groups[2][-1].best_xi)
    finals = [g[-1].best_cost for g in res.groups]
    assert res.best_cost == min(finals)
    assert all(res.best_cost <= c for c in finals)
    np.testing.assert_array_equal(res.best_xi, res.groups[res.best_group][-1].best_xi)
    # each refit uses only that group's elites: the refitted mean of a group
    # is a convex combination of (1-sigma) mu_g and sigma * (its elites)
    for g in range(G):
        st = res.groups[g][0]
        el = st.xi_bar[st.elite_idx]
        w = np.exp(-(st.c_aug[st.elite_idx] - st.c_aug[st.elite_idx].min()) / prm.gamma)
        want = (1 - prm.sigma) * mus[g] + prm.sigma * (w @ el) / w.sum()
        np.testing.assert_allclose(st.mu, want, rtol=1e-12, atol=1e-12)


def test_dpriest_means_fan_out_around_the_straight_line():
    wl = W.C2
    for G in (1, 2, 4, 8):
        m = W.dpriest_means(wl, G)
        assert m.shape == (G, wl.D)
        base = W.initial_mean(wl)
        # the end coefficients stay on the boundary values; the fan is symmetric
        c = m.reshape(G, wl.dims, wl.n_coeff)
        b = base.reshape(wl.dims, wl.n_coeff)
        np.testing.assert_allclose(c[:, :, 0], np.broadcast_to(b[:, 0], (G, wl.dims)), atol=1e-12)
        np.testing.assert_allclose(c[:, :, -1], np.broadcast_to(b[:, -1], (G, wl.dims)), atol=1e-12)
        np.testing.assert_allclose(m.mean(axis=0), base, atol=1e-12)
    # G=1 is the straight line itself
    np.testing.assert_allclose(W.dpriest_means(wl, 1)[0], W.initial_mean(wl), atol=1e-12)


@pytest.mark.parametrize("G", [2, 4])
def test_dpriest_never_worse_than_its_first_group(G):
    wl, bc, obs, prob, prm = _setup(iters=6)
    mus = W.dpriest_means(wl, G)
    res = O.dpriest(prob, bc, obs, mus, [W.initial_cov(wl)] * G, prm, n_cem=1, seed=1)
    assert res.best_cost <= res.groups[0][-1].best_cost
