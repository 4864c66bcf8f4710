"""Pins of the oracle's navigation cost terms (c1 need not be smooth: curvature,
distance to the start-goal segment, car-like steering angle) against closed
forms on polynomial trajectories the Bernstein basis represents exactly."""
import math

import numpy as np
import pytest

import oracle as O


def _prob(dims, K=41, T=4.0, nc=11):
    return O.Problem(dims=dims, n_coeff=nc, n_steps=K, horizon=T, n_obs=0)


def _coeffs(poly_per_axis, T, nc):
    """Bernstein coefficients of x_d(t) = sum_j c_j t^j on [0, T] (j <= nc-1):
    t = T tau, and the monomial tau^j has the Bernstein coefficients
    C(i, j) / C(n, j), i = 0..n (the textbook degree-elevation identity)."""
    n = nc - 1
    out = []
    for cs in poly_per_axis:
        row = np.zeros(nc)
        for j, c in enumerate(cs):
            row += c * T ** j * np.array([math.comb(i, j) / math.comb(n, j) for i in range(nc)])
        out.append(row)
    return np.concatenate(out)


def test_smoothness_cost_closed_forms():
    """c1 = sum_k ||a_k||^2 (Sec. V-A) on trajectories whose acceleration is
    known exactly: a parabola x_d = c_d t^2 has a constant acceleration 2 c_d,
    so c1 = K * sum_d 4 c_d^2; a cubic x = c t^3 has a = 6 c t, so
    c1 = 36 c^2 sum_k t_k^2.  Catches ||a|| written for ||a||^2, a constant
    factor, a dropped axis and a wrong time grid, none of which an invariance
    or a comparison with itself would."""
    T, K = 5.0, 37
    for dims in (2, 3):
        prob = O.Problem(dims=dims, n_coeff=11, n_steps=K, horizon=T, n_obs=0)
        cs = [0.35, -1.2, 0.8][:dims]
        # linear and constant parts add nothing
        xi = _coeffs([(1.0 + d, 0.5 - d, c) for d, c in enumerate(cs)], T, 11)[None]
        want = K * sum(4.0 * c * c for c in cs)
        np.testing.assert_allclose(O.smoothness_cost(prob, xi), [want], rtol=1e-10)
        np.testing.assert_allclose(O.trajectory_cost(prob, np.zeros((dims, 6)), xi), [want],
                                   rtol=1e-10)
        np.testing.assert_allclose(
            O.trajectory_cost(prob, np.zeros((dims, 6)), xi, O.Cost(kind=1, w_acc=1.0)), [want],
            rtol=1e-10)
    prob = O.Problem(dims=2, n_coeff=11, n_steps=K, horizon=T, n_obs=0)
    c = 0.07
    xi = _coeffs([(0.0, 0.0, 0.0, c), (2.0, 1.0, 0.0, 0.0)], T, 11)[None]
    t = O.time_grid(K, T)
    np.testing.assert_allclose(O.smoothness_cost(prob, xi), [36.0 * c * c * np.sum(t * t)],
                               rtol=1e-10)
    # two samples at once: the cost is per sample
    both = np.concatenate([xi, 2.0 * xi])
    np.testing.assert_allclose(O.smoothness_cost(prob, both),
                               36.0 * c * c * np.sum(t * t) * np.array([1.0, 4.0]), rtol=1e-10)


def test_parabola_curvature_and_steering_closed_form():
    c, T, L = 0.35, 4.0, 2.5
    prob = _prob(2, T=T)
    xi = _coeffs([(0.0, 1.0, 0.0), (0.0, 0.0, c)], T, 11)[None]
    t = O.time_grid(prob.n_steps, T)
    kappa = 2 * c / (1 + 4 * c * c * t * t) ** 1.5
    bc = np.zeros((2, 6))
    eps = 1e-14
    got = O.trajectory_cost(prob, bc, xi, O.Cost(kind=1, w_acc=0.0, w_curv=1.0, eps=eps))
    np.testing.assert_allclose(got, [np.sum(kappa ** 2)], rtol=1e-9)
    got = O.trajectory_cost(prob, bc, xi, O.Cost(kind=1, w_acc=0.0, w_steer=1.0, wheelbase=L,
                                                 eps=eps))
    np.testing.assert_allclose(got, [np.sum(np.arctan(L * kappa) ** 2)], rtol=1e-9)
    # mirrored parabola: same unsigned curvature, opposite steering sign (same square)
    xm = _coeffs([(0.0, 1.0, 0.0), (0.0, 0.0, -c)], T, 11)[None]
    C = prob.Pd, prob.Pdd
    v = np.einsum('kc,nac->nak', prob.Pd, xm.reshape(1, 2, 11))
    a = np.einsum('kc,nac->nak', prob.Pdd, xm.reshape(1, 2, 11))
    np.testing.assert_allclose(O.curvature(v, a, eps, signed=True)[0], -kappa, rtol=1e-9)


def test_3d_curvature_closed_form():
    c, d, T = 0.3, 0.7, 4.0
    prob = _prob(3, T=T)
    xi = _coeffs([(0.0, 1.0, 0.0), (0.0, 0.0, c), (1.0, d, 0.0)], T, 11)[None]
    t = O.time_grid(prob.n_steps, T)
    kappa = 2 * c * math.sqrt(1 + d * d) / (1 + d * d + 4 * c * c * t * t) ** 1.5
    got = O.trajectory_cost(prob, np.zeros((3, 6)), xi,
                            O.Cost(kind=1, w_acc=0.0, w_curv=1.0, eps=1e-14))
    np.testing.assert_allclose(got, [np.sum(kappa ** 2)], rtol=1e-9)


def test_rest_is_finite_and_regularised():
    """At rest (v = 0) the curvature is |v x a| / eps^1.5 = 0, not NaN."""
    prob = _prob(2)
    xi = _coeffs([(1.0, 0.0, 0.0), (2.0, 0.0, 0.0)], 4.0, 11)[None]
    got = O.trajectory_cost(prob, np.zeros((2, 6)), xi,
                            O.Cost(kind=1, w_curv=1.0, w_steer=1.0, eps=1e-2))
    assert np.isfinite(got[0]) and abs(got[0]) < 1e-20


def test_segment_distance_closed_forms():
    T = 4.0
    prob = _prob(2, T=T)
    bc = np.zeros((2, 6))
    bc[:, 0] = [1.0, 2.0]          # start
    bc[:, 3] = [7.0, 10.0]         # goal
    u = bc[:, 3] - bc[:, 0]
    n = np.array([-u[1], u[0]]) / np.linalg.norm(u)
    cost = O.Cost(kind=1, w_acc=0.0, w_path=1.0)
    K = prob.n_steps
    # along the segment: zero
    on = _coeffs([(1.0, u[0] / T, 0.0), (2.0, u[1] / T, 0.0)], T, 11)[None]
    assert abs(O.trajectory_cost(prob, bc, on, cost)[0]) < 1e-9
    # parallel offset h inside the segment's span: h at every step
    h = 0.8
    off = _coeffs([(1.0 + h * n[0], u[0] / T, 0.0), (2.0 + h * n[1], u[1] / T, 0.0)], T, 11)[None]
    np.testing.assert_allclose(O.trajectory_cost(prob, bc, off, cost), [K * h], rtol=1e-9)
    # overshooting to 1.5x the segment: beyond the goal the distance is to the goal
    over = _coeffs([(1.0, 1.5 * u[0] / T, 0.0), (2.0, 1.5 * u[1] / T, 0.0)], T, 11)[None]
    tau = O.time_grid(K, T) / T
    want = np.where(1.5 * tau > 1.0, (1.5 * tau - 1.0) * np.linalg.norm(u), 0.0).sum()
    np.testing.assert_allclose(O.trajectory_cost(prob, bc, over, cost), [want], rtol=1e-9, atol=1e-9)
    # starting behind the start: distance to the start point
    back = _coeffs([(1.0 - u[0], u[0] / T, 0.0), (2.0 - u[1], u[1] / T, 0.0)], T, 11)[None]
    want = np.where(tau < 1.0, (1.0 - tau) * np.linalg.norm(u), 0.0).sum()
    np.testing.assert_allclose(O.trajectory_cost(prob, bc, back, cost), [want], rtol=1e-9, atol=1e-9)


def test_kind0_is_smoothness_and_weights_are_linear():
    rng = np.random.default_rng(2)
    prob = _prob(2)
    bc = np.zeros((2, 6))
    bc[:, 3] = [10.0, 10.0]
    xi = rng.normal(5.0, 2.0, (6, prob.D))
    s0 = O.trajectory_cost(prob, bc, xi, O.Cost())
    np.testing.assert_array_equal(s0, O.smoothness_cost(prob, xi))
    terms = [O.trajectory_cost(prob, bc, xi, O.Cost(kind=1, w_acc=float(i == 0), w_curv=float(i == 1),
                                                    w_path=float(i == 2), w_steer=float(i == 3)))
             for i in range(4)]
    w = (0.5, 2.0, 0.3, 1.7)
    both = O.trajectory_cost(prob, bc, xi, O.Cost(kind=1, w_acc=w[0], w_curv=w[1], w_path=w[2],
                                                  w_steer=w[3]))
    np.testing.assert_allclose(both, sum(wi * ti for wi, ti in zip(w, terms)), rtol=1e-12)
    np.testing.assert_allclose(terms[0], s0, rtol=1e-12)


def test_costs_are_rotation_invariant():
    rng = np.random.default_rng(3)
    prob = _prob(2)
    bc = np.zeros((2, 6))
    bc[:, 0] = [0.5, -1.0]
    bc[:, 3] = [9.0, 6.0]
    xi = rng.normal(3.0, 2.0, (5, prob.D))
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    C = xi.reshape(5, 2, 11)
    xr = np.einsum('ij,njc->nic', R, C).reshape(5, -1)
    bcr = R @ bc
    cost = O.Cost(kind=1, w_acc=1.0, w_curv=0.7, w_path=0.4, w_steer=0.9, wheelbase=2.0)
    np.testing.assert_allclose(O.trajectory_cost(prob, bcr, xr, cost),
                               O.trajectory_cost(prob, bc, xi, cost), rtol=1e-10)
