"""Pins of the oracle's polynomial basis and constraint matrices (Sec. II-A eq. (2),
eq. (3b), Appendix eq. (13), Remark 3) against textbook Bernstein facts and an
independent monomial expansion."""
import math

import numpy as np
import numpy.polynomial.polynomial as npp
import pytest

import oracle as O


@pytest.mark.parametrize("n_coeff,K,T", [(11, 50, 10.0), (11, 100, 15.0), (6, 7, 2.0), (3, 5, 1.0)])
def test_partition_of_unity_and_derivative_sums(n_coeff, K, T):
    P, Pd, Pdd = O.basis_matrices(n_coeff, K, T)
    assert P.shape == (K, n_coeff)
    np.testing.assert_allclose(P.sum(1), 1.0, atol=1e-13)
    np.testing.assert_allclose(Pd.sum(1), 0.0, atol=1e-11)
    np.testing.assert_allclose(Pdd.sum(1), 0.0, atol=1e-9)
    assert np.all(P >= 0)


@pytest.mark.parametrize("n_coeff,K,T", [(11, 50, 10.0), (11, 100, 15.0), (5, 9, 3.0)])
def test_derivatives_match_monomial_expansion(n_coeff, K, T):
    """Expand each basis polynomial in monomials and differentiate with numpy's
    polynomial routines: an independent route to Pdot and Pddot."""
    n = n_coeff - 1
    P, Pd, Pdd = O.basis_matrices(n_coeff, K, T)
    tau = np.arange(K) / (K - 1)
    for i in range(n_coeff):
        poly = np.array([math.comb(n, i)], float)
        poly = npp.polymul(poly, np.eye(i + 1)[i])          # tau^i
        poly = npp.polymul(poly, npp.polypow([1.0, -1.0], n - i))  # (1-tau)^(n-i)
        np.testing.assert_allclose(P[:, i], npp.polyval(tau, poly), atol=1e-12)
        np.testing.assert_allclose(Pd[:, i], npp.polyval(tau, npp.polyder(poly)) / T,
                                   atol=1e-9 * max(1, n ** 1 / T))
        np.testing.assert_allclose(Pdd[:, i], npp.polyval(tau, npp.polyder(poly, 2)) / T ** 2,
                                   atol=1e-8 * max(1, n ** 2 / T ** 2))


def test_linear_precision():
    """Evenly spaced coefficients i/n reproduce the straight line tau exactly."""
    n_coeff, K, T = 11, 37, 4.0
    P, Pd, Pdd = O.basis_matrices(n_coeff, K, T)
    c = np.arange(n_coeff) / (n_coeff - 1)
    tau = np.arange(K) / (K - 1)
    np.testing.assert_allclose(P @ c, tau, atol=1e-13)
    np.testing.assert_allclose(Pd @ c, 1.0 / T, atol=1e-12)
    np.testing.assert_allclose(Pdd @ c, 0.0, atol=1e-10)


def test_endpoint_rows():
    """Bernstein endpoint interpolation: P_0 = e_0, P_-1 = e_n, and the end
    derivatives n/T (c_1 - c_0), n/T (c_n - c_{n-1})."""
    n_coeff, K, T = 11, 20, 5.0
    n = n_coeff - 1
    P, Pd, Pdd = O.basis_matrices(n_coeff, K, T)
    np.testing.assert_allclose(P[0], np.eye(n_coeff)[0], atol=1e-15)
    np.testing.assert_allclose(P[-1], np.eye(n_coeff)[-1], atol=1e-15)
    want0 = np.zeros(n_coeff); want0[:2] = [-n / T, n / T]
    wantf = np.zeros(n_coeff); wantf[-2:] = [-n / T, n / T]
    np.testing.assert_allclose(Pd[0], want0, atol=1e-12)
    np.testing.assert_allclose(Pd[-1], wantf, atol=1e-12)
    w2 = n * (n - 1) / T ** 2
    np.testing.assert_allclose(Pdd[0][:3], [w2, -2 * w2, w2], atol=1e-12)


def test_remark3_dimensions():
    """Remark 3: F is 3(n_o+2)n_p x 3n_v and e has 3(n_o+2)n_p entries (3D)."""
    prob = O.Problem(dims=3, n_coeff=11, n_steps=30, horizon=8.0, n_obs=7, v_max=2.0, a_max=3.0)
    F = prob.F()
    assert F.shape == (3 * (7 + 2) * 30, 3 * 11)
    obs = np.zeros((7, 8)); obs[:, 6] = obs[:, 7] = 0.5; obs[:, 0] = np.arange(7)
    xi = np.random.default_rng(0).standard_normal((2, 33))
    assert O.targets(prob, obs, xi).shape == (2, 3 * (7 + 2) * 30)
    # F is block diagonal with identical blocks [P;..;P; Pdot; Pddot]
    blk = F[:(7 + 2) * 30, :11]
    np.testing.assert_array_equal(blk[:30], prob.P)
    np.testing.assert_array_equal(blk[6 * 30:7 * 30], prob.P)
    np.testing.assert_array_equal(blk[7 * 30:8 * 30], prob.Pd)
    np.testing.assert_array_equal(F[(7 + 2) * 30:2 * (7 + 2) * 30, 11:22], blk)
    assert np.all(F[:(7 + 2) * 30, 11:] == 0)


def test_boundary_matrix_rows():
    prob = O.Problem(dims=2, n_coeff=11, n_steps=20, horizon=5.0, n_obs=0, bc_mask=O.BC_DEFAULT)
    A = prob.A()
    assert A.shape == (8, 22)
    np.testing.assert_array_equal(A[0, :11], prob.P[0])
    np.testing.assert_array_equal(A[3, :11], prob.P[-1])
    np.testing.assert_array_equal(A[4:, 11:], A[:4, :11])
    bc = np.array([[1, 2, 3, 4, 5, 6], [7, 8, 9, 10, 11, 12]], float)
    np.testing.assert_array_equal(prob.b_eq(bc), [1, 2, 3, 4, 7, 8, 9, 10])
    rest = O.Problem(dims=2, n_coeff=11, n_steps=20, horizon=5.0, n_obs=0, bc_mask=O.BC_REST)
    assert rest.A().shape == (12, 22)
