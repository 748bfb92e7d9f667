"""Pins of the oracle's density-fitting solve d = V^{-1} gamma (test
infrastructure): a 3 x 3 system solved by hand, the residual and the
factorisation of a random symmetric positive definite matrix."""
import numpy as np

import oracle


def test_fit_coefficients_hand_solved_system():
    # V d = gamma with V = [[4,2,0],[2,5,1],[0,1,3]] and d = (1, -1, 2):
    # gamma = (4 - 2, 2 - 5 + 2, -1 + 6) = (2, -1, 5)
    V = np.array([[4.0, 2.0, 0.0], [2.0, 5.0, 1.0], [0.0, 1.0, 3.0]])
    d = oracle.fit_coefficients(V, np.array([2.0, -1.0, 5.0]))
    assert np.abs(d - np.array([1.0, -1.0, 2.0])).max() <= 1e-15


def test_fit_coefficients_residual_random_spd():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(90, 90))
    V = X @ X.T + 90 * np.eye(90)
    g = rng.normal(size=90)
    d = oracle.fit_coefficients(V, g)
    assert np.abs(V @ d - g).max() <= 1e-12 * np.abs(g).max()
    # the factor behind it reproduces V
    L = np.linalg.cholesky(V)
    assert np.abs(L @ L.T - V).max() <= 1e-13 * np.abs(V).max()
