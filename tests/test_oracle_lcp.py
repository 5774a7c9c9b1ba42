"""Pins of the oracle's LCP solver against brute-force enumeration and KKT conditions."""
import numpy as np
import pytest

from oracle import lcp


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_lemke_matches_enumeration_spd(n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        A = rng.normal(size=(n, n))
        W = A @ A.T + 0.1 * np.eye(n)
        q = rng.normal(size=n)
        y = lcp.lemke(W, q)
        sols = lcp.enumerate_lcp(W, q)
        assert len(sols) == 1
        assert np.allclose(y, sols[0], atol=1e-12 * (1 + np.abs(sols[0]).max()))
        assert lcp.lcp_residual(W, q, y) < 1e-12


def test_lemke_p_matrix_nonsymmetric():
    rng = np.random.default_rng(7)
    for _ in range(30):
        n = 6
        A = rng.normal(size=(n, n))
        W = A @ A.T + np.eye(n) + 0.3 * (rng.normal(size=(n, n)) - rng.normal(size=(n, n)))
        if np.any(np.linalg.eigvalsh(0.5 * (W + W.T)) <= 0):
            continue
        q = rng.normal(size=n)
        y = lcp.lemke(W, q)
        assert lcp.lcp_residual(W, q, y) < 1e-11
        sols = lcp.enumerate_lcp(W, q)
        assert len(sols) == 1 and np.allclose(y, sols[0], atol=1e-11)


def test_lemke_degenerate_ties():
    W = np.eye(3)
    q = np.array([-1.0, -1.0, -1.0])
    assert np.allclose(lcp.lemke(W, q), [1, 1, 1])
    q = np.array([-1.0, 0.0, 2.0])
    assert np.allclose(lcp.lemke(W, q), [1, 0, 0])
