"""Pins of the oracle's LCP solver against brute-force enumeration and KKT conditions."""
import itertools

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


def _brute_force_w(W, q, tol=1e-9):
    """Every complementary index set a of LCP(q, W) with a least-squares y_a >= 0 that
    solves W_aa y_a = -q_a and leaves w >= 0: the gap vectors w = q + W y it yields.
    Works for singular (semidefinite) W, where y is not unique."""
    n = q.size
    scale = tol * (1.0 + np.abs(q).max())
    ws = []
    for k in range(n + 1):
        for a in itertools.combinations(range(n), k):
            a = list(a)
            y = np.zeros(n)
            if a:
                y[a] = np.linalg.lstsq(W[np.ix_(a, a)], -q[a], rcond=None)[0]
                if np.abs(W[np.ix_(a, a)] @ y[a] + q[a]).max() > scale:
                    continue
            w = q + W @ y
            if np.all(y >= -scale) and np.all(w >= -scale):
                ws.append(w)
    return ws


@pytest.mark.parametrize("n,r", [(3, 1), (4, 2), (6, 3), (8, 5)])
def test_lemke_semidefinite_w_matches_enumeration(n, r):
    """Rank-deficient W = B^T B (more contacts at a node than it has directions): the forces
    y are not unique, but w = q + W y is; Lemke's y must be a solution with that w."""
    rng = np.random.default_rng(100 + n)
    for _ in range(10):
        B = rng.normal(size=(r, n))
        W = B.T @ B
        # a solvable problem: pick a complementary pair (y*, w*) and set q = w* - W y*
        act = rng.random(n) < 0.5
        ys = np.where(act, rng.random(n), 0.0)
        ws = np.where(act, 0.0, rng.random(n))
        q = ws - W @ ys
        y = lcp.lemke(W, q)
        w = q + W @ y
        assert np.all(y >= 0.0) and w.min() >= -1e-11
        assert np.abs(y * w).max() <= 1e-11
        sols = _brute_force_w(W, q)
        assert sols, "enumeration found no solution"
        for wb in sols:
            assert np.allclose(wb, w, atol=1e-9 * (1 + np.abs(q).max()))
