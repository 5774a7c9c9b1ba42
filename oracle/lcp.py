"""Linear complementarity problems of the contact forces (oracle).  TEST INFRASTRUCTURE ONLY.

Eq. 12-13 ask for contact forces y >= 0 and gaps w >= 0 with y_i w_i = 0.  After
eliminating the displacement increment, the gaps are affine in the forces,
w = q + W y, which is the LCP(q, W).

* ``lemke``: Lemke's complementary pivoting method with an all-ones covering
  vector and lexicographic ratio tests against cycling (Cottle, Pang & Stone,
  The Linear Complementarity Problem, 1992, Sec. 4.4).
* ``enumerate_lcp``: brute force over all 2^n complementary index sets, for
  small n, as an independent check.
"""
from __future__ import annotations

import itertools
import numpy as np


class LCPFailure(RuntimeError):
    pass


def lemke(W, q, max_pivots=None):
    """Solve w = q + W y, y >= 0, w >= 0, y.w = 0.  Returns y."""
    W = np.asarray(W, float)
    q = np.asarray(q, float)
    n = q.size
    if n == 0 or np.all(q >= 0.0):
        return np.zeros(n)
    if max_pivots is None:
        max_pivots = 50 * (n + 1) ** 2
    # tableau rows: I w - W y - 1 z0 = q ; columns [w(0..n-1) | y(n..2n-1) | z0(2n)]
    Tab = np.zeros((n, 2 * n + 1))
    Tab[:, :n] = np.eye(n)
    Tab[:, n:2 * n] = -W
    Tab[:, 2 * n] = -1.0
    rhs = q.copy()
    basis = list(range(n))          # w basic
    z0 = 2 * n

    def pivot(r, col):
        nonlocal rhs
        piv = Tab[r, col]
        Tab[r, :] /= piv
        rhs[r] /= piv
        for i in range(n):
            if i != r and Tab[i, col] != 0.0:
                f = Tab[i, col]
                Tab[i, :] -= f * Tab[r, :]
                rhs[i] -= f * rhs[r]
        basis[r] = col

    def lex_less(u, v):
        # lexicographic u < v where components closer than the rounding level count as
        # equal: ties of the ratio test are exact in exact arithmetic (a degenerate basis
        # with zero right-hand sides) and must be broken by the B^-1 rows, not by noise
        for a, b in zip(u, v):
            if abs(a - b) > 1e-12 * (1.0 + max(abs(a), abs(b))):
                return a < b
        return False

    def lex_ratio(col, rows):
        # lexicographic minimum of (rhs_i, B^-1 row i) / a_i among rows with a_i > 0;
        # B^-1 is the tableau block under the initial basis (the w columns)
        best = None
        best_key = None
        for i in rows:
            a = Tab[i, col]
            key = np.concatenate([[rhs[i]], Tab[i, :n]]) / a
            if best is None or lex_less(key, best_key):
                best, best_key = i, key
        return best

    # initial pivot: z0 enters and the row of the most negative q leaves; among
    # equal q the highest row index keeps every row lexicographically positive
    qmin = np.min(rhs)
    r = max(i for i in range(n) if rhs[i] == qmin)
    leaving = basis[r]
    pivot(r, z0)
    entering = leaving + n if leaving < n else leaving - n
    for _ in range(max_pivots):
        col = entering
        rows = [i for i in range(n) if Tab[i, col] > 1e-14 * max(1.0, np.max(np.abs(Tab[:, col])))]
        if not rows:
            raise LCPFailure("ray termination")
        r = lex_ratio(col, rows)
        leaving = basis[r]
        pivot(r, col)
        if leaving == z0:
            break
        entering = leaving + n if leaving < n else leaving - n
    else:
        raise LCPFailure("pivot limit")
    y = np.zeros(n)
    for i, b in enumerate(basis):
        if n <= b < 2 * n:
            y[b - n] = rhs[i]
    return np.maximum(y, 0.0)


def enumerate_lcp(W, q, tol=1e-12):
    """All solutions y of LCP(q, W) found by testing every complementary index set."""
    W = np.asarray(W, float)
    q = np.asarray(q, float)
    n = q.size
    sols = []
    for k in range(n + 1):
        for alpha in itertools.combinations(range(n), k):
            a = list(alpha)
            y = np.zeros(n)
            if a:
                try:
                    y[a] = np.linalg.solve(W[np.ix_(a, a)], -q[a])
                except np.linalg.LinAlgError:
                    continue
            w = q + W @ y
            scale = tol * (1.0 + np.max(np.abs(q)))
            if np.all(y >= -scale) and np.all(w >= -scale):
                sols.append(y)
    return sols


def lcp_residual(W, q, y):
    """max(|min(y, w)|) - zero exactly at an LCP solution."""
    w = q + W @ y
    return float(np.max(np.abs(np.minimum(y, w)))) if y.size else 0.0
