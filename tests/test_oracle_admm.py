"""Pins of the oracle's ADMM (OSQP iteration) solution of the linear step's QP.

The iteration (oracle/admm.py) must reach the unique solution of the strictly convex QP
min 1/2 x^T K x - b^T x, A x + g >= 0: checked on small random problems against brute-force
enumeration of the active sets (each a linear KKT system), and against the exact linear step
of the Newton iteration; and a whole Newton trajectory with ADMM steps must end in the
equilibria of the exact one (the QP only decides the iteration path, not the equilibrium).
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle import admm, beam, collision, solver, lcp
from workloads import make_config, load_schedule


def _banded(K):
    n = K.shape[0]
    ab = np.zeros((12, n))
    for d in range(12):
        ab[11 - d, d:] = np.diagonal(K, offset=d)
    return ab


def _brute_force(K, b, A, g):
    """Enumerate active sets: x = K^-1 (b + A_S^T y_S) with A_S x + g_S = 0; keep the one with
    y >= 0 and A x + g >= 0."""
    m = A.shape[0]
    for k in range(m + 1):
        for S in itertools.combinations(range(m), k):
            S = list(S)
            n = K.shape[0]
            M = np.zeros((n + k, n + k))
            M[:n, :n] = K
            M[:n, n:] = -A[S].T
            M[n:, :n] = A[S]
            rhs = np.concatenate([b, -g[S]])
            sol = np.linalg.solve(M, rhs)
            x, yS = sol[:n], sol[n:]
            y = np.zeros(m)
            y[S] = yS
            if np.all(yS >= -1e-12) and np.all(A @ x + g >= -1e-12):
                return x, y
    raise AssertionError("no active set")


@pytest.mark.parametrize("seed", range(4))
def test_admm_qp_matches_active_set_enumeration(seed):
    """Block-tridiagonal SPD K (bandwidth 11) of 5 nodes, 4 contact rows on node
    translations; the ADMM iterate within its tolerance of the enumerated solution."""
    rng = np.random.default_rng([7, seed])
    n = 30
    M = rng.normal(size=(n, n))
    K = M @ M.T / n + np.eye(n)
    K[np.abs(np.subtract.outer(np.arange(n), np.arange(n))) > 11] = 0.0
    K += 2.0 * np.eye(n)                       # keep it definite after the banding
    assert np.all(np.linalg.eigvalsh(K) > 0)
    b = rng.normal(size=n)
    m = 4
    A = np.zeros((m, n))
    for c in range(m):
        node = rng.integers(0, 5)
        v = rng.normal(size=3)
        A[c, 6 * node:6 * node + 3] = v / np.linalg.norm(v)
    g = rng.normal(size=m) * 0.3
    xe, ye = _brute_force(K, b, A, g)
    x, y, it, ok = admm.admm_qp(_banded(K), b, A, g, [], rho=1.0, eps_abs=1e-12, eps_rel=1e-12,
                                max_iter=200000)
    assert ok
    assert np.abs(x - xe).max() <= 1e-8 * max(1.0, np.abs(xe).max())
    assert np.abs(y - ye).max() <= 1e-8 * max(1.0, np.abs(ye).max())


def test_admm_linear_step_matches_exact_step():
    """A linear step of the straight-tube robot with active contacts: the ADMM step agrees
    with the exact one (banded Cholesky + Schur complement + Lemke) to its tolerance."""
    rb, V, T = make_config(0)
    rob = solver.robots_from_batch(rb, collision.Mesh(V, T))[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(rb, k))
    P, R, _ = solver.solve_robot(rob, sched, 11, tol=1e-10, stag_tol=1e-9, max_iter=60)
    d, t = sched(12)
    F = solver.out_of_balance(rob, P, R, 0, t)
    cont = solver.detect(rob, P, None, None)
    assert len(cont) >= 3
    ab = beam.tangent_qp_upper_banded(P, R, rob.K12)
    dXe, ye, _ = solver.linear_step(rob, P, R, F, ab, rob.base_target(d), cont, None, beta=1e9)
    dXa, ya, _, it = admm.linear_step_admm(rob, P, R, F, ab, rob.base_target(d), cont, None, beta=1e9,
                                            rho=1.0, eps=1e-13, max_iter=200000)
    # contact forces at a node are unique (several rows on a node may split them)
    fe = np.zeros((rob.n_elem + 1, 3))
    fa = np.zeros((rob.n_elem + 1, 3))
    for c, ct in enumerate(cont):
        fe[ct["node"]] += ye[c] * ct["n"]
        fa[ct["node"]] += ya[c] * ct["n"]
    assert np.abs(dXa - dXe).max() <= 1e-7 * np.abs(dXe).max()
    assert np.abs(fa - fe).max() <= 1e-7 * np.abs(fe).max()


def test_admm_newton_reaches_the_exact_equilibria():
    """The straight-tube robot through its 20-step tension ramp with ADMM linear steps
    (tolerance 1e-11) ends every load step in the equilibrium of the exact method: both stop
    at a residual below 1e-10 N, which fixes positions to within the robot's compliance
    (a cantilever, L^3 / 3 EI = 56 m/N) times the two residuals."""
    rb, V, T = make_config(0)
    rob = solver.robots_from_batch(rb, collision.Mesh(V, T))[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(rb, k))
    _, _, te = solver.solve_robot(rob, sched, 20, tol=1e-10, stag_tol=1e-9, max_iter=100)
    _, _, ta = solver.solve_robot(rob, sched, 20, tol=1e-10, stag_tol=1e-9, max_iter=100,
                                  qp=dict(rho=1.0, eps=1e-11))
    P0 = rob.reference()[0]
    scale = max(np.linalg.norm(s["P"] - P0, axis=1).max() for s in te)
    EI = float(np.min(rob.EI))
    C = rob.length ** 3 / (3.0 * EI)
    for se, sa in zip(te, ta):
        assert se["info"]["status"] == sa["info"]["status"] == solver.OK
        bound = 1e-9 * scale + C * (se["info"]["res_norm"] + sa["info"]["res_norm"])
        assert np.linalg.norm(se["P"] - sa["P"], axis=1).max() <= bound
        assert sa["info"]["qp_iters"] > 0
