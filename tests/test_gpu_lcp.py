"""GPU parity of the device LCP routines (fem_lcp) and of the wide contact path.

fem_lcp runs the routines fem_solve applies to a robot's contact set on a given W: the
LDS active set (m <= 64), the wavefront active set with the factor in LDS (m > 64), and
its rerun with the factor in device memory once the active set outgrows 128 positions.
Each is compared with the oracle's Lemke method on seeded symmetric positive definite
problems; the contact forces of such an LCP are unique, so they are compared entry by
entry (1e-10 relative) and the active sets exactly.
"""
import numpy as np
import pytest

from oracle import lcp, solver
from workloads import robots_for_config, load_schedule
from workloads.lumen import straight_cylinder_mesh
from tests.gpu_helpers import gpu_context, oracle_robots, displacement_error, compare_contact_keys, node_forces

pytestmark = pytest.mark.gpu


def _problem(m, q_shift, seed):
    """W = M M^T / k + I/2 (condition number below ~10) and q ~ N(q_shift, 1)."""
    rng = np.random.default_rng([m, seed])
    k = m + 8
    M = rng.normal(size=(m, k))
    W = M @ M.T / k + 0.5 * np.eye(m)
    q = rng.normal(size=m) + q_shift
    return W, q


@pytest.mark.parametrize("m,q_shift,path", [
    (1, -0.5, 0), (9, 0.0, 0), (64, 0.0, 0),        # LDS active set
    (65, 0.3, 1), (200, 0.6, 1), (200, 0.2, 1),     # factor in LDS (active sets up to 128)
    (300, -0.2, 2), (700, 0.2, 2),                  # active set beyond 128: factor in HBM
])
def test_lcp_routines_match_lemke(m, q_shift, path):
    from paper_2503_06922_amd import fem
    for seed in range(2):
        W, q = _problem(m, q_shift, seed)
        y, p = fem.fem_lcp(W, q)
        yo = lcp.lemke(W, q)
        assert lcp.lcp_residual(W, q, yo) <= 1e-10
        assert p == path, (m, p, int(np.sum(yo > 0)))
        assert np.array_equal(y > 0, yo > 1e-12), (m, seed)
        assert np.abs(y - yo).max() <= 1e-10 * max(np.abs(yo).max(), 1.0), (m, seed)


def test_lcp_edge_cases():
    from paper_2503_06922_amd import fem
    # q >= 0: the zero solution, on every path
    for m in (3, 100):
        W, _ = _problem(m, 0.0, 5)
        y, _ = fem.fem_lcp(W, np.abs(np.linspace(0.1, 1.0, m)))
        assert np.all(y == 0.0)
    # every constraint active: y = -W^-1 q
    W, _ = _problem(150, 0.0, 6)
    q = -W @ np.full(150, 0.25)
    y, p = fem.fem_lcp(W, q)
    assert p == 2 and np.abs(y - 0.25).max() <= 1e-12
    with pytest.raises(fem.FemError) as e:
        fem.fem_lcp(np.eye(1025), np.zeros(1025))
    assert e.value.status == fem.FEM_E_INVAL


def test_wide_contact_set_trajectory_matches_oracle():
    """60 elements in a 3 mm straight tube, base 0.6 mm off the axis: every node lies
    within the detection band of about three facets, 124-143 contacts per Newton
    iterate (beyond the 64 of the LDS path), through a 20-step tension ramp."""
    rb = robots_for_config(0)
    rb.n_elem[:] = 60
    rb.base_pos[0] = [0.6e-3, 0.0, 0.0]
    rb.tensions[0] = [2.0, 0.5, 0.0]
    V, T = straight_cylinder_mesh(radius=3e-3, axis_xy=(0.0, 0.0))
    robs, _ = oracle_robots(rb, V, T)
    rob = robs[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(rb, k))
    P, R, traj = solver.solve_robot(rob, sched, rb.n_load_steps, tol=1e-10, stag_tol=1e-9)
    ctx = gpu_context(rb, V, T, newton_tol=1e-10, stag_tol=1e-9, max_newton=100,
                      contact_capacity=256)
    Pref, _ = rob.reference()
    wide = 0
    for k in range(1, rb.n_load_steps + 1):
        d, t = load_schedule(rb, k)
        ctx.fem_set_actuation(0, t.ravel(), d)
        out = ctx.fem_solve(1)
        o = traj[k - 1]
        assert out["info"][0]["status"] == 0 and o["info"]["status"] == solver.OK
        wide += out["info"][0]["n_contacts"] > 64
        Pg = out["state"][:, 0:3]
        assert displacement_error(Pg, o["P"], Pref) <= 1e-9, k
        gc = ctx.fem_contacts(0)
        compare_contact_keys(gc, list(zip(o["contacts"], o["y"])), o["P"], rob)
        fg = node_forces(gc, Pg.shape[0])
        fo = node_forces([dict(c, force=y) for c, y in zip(o["contacts"], o["y"])], Pg.shape[0])
        assert np.abs(fg - fo).max() <= 1e-7 * max(np.abs(fo).max(), 1e-12) + 1e-13
    assert wide == rb.n_load_steps


def _singular_problem(m, r, seed):
    """W = B B^T / r of rank r < m (more constraints than independent directions, as when
    several contacts share a node) and q = w* - W y* from a complementary pair with y* > 0 on
    r + 3 constraints: solvable, and no solution's active set is independent of the rest."""
    rng = np.random.default_rng([m, r, seed])
    B = rng.normal(size=(m, r))
    W = B @ B.T / r
    S = rng.permutation(m)[: r + 3]
    y = np.zeros(m)
    y[S] = rng.uniform(0.2, 1.0, size=len(S))
    w = rng.uniform(0.1, 1.0, size=m)
    w[S] = 0.0
    return W, w - W @ y


@pytest.mark.parametrize("m,r,path", [(9, 4, 0), (40, 12, 0), (100, 30, 1), (700, 200, 2)])
def test_lcp_routines_semidefinite_W(m, r, path):
    """Singular W: y is not unique, but w = W y + q is (a convex QP's gradient is constant on
    its optimal set); the routines must exchange dependent constraints instead of failing."""
    from paper_2503_06922_amd import fem
    for seed in range(2):
        W, q = _singular_problem(m, r, seed)
        y, p = fem.fem_lcp(W, q)
        yo = lcp.lemke(W, q)
        assert p == path, (m, p)
        scale = max(np.abs(q).max(), 1.0)
        w, wo = W @ y + q, W @ yo + q
        assert np.all(y >= 0.0)
        assert w.min() >= -1e-10 * scale, (m, seed, w.min())
        assert np.max(y * np.abs(w)) <= 1e-10 * scale * max(y.max(), 1.0), (m, seed)
        assert np.abs(w - wo).max() <= 1e-9 * scale, (m, seed, np.abs(w - wo).max())
