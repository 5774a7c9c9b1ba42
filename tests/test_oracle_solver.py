"""Pins of the oracle's Newton/QP iteration: KKT of each linear step, the step limit,
and equilibrium conditions (complementarity, global balance) on the straight-tube workload."""
import numpy as np
import pytest

from oracle import solver, collision, beam, actuation, lcp
from workloads import make_config, load_schedule


@pytest.fixture(scope="module")
def cfg0():
    rb, V, T = make_config(0)
    mesh = collision.Mesh(V, T)
    rob = solver.robots_from_batch(rb, mesh)[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(rb, k))
    P, R, traj = solver.solve_robot(rob, sched, rb.n_load_steps, tol=1e-13, stag_tol=1e-9)
    return rb, rob, traj


def test_cfg0_all_steps_converge_with_contacts(cfg0):
    rb, rob, traj = cfg0
    assert len(traj) == rb.n_load_steps
    assert all(t["info"]["status"] == solver.OK for t in traj)
    assert max(int(np.sum(t["y"] > 0)) for t in traj) >= 1


def test_cfg0_equilibrium_conditions(cfg0):
    rb, rob, traj = cfg0
    for k, t in enumerate(traj, start=1):
        P, R, cont, y = t["P"], t["R"], t["contacts"], t["y"]
        _, T = load_schedule(rb, k)
        F = solver.out_of_balance(rob, P, R, actuation.CABLES, T[0])
        r = solver.contact_residual(F, cont, y)
        assert np.linalg.norm(r) <= 1e-9
        gaps = np.array([c["gap"] for c in cont])
        # Signorini: y >= 0, g >= 0 (to 1e-9 m), y g = 0 (eq. 12-13)
        assert np.all(y >= 0)
        if gaps.size:
            assert gaps.min() >= -1e-9
            assert np.abs(y * gaps).max() <= 1e-12
        # global balance: base reaction + contact forces + actuation = 0 (forces and moments)
        fa = actuation.load_vector(R, actuation.CABLES, T[0], rob.cable_radius, rob.cable_angle)
        fint = beam.internal_forces(P, R, rob.l0, rob.K7)
        # the clamp's reaction on the robot equals the internal force at the base node
        ext_f = fint[0, 0:3] + fa[-1, 0:3]
        ext_m = fint[0, 3:6] + np.cross(P[0], fint[0, 0:3]) + fa[-1, 3:6] + np.cross(P[-1], fa[-1, 0:3])
        for c, yy in zip(cont, y):
            ext_f += yy * c["n"]
            ext_m += np.cross(P[c["node"]], yy * c["n"])
        assert np.abs(ext_f).max() <= 1e-9
        assert np.abs(ext_m).max() <= 1e-9


def test_linear_step_is_qp_optimal(cfg0):
    """dx solves eq. 23: K dx + r = A^T y, y >= 0, g + A dx >= 0, y (g + A dx) = 0."""
    rb, rob, traj = cfg0
    P, R = traj[4]["P"], traj[4]["R"]
    _, T = load_schedule(rb, 7)
    F = solver.out_of_balance(rob, P, R, actuation.CABLES, T[0])
    cont = solver.detect(rob, P)
    assert len(cont) >= 1
    ab = beam.tangent_qp_upper_banded(P, R, rob.K12)
    big = solver.Robot(**{**{k: getattr(rob, k) for k in ("n_elem", "length", "base_pos", "base_dir",
                                                           "base_up", "EA", "EI", "GJ", "cable_radius",
                                                           "cable_angle", "r_c", "delta", "guide_len",
                                                           "mesh")}, "beta0": 1.0})
    dX, y, lim = solver.linear_step(big, P, R, F, ab, rob.base_target(0.0), cont)
    assert not lim
    N = P.shape[0]
    K = beam.upper_banded_to_dense(ab, 6 * N)[6:, 6:]
    A = np.zeros((len(cont), 6 * (N - 1)))
    for c, ct in enumerate(cont):
        A[c, 6 * (ct["node"] - 1):6 * (ct["node"] - 1) + 3] = ct["n"]
    g = np.array([c["gap"] for c in cont])
    dx = dX[1:].ravel()
    stat = K @ dx + F[1:].ravel() - A.T @ y
    assert np.abs(stat).max() <= 1e-10 * max(1.0, np.abs(F).max())
    w = g + A @ dx
    assert np.all(y >= 0) and w.min() >= -1e-15
    assert np.abs(y * w).max() <= 1e-16


def test_step_limit_scales_step_and_multipliers(cfg0):
    rb, rob, traj = cfg0
    P, R = rob.reference()
    _, T = load_schedule(rb, 20)
    F = solver.out_of_balance(rob, P, R, actuation.CABLES, T[0])
    ab = beam.tangent_qp_upper_banded(P, R, rob.K12)
    big = solver.Robot(**{**{k: getattr(rob, k) for k in ("n_elem", "length", "base_pos", "base_dir",
                                                           "base_up", "EA", "EI", "GJ", "cable_radius",
                                                           "cable_angle", "r_c", "delta", "guide_len",
                                                           "mesh")}, "beta0": 10.0})
    dX_full, _, lim_full = solver.linear_step(big, P, R, F, ab, rob.base_target(0.0), [])
    dX, _, lim = solver.linear_step(rob, P, R, F, ab, rob.base_target(0.0), [])
    assert not lim_full and lim
    nrm = np.max(np.linalg.norm(dX[:, 0:3], axis=1))
    assert nrm == pytest.approx(rob.beta0, rel=1e-15)
    f = rob.beta0 / np.max(np.linalg.norm(dX_full[:, 0:3], axis=1))
    assert np.allclose(dX, f * dX_full, rtol=1e-15, atol=0)


def test_guide_holds_lateral_position():
    rb, V, T = make_config(1)
    rob = solver.robots_from_batch(rb, None)[0]       # no lumen: guide only
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(rb, k))
    P, R, traj = solver.solve_robot(rob, sched, 5, tol=1e-10)
    assert all(t["info"]["status"] == solver.OK for t in traj)
    d, _ = load_schedule(rb, 5)
    g = rob.guided(d[0])
    assert g.sum() > 0
    assert np.abs(P[g, 0:2] - rob.base_pos[0:2]).max() <= 1e-15
    assert P[0, 2] == pytest.approx(rob.base_pos[2] + d[0], abs=1e-15)


def test_literal_cable_force_reading_makes_qp_iteration_diverge():
    """Evidence for the actuation reading: applying the summed cable pull as an external
    compressive follower force (~10^2-10^3 Euler loads here) makes the paper's symmetric
    QP-tangent iteration diverge (spectral radius of I - K^-1 J above 1) already at 1/20
    of the configured tensions; the follower moment alone keeps it far below 1."""
    rb, V, T = make_config(0)
    rob = solver.robots_from_batch(rb, None)[0]
    Tn = rb.tensions[0] / 20.0
    P, R = rob.reference()
    N = P.shape[0]

    def rho(resid):
        J = beam.banded_to_dense(beam.fd_jacobian_banded(resid, P, R), 6 * N)[6:, 6:]
        K = beam.upper_banded_to_dense(beam.tangent_qp_upper_banded(P, R, rob.K12), 6 * N)[6:, 6:]
        return np.abs(np.linalg.eigvals(np.eye(J.shape[0]) - np.linalg.solve(K, J))).max()

    def literal(P_, R_):
        F = beam.internal_forces(P_, R_, rob.l0, rob.K7)
        F[-1] -= actuation.literal_cable_wrench(R_[-1], Tn, rob.cable_radius, rob.cable_angle)
        return F

    model = lambda P_, R_: solver.out_of_balance(rob, P_, R_, actuation.CABLES, Tn)
    assert rho(literal) > 1.0
    assert rho(model) < 0.2


def test_convex_ridge_fallback_keeps_node_constrained():
    """Two triangles meeting at a convex ridge: a node whose centre lies over the ridge,
    r_c off the wall, is in neither face region and must still get the edge contact."""
    V = np.array([[0, -0.01, 0], [0, 0.01, 0], [-0.01, 0, -0.002], [0.01, 0, -0.002]], float)
    T = np.array([[0, 1, 2], [1, 0, 3]])
    m = collision.Mesh(V, T)
    assert m.n[0][2] > 0 and m.n[1][2] > 0
    p = np.array([0.0, 0.0, 1.6e-3])
    c = collision.detect(np.array([[0, 0, -1.0], p]), m, 1.5e-3, 1e-3)
    assert len(c) == 1 and c[0]["kind"] == 1
    assert np.allclose(c[0]["n"], [0, 0, 1]) and c[0]["gap"] == pytest.approx(0.1e-3, abs=1e-15)
