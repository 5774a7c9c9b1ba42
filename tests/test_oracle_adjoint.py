"""Pins of the oracle adjoint gradient (dL/du at a converged equilibrium).

1. Closed forms at the unloaded straight cantilever: with the tip wrench as u and
   L = a sensor's position component, dL/du is a column of the flexibility of an
   Euler-Bernoulli cantilever (exact at the nodes for cubic Hermite elements):
   y(a) under a tip force F_y is F a^2 (3L - a) / (6 EI), under a tip moment M_z it
   is M a^2 / (2 EI), axial x(a) under F_x is F a / EA.
2. Central differences of complete re-solves (forward solver pinned elsewhere) at
   a loaded state with active lumen contacts and the follower cable moment, where
   the Jacobian is not symmetric.
"""
import numpy as np
import pytest

from oracle import actuation, adjoint, beam, collision, solver
from workloads import make_config


def cantilever(n_e=10, L=0.3):
    EA, EI, GJ = beam.section_stiffness(1.5e-3, 1e-3, 50e6, 0.45)
    return solver.Robot(n_e, L, np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 1.0, 0]),
                        EA, EI, GJ, 1.2e-3, np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3]),
                        1.5e-3, 1e-3, 1e-3), EA, EI


@pytest.mark.parametrize("node", [10, 4])
def test_adjoint_flexibility_closed_form(node):
    rob, EA, EI = cantilever()
    P, R = rob.reference()
    a = node * rob.l0
    L = rob.length
    for axis, expect in ((1, dict(f=(1, a * a * (3 * L - a) / (6 * EI)), m=(5, a * a / (2 * EI)))),
                         (0, dict(f=(0, a / EA)))):
        dLdp = np.zeros((1, 3))
        dLdp[0, axis] = 1.0
        g = adjoint.tension_gradient(rob, P, R, [], np.zeros(0), np.zeros(6), [node], dLdp,
                                     act_kind=actuation.TIP_GLOBAL)
        ref = np.zeros(6)
        for idx, val in expect.values():
            ref[idx] = val
        assert np.allclose(g, ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())


def test_adjoint_cable_gradient_closed_form():
    """Cable tensions at zero load: dL/dT_j = (M_z flexibility) * (moment arm of cable j)."""
    rob, EA, EI = cantilever()
    P, R = rob.reference()
    dLdp = np.array([[0.0, 1.0, 0.0]])
    g = adjoint.tension_gradient(rob, P, R, [], np.zeros(0), np.zeros(3), [rob.n_elem], dLdp)
    # cable j's moment in the tip frame is rc (0, -sin, cos); about z its arm is rc cos(angle)
    # when the tip triad is the reference one (R = [e_x, e_y, e_z])
    Rt = R[-1]
    # eq. 16: M_j = d_j x F_j with the attachment d_j and the pull F_j = -e_x per unit tension
    m = np.array([Rt @ np.cross(rob.cable_radius * np.array([0.0, np.cos(t), np.sin(t)]),
                                [-1.0, 0.0, 0.0])
                  for t in rob.cable_angle])
    flex_M = np.array([0.0, 0.0, 0.0])  # tip y under M = (Mx, My, Mz): only Mz acts
    flex_M[2] = rob.length ** 2 / (2 * EI)
    assert np.allclose(g, m @ flex_M, rtol=1e-6, atol=1e-12)


def test_adjoint_matches_finite_difference_resolves():
    rb, V, T = make_config(0)
    mesh = collision.Mesh(V, T)
    rob = solver.robots_from_batch(rb, mesh)[0]
    Tf = rb.tensions[0]
    n_steps = 20

    def run(Tv):
        sched = lambda k: (0.0, Tv * k / n_steps)
        P, R, traj = solver.solve_robot(rob, sched, n_steps, tol=1e-13, stag_tol=1e-9, max_iter=300)
        assert all(t["info"]["status"] == solver.OK for t in traj)
        return P, R, traj[-1]

    P, R, last = run(Tf)
    assert int(np.sum(last["y"] > 0)) >= 2  # the pin must exercise the contact KKT
    sens = [rob.n_elem - 2, rob.n_elem]
    targets = P[sens] + np.array([[1e-3, -2e-3, 0.5e-3], [-1e-3, 1e-3, 2e-3]])
    _, dLdp = adjoint.sensor_loss(P, sens, targets)
    g = adjoint.tension_gradient(rob, P, R, last["contacts"], last["y"], Tf, sens, dLdp)
    h = 1e-6
    fd = np.zeros(3)
    for j in range(3):
        Tp, Tm = Tf.copy(), Tf.copy()
        Tp[j] += h
        Tm[j] -= h
        fd[j] = (adjoint.sensor_loss(run(Tp)[0], sens, targets)[0]
                 - adjoint.sensor_loss(run(Tm)[0], sens, targets)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max()


def test_adjoint_cable_wrench_matches_finite_difference_resolves():
    """Eq. 17 as printed (CABLE_WRENCH): the follower cable force adds a load stiffness and
    a force column to dF_a/dT; the adjoint must still match central differences of complete
    re-solves (a narrow tube, so that contacts are active, at tensions where the iteration
    of eq. 20-23 converges)."""
    from workloads.lumen import straight_cylinder_mesh
    rb, _, _ = make_config(0)
    V, T = straight_cylinder_mesh(radius=2.2e-3, axis_xy=(0.0, 0.2e-3))
    rob = solver.robots_from_batch(rb, collision.Mesh(V, T))[0]
    Tf = rb.tensions[0] * 0.01
    n_steps = 20

    def run(Tv):
        sched = lambda k: (0.0, Tv * k / n_steps)
        P, R, traj = solver.solve_robot(rob, sched, n_steps, act_kind=actuation.CABLE_WRENCH,
                                        tol=1e-13, stag_tol=1e-9, max_iter=300)
        assert all(t["info"]["status"] == solver.OK for t in traj)
        return P, R, traj[-1]

    P, R, last = run(Tf)
    assert int(np.sum(last["y"] > 0)) >= 1
    sens = [rob.n_elem - 4, rob.n_elem]
    targets = P[sens] + np.array([[1e-3, -2e-3, 0.5e-3], [-1e-3, 1e-3, 2e-3]])
    _, dLdp = adjoint.sensor_loss(P, sens, targets)
    g = adjoint.tension_gradient(rob, P, R, last["contacts"], last["y"], Tf, sens, dLdp,
                                 act_kind=actuation.CABLE_WRENCH)
    h = 1e-7
    fd = np.zeros(3)
    for j in range(3):
        Tp, Tm = Tf.copy(), Tf.copy()
        Tp[j] += h
        Tm[j] -= h
        fd[j] = (adjoint.sensor_loss(run(Tp)[0], sens, targets)[0]
                 - adjoint.sensor_loss(run(Tm)[0], sens, targets)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-5 * np.abs(fd).max()
