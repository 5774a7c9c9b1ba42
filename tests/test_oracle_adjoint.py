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


def _ridge_robot():
    """A 10-element cantilever along x whose node 2 rests on a convex ridge running along the
    robot (two triangles meeting at the line y = 0, z = -1.7 mm between x = 0.04 and 0.08 m):
    the node's centre lies over the ridge, in neither face region, so its contact is the
    edge fallback."""
    EA, EI, GJ = beam.section_stiffness(1.5e-3, 1e-3, 50e6, 0.45)
    zr = -1.7e-3
    V = np.array([[0.04, 0.0, zr], [0.08, 0.0, zr], [0.06, -0.01, zr - 0.002], [0.06, 0.01, zr - 0.002]])
    T = np.array([[0, 2, 1], [1, 3, 0]])
    m = collision.Mesh(V, T)
    assert m.n[0][2] > 0 and m.n[1][2] > 0
    return solver.Robot(10, 0.3, np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), EA, EI, GJ,
                        1.2e-3, np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3]), 1.5e-3, 1e-3, 1e-3, 0.0, m)


def test_edge_contact_normal_derivative_against_detection():
    """The constraint curvature of an edge/vertex contact, dn/dp = (I - n n^T - t t^T)/rho
    (edge) or (I - n n^T)/rho (vertex), against central differences of the normal that the
    detection itself returns at displaced node positions."""
    rob = _ridge_robot()
    m = rob.mesh
    # an edge point (over the ridge) and a vertex point (beyond the ridge's end)
    for p, tri in ((np.array([0.055, 1e-4, 0.1e-3]), 0), (np.array([0.0805, 2e-4, -1.2e-3]), 0)):
        det = collision.detect(np.array([[-1.0, 0, 0], p]), m, 1.5e-3, 1e-3)
        assert len(det) == 1 and det[0]["kind"] == 1
        H = adjoint.normal_derivative(p, m, det[0]["tri"])
        h = 1e-7
        fd = np.zeros((3, 3))
        for k in range(3):
            dp = np.zeros(3)
            dp[k] = h
            np_ = collision.detect(np.array([[-1.0, 0, 0], p + dp]), m, 1.5e-3, 1e-3)[0]["n"]
            nm_ = collision.detect(np.array([[-1.0, 0, 0], p - dp]), m, 1.5e-3, 1e-3)[0]["n"]
            fd[:, k] = (np_ - nm_) / (2 * h)
        assert np.abs(H - fd).max() <= 1e-6 * np.abs(H).max(), (H, fd)
        assert np.abs(H).max() > 100.0       # 1/rho with rho near 1.6 mm


def test_adjoint_edge_contact_matches_finite_difference_resolves():
    """A node pressed onto a convex ridge by a tip load: the edge contact's normal turns with
    the node, and the adjoint with that constraint curvature matches central differences of
    complete re-solves for every component of the tip wrench (the lateral ones move the node
    across the ridge); without it the lateral components are 14 % off.  The re-solves stop
    at a stagnating residual near 1e-10 N, which the compliant tip (56 m/N) turns into
    ~1e-8 m of noise against a response of ~6e-5 m at h = 1e-6 N, so the agreement is
    checked to 2e-4."""
    rob = _ridge_robot()
    u0 = np.array([0.0, 0.0, -3e-4, 0.0, 0.0, 0.0])
    n_steps = 10

    def run(u):
        sched = lambda k: (0.0, u * k / n_steps)
        P, R, traj = solver.solve_robot(rob, sched, n_steps, act_kind=actuation.TIP_GLOBAL, tol=1e-13,
                                        stag_tol=1e-9, max_iter=300)
        assert all(t["info"]["status"] == solver.OK for t in traj)
        return P, R, traj[-1]

    P, R, last = run(u0)
    act = [(c["node"], c["kind"]) for c, y in zip(last["contacts"], last["y"]) if y > 0]
    assert act == [(2, 1)]
    sens = [2, 10]
    targets = P[sens] + np.array([[1e-3, -2e-3, 0.5e-3], [-1e-3, 1e-3, 2e-3]])
    _, dLdp = adjoint.sensor_loss(P, sens, targets)
    g = adjoint.tension_gradient(rob, P, R, last["contacts"], last["y"], u0, sens, dLdp,
                                 act_kind=actuation.TIP_GLOBAL)
    h = 1e-6
    fd = np.zeros(6)
    for j in range(6):
        up, um = u0.copy(), u0.copy()
        up[j] += h
        um[j] -= h
        fd[j] = (adjoint.sensor_loss(run(up)[0], sens, targets)[0]
                 - adjoint.sensor_loss(run(um)[0], sens, targets)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 2e-4 * np.abs(fd).max(), (g, fd)
