"""Pins of the oracle's Newton/QP iteration: KKT of each linear step, the step limit,
and equilibrium conditions (complementarity, global balance) on the straight-tube workload."""
import numpy as np
import scipy.spatial.transform
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


def _scripted_loop(monkeypatch, rob, contact_sets, residuals, limited=None, tol=1e-14):
    """Run solve_load_step with detection, residual and linear step replaced by scripts:
    iterate k detects contact_sets[k], sees residual norm residuals[k] and takes a zero
    step (limited[k]).  Returns (betas passed to the linear step, info)."""
    betas = []
    k = {"det": 0, "res": 0, "lin": 0}
    N = rob.n_elem + 1

    def fake_detect(robot, P, guided=None, prev=None):
        i = min(k["det"], len(contact_sets) - 1)
        k["det"] += 1
        return [dict(node=n, tri=t, kind=0, n=np.array([0.0, 0.0, 1.0]), gap=1e-3)
                for n, t in contact_sets[i]]

    def fake_residual(F, contacts, y, robot=None, guided=None):
        i = min(k["res"], len(residuals) - 1)
        k["res"] += 1
        r = np.zeros((N - 1, 6))
        r[0, 0] = residuals[i]
        return r

    def fake_step(robot, P, R, F, ab, base_target, contacts, guided=None, beta=None):
        betas.append(beta)
        i = k["lin"]
        k["lin"] += 1
        lim = bool(limited[i]) if limited is not None and i < len(limited) else False
        return np.zeros((N, 6)), np.zeros(len(contacts)), lim

    monkeypatch.setattr(solver, "detect", fake_detect)
    monkeypatch.setattr(solver, "contact_residual", fake_residual)
    monkeypatch.setattr(solver, "linear_step", fake_step)
    P, R = rob.reference()
    *_, info = solver.solve_load_step(rob, P, R, rob.base_target(0.0), actuation.CABLES,
                                      np.zeros(3), tol=tol, stag_tol=1e-9, max_iter=75)
    return betas, info


def _plain_robot():
    rb, _, _ = make_config(0)
    return solver.robots_from_batch(rb, None)[0]


def test_step_limit_halves_every_ten_contact_set_changes(monkeypatch):
    """The step limit is beta0 until the detected contact set has changed 10 times within
    the load step, then beta0/2 until 20 changes, ... and never below beta0/64 (reading of
    the unstated beta of eq. 25-26)."""
    rob = _plain_robot()
    sets = [[(5, 0)] if k % 2 == 0 else [(6, 1)] for k in range(80)]   # a change every iterate
    betas, info = _scripted_loop(monkeypatch, rob, sets, [1.0])
    assert info["status"] == solver.NOCONV and len(betas) == 75
    b0 = rob.beta0
    expected = ([b0] * 10 + [b0 / 2] * 10 + [b0 / 4] * 10 + [b0 / 8] * 10 + [b0 / 16] * 10
                + [b0 / 32] * 10 + [b0 / 64] * 15)
    assert betas == expected
    # a fixed contact set never halves
    betas, _ = _scripted_loop(monkeypatch, rob, [[(5, 0)]], [1.0])
    assert betas == [b0] * 75


def test_stagnation_acceptance(monkeypatch):
    """A residual below the stagnation level is accepted once it stops halving; while it
    still halves, or above the level, the iteration goes on; below tol it stops at once;
    a limited last step is never accepted."""
    rob = _plain_robot()
    stag = solver.stagnation_tol(rob, 1e-9)
    assert stag >= 1e-9
    same = [[(5, 0)]]
    # the first residual is seen at iterate 1 (iterate 0 has no previous step)
    seq = [None, 1e-3, 1e-6, 0.4 * stag, 0.3 * stag]            # accepted at the 4th
    _, info = _scripted_loop(monkeypatch, rob, same, seq[1:])
    assert info["status"] == solver.OK and info["iters"] == 4
    seq = [1e-3, 0.9 * stag, 0.4 * stag, 0.15 * stag, 0.07 * stag, 0.06 * stag]
    _, info = _scripted_loop(monkeypatch, rob, same, seq)     # halving until the last
    assert info["status"] == solver.OK and info["iters"] == 6
    _, info = _scripted_loop(monkeypatch, rob, same, [1e-3, 2.0 * stag])   # never below
    assert info["status"] == solver.NOCONV
    _, info = _scripted_loop(monkeypatch, rob, same, [1e-3, 5e-11], tol=1e-10)  # below tol
    assert info["status"] == solver.OK and info["iters"] == 2
    _, info = _scripted_loop(monkeypatch, rob, same, [1e-3, 5e-11, 5e-11], tol=1e-10,
                             limited=[False, True, False])
    assert info["status"] == solver.OK and info["iters"] == 3
    # a changing contact set is never accepted, whatever the residual
    _, info = _scripted_loop(monkeypatch, rob, [[(5, 0)], [(6, 0)]], [1e-12], tol=1e-10)
    assert info["status"] == solver.OK and info["iters"] == 2


def test_stagnation_level_lies_above_the_rounding_floor():
    """The out-of-balance force of a stress-free robot moved rigidly to coordinates of
    order 1 m is pure rounding; the stagnation level must exceed it (or a stagnating
    iteration at that floor would never be accepted) without being loose by more than
    about three orders of magnitude."""
    rb, _, _ = make_config(3, n_robots=8)
    rng = np.random.default_rng(3)
    for rob in solver.robots_from_batch(rb, None):
        P, R = rob.reference()
        for _ in range(3):
            Q = scipy.spatial.transform.Rotation.random(random_state=rng).as_matrix()
            t = rng.uniform(-1.0, 1.0, 3)
            P2 = P @ Q.T + t
            R2 = np.einsum("ij,njk->nik", Q, R)
            F = beam.internal_forces(P2, R2, rob.l0, rob.K7)
            floor = float(np.linalg.norm(F[1:]))
            level = solver.stagnation_tol(rob, 0.0)
            assert floor < level, (floor, level)
            assert level < 3e3 * max(floor, 1e-300) or floor == 0.0
