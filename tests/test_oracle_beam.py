"""Pins of the oracle's co-rotational beam element against closed forms and invariants."""
import numpy as np
import pytest

from oracle import beam, actuation, solver
from workloads import robots_for_config


@pytest.fixture(scope="module")
def sec():
    return beam.section_stiffness(1.5e-3, 1.0e-3, 50e6, 0.45)


def test_section_closed_form(sec):
    EA, EI, GJ = sec
    A = np.pi * (1.5e-3**2 - 1.0e-3**2)
    I = np.pi / 4 * (1.5e-3**4 - 1.0e-3**4)
    assert A == pytest.approx(3.92699e-6, rel=1e-5)
    assert I == pytest.approx(3.19068e-12, rel=1e-5)
    assert EA == pytest.approx(196.35, rel=1e-5)
    assert EI == pytest.approx(1.59534e-4, rel=1e-5)
    assert GJ == pytest.approx(1.10023e-4, rel=1e-5)


def test_local_stiffness_textbook_entries(sec):
    EA, EI, GJ = sec
    l0 = 0.015
    K = beam.local_stiffness_12(l0, EA, EI, GJ)
    assert np.allclose(K, K.T, rtol=0, atol=0)
    assert K[0, 0] == EA / l0 and K[0, 6] == -EA / l0
    assert K[3, 3] == GJ / l0 and K[3, 9] == -GJ / l0
    assert K[1, 1] == pytest.approx(12 * EI / l0**3)
    assert K[5, 5] == pytest.approx(4 * EI / l0) and K[5, 11] == pytest.approx(2 * EI / l0)
    assert K[1, 5] == pytest.approx(6 * EI / l0**2) and K[2, 4] == pytest.approx(-6 * EI / l0**2)
    # null space = the six rigid-body modes of the straight element
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-9 * ev.max()) == 6
    rigid = np.zeros((12, 6))
    x = np.array([[0, 0, 0], [l0, 0, 0]])
    for n in range(2):
        rigid[6 * n:6 * n + 3, 0:3] = np.eye(3)
        rigid[6 * n:6 * n + 3, 3:6] = -beam.hat(x[n])
        rigid[6 * n + 3:6 * n + 6, 3:6] = np.eye(3)
    assert np.abs(K @ rigid).max() < 1e-9 * np.abs(K).max()


def _random_element(rng, l0, scale_p=1e-3, scale_r=0.3):
    P, R = beam.reference_state(1, l0, rng.normal(size=3) * 0.1, [0, 0, 1.0], [1.0, 0, 0])
    dX = np.zeros((2, 6))
    dX[:, 0:3] = rng.normal(size=(2, 3)) * scale_p
    dX[:, 3:6] = rng.normal(size=(2, 3)) * scale_r
    return beam.apply_increment(P, R, dX)


def test_inverse_left_jacobian(sec):
    rng = np.random.default_rng(3)
    for th_scale in (1e-4, 0.05, 0.8):
        th = rng.normal(size=3) * th_scale
        w = rng.normal(size=3) * 1e-7
        lhs = beam.logm_so3(beam.expm_so3(w) @ beam.expm_so3(th))
        assert np.allclose(lhs - th, beam.jl_inv(th) @ w, rtol=0, atol=1e-12)


def test_element_force_is_energy_gradient(sec):
    EA, EI, GJ = sec
    l0 = 0.015
    K7 = beam.local_stiffness_7(l0, EA, EI, GJ)
    rng = np.random.default_rng(0)
    for _ in range(5):
        P, R = _random_element(rng, l0)
        fe = beam.element_forces(P[0], R[0], P[1], R[1], l0, K7)
        h = 1e-6
        g = np.zeros(12)
        for k in range(12):
            d = np.zeros((2, 6))
            d[k // 6, k % 6] = h
            Pp, Rp = beam.apply_increment(P, R, d)
            Pm, Rm = beam.apply_increment(P, R, -d)
            g[k] = (beam.element_energy(Pp[0], Rp[0], Pp[1], Rp[1], l0, K7)
                    - beam.element_energy(Pm[0], Rm[0], Pm[1], Rm[1], l0, K7)) / (2 * h)
        assert np.abs(fe - g).max() <= 1e-7 * np.abs(fe).max()


def test_element_self_equilibrium_and_objectivity(sec):
    EA, EI, GJ = sec
    l0 = 0.015
    K7 = beam.local_stiffness_7(l0, EA, EI, GJ)
    rng = np.random.default_rng(1)
    P, R = _random_element(rng, l0)
    fe = beam.element_forces(P[0], R[0], P[1], R[1], l0, K7)
    assert np.abs(fe[0:3] + fe[6:9]).max() < 1e-14 * np.abs(fe).max()
    mom = np.cross(P[0], fe[0:3]) + np.cross(P[1], fe[6:9]) + fe[3:6] + fe[9:12]
    assert np.abs(mom).max() < 1e-13 * np.abs(fe).max()
    Q = beam.expm_so3(rng.normal(size=3))
    t = rng.normal(size=3)
    P2 = P @ Q.T + t
    R2 = Q[None] @ R
    fe2 = beam.element_forces(P2[0], R2[0], P2[1], R2[1], l0, K7)
    rot = np.concatenate([Q @ fe[0:3], Q @ fe[3:6], Q @ fe[6:9], Q @ fe[9:12]])
    assert np.abs(fe2 - rot).max() < 1e-12 * np.abs(fe).max()


def test_zero_force_at_reference_and_qp_tangent_equals_jacobian(sec):
    rb = robots_for_config(0)
    rob = solver.robots_from_batch(rb)[0]
    P, R = rob.reference()
    F = beam.internal_forces(P, R, rob.l0, rob.K7)
    # only the rounding of the node coordinates (ulp ~ 5e-17 m) times EA/l0 remains
    assert np.abs(F).max() <= 8 * (rob.EA[0] / rob.l0) * np.spacing(rob.length)
    resid = lambda P_, R_: beam.internal_forces(P_, R_, rob.l0, rob.K7)
    N = P.shape[0]
    J = beam.banded_to_dense(beam.fd_jacobian_banded(resid, P, R), 6 * N)
    K = beam.upper_banded_to_dense(beam.tangent_qp_upper_banded(P, R, rob.K12), 6 * N)
    assert np.allclose(K, K.T, rtol=0, atol=0)
    assert np.abs(J - K).max() <= 1e-7 * np.abs(K).max()
    # positive definite once the base node is fixed
    np.linalg.cholesky(K[6:, 6:])


def _tip_solve(rob, wrench, kind, n_steps=1, tol=1e-13):
    sched = lambda k: (0.0, np.asarray(wrench) * k / n_steps)
    P, R, traj = solver.solve_robot(rob, sched, n_steps, act_kind=kind, tol=tol, stag_tol=1e-9,
                                    max_iter=400, stop_on_failure=True)
    assert all(t["info"]["status"] == solver.OK for t in traj)
    return P, R


def test_pure_tip_moment_gives_discrete_circle():
    """Follower end moment M: every node lies on a circle with chord l0 and turn alpha = M l0 / EI."""
    rb = robots_for_config(0)
    rob = solver.robots_from_batch(rb)[0]
    EI = rob.EI[0]
    L = rob.length
    M = EI * (np.pi / 2) / L      # quarter circle
    P, R = _tip_solve(rob, [0, 0, 0, 0, 0, M], actuation.TIP_LOCAL, n_steps=4)
    alpha = M * rob.l0 / EI
    rho_h = rob.l0 / (2 * np.sin(alpha / 2))
    k = np.arange(P.shape[0])
    # base along +z, section z-axis = base_dir x base_up = +y: bending about +y turns +z toward -x? use geometry
    t = np.array([0, 0, 1.0]); u = np.array([1.0, 0, 0]); b = np.cross(t, u)
    n_dir = np.cross(b, t)    # direction the centreline turns toward for a moment about +b
    exp = (rho_h * np.sin(k * alpha))[:, None] * t + (rho_h * (1 - np.cos(k * alpha)))[:, None] * n_dir
    err = np.abs(P - exp).max()
    assert err <= 1e-11, err
    # against the continuum arc rho = EI/M the discrete model differs by ~alpha^2/24
    rho = EI / M
    tip_c = rho * np.sin(L / rho) * t + rho * (1 - np.cos(L / rho)) * n_dir
    rel = np.linalg.norm(P[-1] - tip_c) / np.linalg.norm(tip_c)
    assert rel <= 2 * alpha**2 / 24 + 1e-12


def test_small_deflection_cantilever():
    """Dead transverse tip load P: delta = P L^3 / 3EI, tip rotation P L^2 / 2EI."""
    rb = robots_for_config(0)
    rob = solver.robots_from_batch(rb)[0]
    EI = rob.EI[0]
    L = rob.length
    Pld = 1e-4 * 3 * EI / L**2        # delta / L = 1e-4
    P, R = _tip_solve(rob, [Pld, 0, 0, 0, 0, 0], actuation.TIP_GLOBAL)
    delta = Pld * L**3 / (3 * EI)
    assert P[-1, 0] == pytest.approx(delta, rel=1e-6)
    assert abs(P[-1, 1]) < 1e-15
    rot = beam.logm_so3(R[-1] @ R[0].T)
    assert np.linalg.norm(rot) == pytest.approx(Pld * L**2 / (2 * EI), rel=1e-6)


def test_axial_follower_force_uniform_shortening():
    """Axial tip force F along the tip tangent: straight, every element shortened by F l0 / EA."""
    rb = robots_for_config(0)
    rob = solver.robots_from_batch(rb)[0]
    F = -0.9
    P, R = _tip_solve(rob, [F, 0, 0, 0, 0, 0], actuation.TIP_LOCAL)
    assert np.abs(P[:, 0:2]).max() < 1e-15
    assert P[-1, 2] == pytest.approx(rob.length * (1 + F / rob.EA[0]), rel=1e-14)


def test_cable_moments_of_equal_tensions_cancel():
    """Eq. 16 with three cables at 120 degrees: equal tensions give no moment, a single
    cable's moment is T r about the section axis normal to its attachment direction."""
    rb = robots_for_config(0)
    rob = solver.robots_from_batch(rb)[0]
    r = rob.cable_radius
    F, M = actuation.cable_wrench_local([0.7, 0.7, 0.7], r, rob.cable_angle)
    assert np.abs(M).max() <= 1e-16 and F == pytest.approx([-2.1, 0, 0], abs=1e-15)
    for j, phi in enumerate(rob.cable_angle):
        T = np.zeros(3)
        T[j] = 1.3
        _, M = actuation.cable_wrench_local(T, r, rob.cable_angle)
        d = r * np.array([0.0, np.cos(phi), np.sin(phi)])       # attachment point
        assert np.linalg.norm(M) == pytest.approx(1.3 * r, rel=1e-15)
        assert abs(M @ d) <= 1e-18 and M[0] == 0.0             # normal to d and the axis
        # pulling toward the base at d turns the section toward d: M = d x (-T e_x)
        assert np.allclose(M, np.cross(d, [-1.3, 0, 0]), rtol=0, atol=1e-18)


@pytest.mark.parametrize("phi,tol", [(0.0, 1e-11), (np.pi / 2, 1e-11), (2 * np.pi / 3, 1e-7)])
def test_single_cable_bends_toward_it_on_a_circle(phi, tol):
    """One tensioned cable at angle phi (the moment-only CABLES kind): a follower end moment
    T r, so the nodes lie on the discrete circle of turn alpha = T r l0 / EI, curving toward
    the side of the section the cable is attached to (Sec. II-E, Fig. 1c).  Exact in the
    planes of the section axes; in an oblique plane the element frame (built from the
    nodes' section y-axes) couples bending and torsion at second order, which leaves a
    relative twist of ~2e-8 per element here, hence the looser bound there."""
    rb = robots_for_config(0)
    rob = solver.robots_from_batch(rb)[0]
    rob.cable_angle = np.array([phi, phi + 2 * np.pi / 3, phi + 4 * np.pi / 3])
    EI, L, r = rob.EI[0], rob.length, rob.cable_radius
    Tn = EI * (np.pi / 2) / (L * r)        # a quarter circle
    P, R = _tip_solve(rob, [Tn, 0.0, 0.0], actuation.CABLES, n_steps=4)
    alpha = Tn * r * rob.l0 / EI
    rho_h = rob.l0 / (2 * np.sin(alpha / 2))
    k = np.arange(P.shape[0])
    t = np.asarray(rob.base_dir, float)
    u = np.asarray(rob.base_up, float)
    b = np.cross(t, u)
    side = np.cos(phi) * u + np.sin(phi) * b        # the cable's side of the section
    exp = (np.asarray(rob.base_pos, float) + (rho_h * np.sin(k * alpha))[:, None] * t
           + (rho_h * (1 - np.cos(k * alpha)))[:, None] * side)
    assert np.abs(P - exp).max() <= tol * L


def test_cable_wrench_equal_tensions_shorten_the_straight_robot():
    """Eq. 17 as printed (CABLE_WRENCH): equal tensions give no moment and the summed cable
    force compresses the robot along its axis, so it stays straight and every element
    shortens by sum(T) l0 / EA (exact for the l - l0 strain measure)."""
    rb = robots_for_config(0)
    rob = solver.robots_from_batch(rb)[0]
    T = np.full(3, 0.3)
    P, R = _tip_solve(rob, T, actuation.CABLE_WRENCH)
    # the cable moments cancel to rounding (~1e-19 N m), which the axial follower
    # compression (about 200 Euler loads) amplifies into ~1e-13 m of lateral offset
    assert np.abs(P[:, 0:2] - np.asarray(rob.base_pos)[0:2]).max() <= 1e-12
    dz = np.diff(P[:, 2])
    assert np.allclose(dz, rob.l0 * (1 - T.sum() / rob.EA[0]), rtol=1e-14, atol=0)
    # the moment-only kind leaves the robot untouched
    P2, _ = _tip_solve(rob, T, actuation.CABLES)
    assert np.abs(P2 - rob.reference()[0]).max() <= 1e-15


def test_cable_wrench_single_cable_load_reaches_the_base():
    """Eq. 17 with one cable: at equilibrium (no wall) the clamp carries the cable's pull,
    i.e. the internal force at the base node is -sum_j F_j turned by the tip triad, T e1_tip,
    and the robot bends toward the cable."""
    rb = robots_for_config(0)
    rob = solver.robots_from_batch(rb)[0]
    T = np.array([4e-3, 0.0, 0.0])          # about one Euler load pi^2 EI / 4 L^2
    P, R = _tip_solve(rob, T, actuation.CABLE_WRENCH, n_steps=4)
    fint = beam.internal_forces(P, R, rob.l0, rob.K7)
    assert np.allclose(fint[0, 0:3], T.sum() * R[-1][:, 0], rtol=0, atol=1e-12)
    side = np.asarray(rob.base_up, float)    # cable 0 at angle 0: the section y-axis
    assert (P[-1] - P[0]) @ side > 0.0
