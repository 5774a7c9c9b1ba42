"""Pins of contact along an element (Sec. II-C, eq. 3-7 at 0 < xi < l0) in the oracle:
segment closest points against brute force, the knife-edge detection, static equivalence of
the distributed contact force, the propped cantilever against beam theory, and the adjoint
with an element contact against central differences of complete re-solves."""
import numpy as np
import pytest

from oracle import actuation, adjoint, collision, solver
from tests.element_fixtures import cantilever_influence, knife_edge_case


def test_segment_closest_points_match_brute_force():
    """Random segment pairs: the returned pair attains a distance no larger than any sampled
    pair and within the sampling resolution of the sampled minimum."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        p1, p2, q1, q2 = rng.normal(size=(4, 3))
        if rng.uniform() < 0.3:                        # nearly crossing or nearly parallel
            q1 = p1 + 0.3 * (p2 - p1) + 1e-3 * rng.normal(size=3)
            q2 = q1 + (p2 - p1) * rng.choice([1.0, -0.5]) + rng.normal(size=3) * rng.choice([1e-3, 1.0])
        s, u, dist, sin2 = collision.segment_closest(p1, p2, q1, q2)
        assert 0.0 <= s <= 1.0 and 0.0 <= u <= 1.0
        assert dist == pytest.approx(np.linalg.norm(p1 + s * (p2 - p1) - q1 - u * (q2 - q1)), abs=1e-12)
        g = np.linspace(0.0, 1.0, 401)
        P = p1[None, :] + g[:, None] * (p2 - p1)[None, :]
        Q = q1[None, :] + g[:, None] * (q2 - q1)[None, :]
        D = np.linalg.norm(P[:, None, :] - Q[None, :, :], axis=2)
        res = (np.linalg.norm(p2 - p1) + np.linalg.norm(q2 - q1)) / 400
        assert dist <= D.min() + 1e-12
        assert dist >= D.min() - res
        d1, d2 = p2 - p1, q2 - q1
        assert sin2 == pytest.approx(1.0 - (d1 @ d2) ** 2 / ((d1 @ d1) * (d2 @ d2)), abs=1e-12)


def test_knife_edge_is_an_element_contact():
    """The chord of element 7 touches the ridge at s = 0.3 with gap 0, normal -x; no node
    of the robot is within the band of the wall, so node contacts alone see nothing."""
    rb, V, T, a = knife_edge_case()
    rob = solver.robots_from_batch(rb, collision.Mesh(V, T))[0]
    P, R = rob.reference()
    assert collision.active(collision.detect(P, rob.mesh, rob.r_c, rob.delta)) == []
    for cull in (True, False):
        c = collision.detect_elements(P, rob.mesh, rob.r_c, rob.delta, cull=cull)
        assert len(c) == 1 and c[0]["node"] == 7 and c[0]["kind"] == collision.ELEMENT
        assert c[0]["s"] == pytest.approx(0.3, abs=1e-12)
        assert c[0]["gap"] == pytest.approx(0.0, abs=1e-15)
        assert np.allclose(c[0]["n"], [-1.0, 0.0, 0.0], atol=1e-12)
        assert not c[0]["ambiguous"]


def test_element_contact_force_is_statically_equivalent():
    """The row's nodal forces sum to y n and have no moment about the contact point: the
    weights (1 - s, s) are the ones that interpolate p(s) from the nodes."""
    rng = np.random.default_rng(3)
    P = np.cumsum(rng.normal(size=(6, 3)) * 0.01, axis=0)
    for s in (0.1, 0.5, 0.83):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        ct = dict(node=2, tri=0, kind=collision.ELEMENT, s=s, n=n, gap=0.0)
        F = np.zeros((6, 6))
        r = solver.contact_residual(F, [ct], np.array([0.7]))
        f = -r[:, 0:3]                               # contact forces on the free nodes 1..5
        p = (1 - s) * P[2] + s * P[3]
        assert np.allclose(f.sum(axis=0), 0.7 * n, atol=1e-15)
        mom = sum(np.cross(P[i + 1] - p, f[i]) for i in range(5))
        assert np.abs(mom).max() <= 1e-16


def _propped(P_tip, elements=True, n_steps=1):
    rb, V, T, a = knife_edge_case()
    rob = solver.robots_from_batch(rb, collision.Mesh(V, T))[0]
    rob.elements = elements
    sched = lambda k: (0.0, np.array(P_tip, float) * k / n_steps)
    P, R, traj = solver.solve_robot(rob, sched, n_steps, act_kind=actuation.TIP_GLOBAL, tol=1e-13,
                                    stag_tol=1e-9, max_iter=200)
    return rob, P, R, traj


def test_propped_cantilever_matches_beam_theory():
    """Tip force P towards the ridge: the element contact props the cantilever at z = a.  With
    the reaction y split as (1 - s) y, s y on nodes 7 and 8 (Euler-Bernoulli elements are
    exact at the nodes for nodal loads), the chord point does not move: (1 - s) w_7 + s w_8 = 0
    gives y in closed form.  Without element contacts the chord passes through the ridge."""
    rb, V, T, a = knife_edge_case()
    rob0 = solver.robots_from_batch(rb)[0]
    EI, L, l0, s = rob0.EI[0], rob0.length, rob0.l0, 0.3
    Pld = 1e-4 * 3 * EI / L ** 2
    rob, P, R, traj = _propped([Pld, 0, 0, 0, 0, 0])
    last = traj[-1]
    assert last["info"]["status"] == solver.OK
    act = [(c, y) for c, y in zip(last["contacts"], last["y"]) if y > 0]
    assert len(act) == 1 and act[0][0]["kind"] == collision.ELEMENT and act[0][0]["node"] == 7
    z7, z8 = 7 * l0, 8 * l0
    G = lambda x, c: cantilever_influence(x, c, EI)
    y_cf = Pld * ((1 - s) * G(z7, L) + s * G(z8, L)) / (
        (1 - s) ** 2 * G(z7, z7) + 2 * s * (1 - s) * G(z7, z8) + s ** 2 * G(z8, z8))
    assert act[0][1] == pytest.approx(y_cf, rel=1e-6)
    # the chord tilts by ~1e-4 rad, which moves its nearest point to the ridge by ~r_c 1e-4
    assert act[0][0]["s"] == pytest.approx(s, abs=1e-5)
    tip_cf = Pld * G(L, L) - y_cf * ((1 - s) * G(L, z7) + s * G(L, z8))
    assert P[-1, 0] == pytest.approx(tip_cf, rel=1e-6)
    chord_x = (1 - s) * P[7, 0] + s * P[8, 0]
    assert abs(chord_x) <= 1e-12
    _, Pn, _, trn = _propped([Pld, 0, 0, 0, 0, 0], elements=False)
    assert trn[-1]["info"]["status"] == solver.OK and trn[-1]["contacts"] == []
    assert (1 - s) * Pn[7, 0] + s * Pn[8, 0] > 1e-6       # through the ridge by micrometres


def test_element_contact_adjoint_matches_central_differences():
    """dL/du of a tip loss for the tip wrench u, with the element contact active, against
    central differences of complete re-solves (the row (1 - s) n, s n and the curvature of
    the distance to the ridge line both enter)."""
    rb, V, T, a = knife_edge_case()
    rob0 = solver.robots_from_batch(rb)[0]
    EI, L = rob0.EI[0], rob0.length
    Pld = 3e-3 * 3 * EI / L ** 2
    u0 = np.array([Pld, 0.4 * Pld, 0.0, 0.0, 0.0, 0.2 * Pld * L])
    target = np.array([5e-3, 4e-3, 0.31])

    def solve(u):
        rob, P, R, traj = _propped(u, n_steps=2)
        assert traj[-1]["info"]["status"] == solver.OK
        return rob, P, R, traj[-1]

    rob, P, R, last = solve(u0)
    assert any(c["kind"] == collision.ELEMENT and y > 0 for c, y in zip(last["contacts"], last["y"]))
    sens = [P.shape[0] - 1]
    L0, dLdp = adjoint.sensor_loss(P, sens, target[None, :])
    g = adjoint.tension_gradient(rob, P, R, last["contacts"], last["y"], u0, sens, dLdp,
                                 act_kind=actuation.TIP_GLOBAL)
    for j, h in ((0, 1e-3 * Pld), (1, 1e-3 * Pld), (5, 1e-3 * Pld * L)):
        du = np.zeros(6)
        du[j] = h
        Lp = adjoint.sensor_loss(solve(u0 + du)[1], sens, target[None, :])[0]
        Lm = adjoint.sensor_loss(solve(u0 - du)[1], sens, target[None, :])[0]
        fd = (Lp - Lm) / (2 * h)
        # dropping the curvature term changes these gradients by 6e-6, 3e-7 and 1e-5 relative;
        # the differences agree with the adjoint to 2e-11, 8e-11 and 3e-7
        assert g[j] == pytest.approx(fd, rel=1e-6), (j, g[j], fd)


def test_element_gap_gradient_matches_differences():
    """(1 - s) n, s n is the gradient of the chord's distance to a line or a point."""
    rng = np.random.default_rng(5)
    for feat in ("line", "point"):
        xa = np.array([0.0, 0.0, 0.0]) + 1e-3 * rng.normal(size=3)
        xb = np.array([0.0, 0.0, 0.01]) + 1e-3 * rng.normal(size=3)
        q1 = np.array([2e-3, -4e-3, 0.004])
        q2 = np.array([2.5e-3, 4e-3, 0.006]) if feat == "line" else None

        def dist(x):
            a, b = x[0:3], x[3:6]
            if q2 is None:
                return collision.segment_closest(a, b, q1, q1 + 1e-12)[2]
            d2 = q2 - q1
            # distance from the chord to the infinite line: closest pair with u unclamped
            d1 = b - a
            r = a - q1
            A = np.array([[d1 @ d1, -d1 @ d2], [-d1 @ d2, d2 @ d2]])
            st = np.linalg.solve(A, np.array([-(d1 @ r), d2 @ r]))
            return np.linalg.norm(a + st[0] * d1 - q1 - st[1] * d2)

        x = np.concatenate([xa, xb])
        gr = adjoint.element_gap_gradient(xa, xb, q1, q2)
        h = 1e-8
        fd = np.array([(dist(x + h * e) - dist(x - h * e)) / (2 * h) for e in np.eye(6)])
        assert np.allclose(gr, fd, rtol=0, atol=1e-6), (feat, gr, fd)


def test_element_detection_cull_keeps_every_contact():
    """Chords scattered near the wall of a patch of the branching lumen: the k-d-tree superset
    of triangles gives exactly the contacts of the loop over every triangle."""
    from workloads import make_config
    rb, V, T = make_config(1)
    full = collision.Mesh(V, T)
    rng = np.random.default_rng(9)
    centre = full.centroid[rng.integers(len(T))]
    keep = np.nonzero(np.linalg.norm(full.centroid - centre, axis=1) < 0.02)[0]
    mesh = collision.Mesh(V, T[keep])
    n = 40
    vid = rng.choice(np.unique(T[keep]), size=n)
    nrm = mesh.n[rng.integers(len(keep), size=n)]
    P = V[vid] + nrm * rng.uniform(1e-3, 3e-3, size=(n, 1)) + rng.normal(size=(n, 3)) * 2e-3
    a = collision.detect_elements(P, mesh, 1.5e-3, 1e-3, cull=True)
    b = collision.detect_elements(P, mesh, 1.5e-3, 1e-3, cull=False)
    key = lambda c: (c["node"], c["tri"], c["kind"], c["ambiguous"])
    assert [key(c) for c in a] == [key(c) for c in b]
    assert sum(1 for c in b if c["tri"] >= 0) >= 3


def test_sharp_features_of_folds():
    """Two triangles folded about their common edge: a convex fold of 30 degrees is a sharp
    feature (its edge and both end vertices), 5 degrees or a flat pair or a concave fold of 30
    degrees is not; the other edges (rims) are."""
    def fold(deg):
        a = np.radians(deg)
        # common edge along y; one face in the plane z = 0 (x < 0), the other turned by a about y
        V = np.array([[0, -1, 0], [0, 1, 0], [-1, 0, 0], [np.cos(a), 0, -np.sin(a)]], float)
        T = np.array([[0, 1, 2], [1, 0, 3]])
        return collision.Mesh(V, T)
    for deg, sharp in ((30.0, True), (5.0, False), (0.0, False), (-30.0, False)):
        m = fold(deg)
        assert m.n[0][2] > 0 and m.n[1][2] > 0             # both face the lumen (+z)
        assert bool(m.sharp[0, 0]) == sharp and bool(m.sharp[1, 0]) == sharp, deg
        assert bool(m.sharp[0, 3]) and bool(m.sharp[0, 4])   # the vertices also lie on rims
        assert m.sharp[0, 1] and m.sharp[0, 2] and m.sharp[1, 1] and m.sharp[1, 2]
    # the knife-edge ridge of the propped cantilever is sharp
    rb, V, T, a = knife_edge_case()
    assert collision.Mesh(V, T).sharp[0, 0]
