"""Pins of the oracle's contact detection: hand-computed triangles, a faceted tube,
brute force against a dense-sampling closest point, and culled against unculled."""
import numpy as np
import pytest

from oracle import collision
from workloads import straight_cylinder_mesh, make_config


def one_triangle():
    V = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0]], float)
    T = np.array([[0, 1, 2]])
    return collision.Mesh(V, T)          # normal +z


def test_single_triangle_face_contact_by_hand():
    m = one_triangle()
    assert np.allclose(m.n[0], [0, 0, 1])
    P = np.array([[0, 0, -1.0], [0.002, 0.003, 0.0021]])
    c = collision.detect(P, m, r_c=1.5e-3, delta=1e-3)
    assert len(c) == 1 and c[0]["node"] == 1 and c[0]["tri"] == 0 and c[0]["kind"] == 0
    assert c[0]["gap"] == pytest.approx(0.0021 - 1.5e-3, abs=1e-18)
    assert np.allclose(c[0]["n"], [0, 0, 1])
    # outside the band (s > r_c + delta) and behind it (s < -r_c): nothing
    for z in (2.6e-3, -1.6e-3):
        assert collision.detect(np.array([[0, 0, -1.0], [0.002, 0.003, z]]), m, 1.5e-3, 1e-3) == []


def test_single_triangle_edge_and_vertex_fallback_by_hand():
    m = one_triangle()
    # beyond edge AB (y < 0), in front of the plane: closest point on the edge
    p = np.array([0.004, -0.001, 0.0015])
    c = collision.detect(np.array([[0, 0, -1.0], p]), m, 1.5e-3, 1e-3)
    assert len(c) == 1 and c[0]["kind"] == 1
    d = np.hypot(0.001, 0.0015)
    assert c[0]["gap"] == pytest.approx(d - 1.5e-3, abs=1e-18)
    assert np.allclose(c[0]["n"], np.array([0, -0.001, 0.0015]) / d)
    # beyond vertex A: closest point is the vertex
    p = np.array([-0.001, -0.001, 0.001])
    c = collision.detect(np.array([[0, 0, -1.0], p]), m, 1.5e-3, 1e-3)
    assert len(c) == 1 and c[0]["kind"] == 1
    assert c[0]["gap"] == pytest.approx(np.linalg.norm(p) - 1.5e-3, abs=1e-18)


def test_closest_point_regions_against_dense_sampling():
    rng = np.random.default_rng(5)
    for _ in range(200):
        V = rng.normal(size=(3, 3)) * 0.01
        m = collision.Mesh(V, np.array([[0, 1, 2]]))
        p = rng.normal(size=3) * 0.01
        cpt, region, _ = collision.closest_points(p, m, np.array([0]))
        u, v = np.meshgrid(np.linspace(0, 1, 401), np.linspace(0, 1, 401))
        ok = u + v <= 1
        S = V[0] + u[ok, None] * (V[1] - V[0]) + v[ok, None] * (V[2] - V[0])
        dmin = np.min(np.linalg.norm(S - p, axis=1))
        d = np.linalg.norm(cpt[0] - p)
        assert d <= dmin + 1e-12
        assert d >= dmin - 3e-4 * np.max(np.linalg.norm(V - V.mean(0), axis=1))


def test_sixteen_gon_tube_facet_distance():
    """Straight 16-gon tube of vertex radius 4 mm: facet planes at 4 cos(pi/16) = 3.9231 mm."""
    V, T = straight_cylinder_mesh(radius=4e-3, axis_xy=(0.0, 0.0))
    m = collision.Mesh(V, T)
    ang = np.pi / 16        # mid-facet direction of facet 0
    for off in (1.5e-3, 2.0e-3, 2.4e-3):
        p = np.array([off * np.cos(ang), off * np.sin(ang), 0.1])
        c = collision.detect(np.array([[0, 0, 0], p]), m, 1.5e-3, 1e-3)
        gaps = sorted(ct["gap"] for ct in c)
        assert len(c) >= 1
        assert gaps[0] == pytest.approx(4e-3 * np.cos(np.pi / 16) - off - 1.5e-3, abs=1e-15)


def test_culled_equals_brute_force_on_branching_mesh():
    rb, V, T = make_config(1)
    m = collision.Mesh(V, T)
    rng = np.random.default_rng(11)
    # points near the wall: mesh vertices pushed inward along random directions
    vid = rng.choice(len(V), size=60, replace=False)
    cen = m.centroid[rng.choice(len(T), size=60, replace=False)]
    P = np.concatenate([[[0, 0, -1.0]], V[vid] * 0.9 + 0.1 * cen], axis=0)
    a = collision.detect(P, m, 1.5e-3, 1e-3, cull=True)
    b = collision.detect(P, m, 1.5e-3, 1e-3, cull=False)
    assert collision.contact_set(a) == collision.contact_set(b)
    assert len(collision.contact_set(a)) > 10


def _persist_robot(mesh):
    from oracle import solver
    return solver.Robot(2, 0.02, np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 1.0, 0]),
                        1.0, 1e-3, 1e-3, 1e-3, np.zeros(1), 1.5e-3, 1e-3, 1e-3, mesh=mesh)


def test_persisting_face_contact_rules_by_hand():
    """A convex ridge along x = 0: face 0 (z = 0 for x <= 0) and face 1 tilted down for
    x >= 0; inward normals point to +z.  A node that was pressed on face 0 and is now past
    the ridge (in the edge region, no face contact) keeps face 0's plane while it is within
    the band of that triangle; not once it is farther, nor if the previous force was zero."""
    from oracle import solver
    s = np.sin(np.radians(20.0)); c = np.cos(np.radians(20.0))
    V = np.array([[-0.01, -0.01, 0.0], [0.0, -0.01, 0.0], [0.0, 0.01, 0.0], [-0.01, 0.01, 0.0],
                  [0.01 * c, -0.01, -0.01 * s], [0.01 * c, 0.01, -0.01 * s]])
    T = np.array([[0, 1, 2], [0, 2, 3], [1, 4, 5], [1, 5, 2]])
    mesh = collision.Mesh(V, T)
    rob = _persist_robot(mesh)
    r_c, band = rob.r_c, rob.r_c + rob.delta
    prev = [dict(node=1, tri=0, kind=0, n=mesh.n[0].copy(), gap=0.0)]
    # node just past the ridge, 1.6 mm above the ridge line: fallback edge contact only
    P = np.array([[-0.015, 0.0, 0.01], [0.0005, -0.002, 0.0016], [0.015, 0.0, 0.01]])
    det = solver.detect(rob, P)
    assert [(c["node"], c["kind"]) for c in det] == [(1, 1)]
    got = solver.detect(rob, P, prev=(prev, np.array([0.3])))
    assert [(c["node"], c["tri"], c["kind"]) for c in got] == [(1, 0, 0), (1, det[0]["tri"], 1)]
    assert got[0]["gap"] == pytest.approx(0.0016 - r_c, abs=1e-15)
    # no force in the previous iterate: nothing persists
    assert collision.contact_set(solver.detect(rob, P, prev=(prev, np.array([0.0])))) == \
        collision.contact_set(det)
    # farther than the band from triangle 0: nothing persists
    P2 = P.copy()
    P2[1] = [band + 0.0005, -0.002, 0.0016]
    assert collision.contact_set(solver.detect(rob, P2, prev=(prev, np.array([0.3])))) == \
        collision.contact_set(solver.detect(rob, P2))


def test_persisting_face_skips_coplanar_duplicate():
    """Triangles 0 and 1 are coplanar halves of one quad: a node that moved from the face
    region of 0 into that of 1 gets face 1 detected, and face 0 (same plane) does not persist."""
    from oracle import solver
    V = np.array([[-0.01, -0.01, 0.0], [0.01, -0.01, 0.0], [0.01, 0.01, 0.0], [-0.01, 0.01, 0.0]])
    T = np.array([[0, 1, 2], [0, 2, 3]])
    mesh = collision.Mesh(V, T)
    rob = _persist_robot(mesh)
    P = np.array([[-0.015, 0.0, 0.01], [-0.004, 0.006, 0.0012], [0.015, 0.0, 0.01]])
    det = solver.detect(rob, P)
    assert [(c["node"], c["tri"], c["kind"]) for c in det] == [(1, 1, 0)]
    prev = [dict(node=1, tri=0, kind=0, n=mesh.n[0].copy(), gap=0.0)]
    assert collision.contact_set(solver.detect(rob, P, prev=(prev, np.array([0.2])))) == \
        collision.contact_set(det)


def test_persisting_edge_contact_rules_by_hand():
    """The same convex ridge along x = 0 (shared by triangles 0 and 3).  A node that was pressed
    on the ridge through an edge contact of triangle 3 and is now back over face 0 (face 0
    detected, so no fallback) keeps that contact as the direction from the ridge:
    n = (p - q) / |p - q| with q the foot of p on the ridge line, gap |p - q| - r_c.  The same
    contact taken on triangle 0, whose nearest point is now the foot on face 0, lies on face
    0's plane and is dropped; below the plane of triangle 3 it is not kept."""
    from oracle import solver
    s = np.sin(np.radians(20.0)); c = np.cos(np.radians(20.0))
    V = np.array([[-0.01, -0.01, 0.0], [0.0, -0.01, 0.0], [0.0, 0.01, 0.0], [-0.01, 0.01, 0.0],
                  [0.01 * c, -0.01, -0.01 * s], [0.01 * c, 0.01, -0.01 * s]])
    T = np.array([[0, 1, 2], [0, 2, 3], [1, 4, 5], [1, 5, 2]])
    mesh = collision.Mesh(V, T)
    rob = _persist_robot(mesh)
    r_c = rob.r_c
    P = np.array([[-0.015, 0.0, 0.01], [-0.0005, -0.002, 0.0016], [0.015, 0.0, 0.01]])
    det = solver.detect(rob, P)
    assert [(c_["node"], c_["tri"], c_["kind"]) for c_ in det] == [(1, 0, 0)]
    prev = [dict(node=1, tri=3, kind=1, n=np.array([0.0, 0.0, 1.0]), gap=0.0)]
    got = solver.detect(rob, P, prev=(prev, np.array([0.4])))
    assert [(c_["node"], c_["tri"], c_["kind"]) for c_ in got] == [(1, 0, 0), (1, 3, 1)]
    q = np.array([0.0, -0.002, 0.0])
    dq = P[1] - q
    assert np.allclose(got[1]["n"], dq / np.linalg.norm(dq), rtol=0, atol=1e-14)
    assert got[1]["gap"] == pytest.approx(np.linalg.norm(dq) - r_c, abs=1e-15)
    # the same contact on triangle 0: its nearest point is the foot on face 0 -> same plane
    prev0 = [dict(node=1, tri=0, kind=1, n=np.array([0.0, 0.0, 1.0]), gap=0.0)]
    assert collision.contact_set(solver.detect(rob, P, prev=(prev0, np.array([0.4])))) == \
        collision.contact_set(det)
    # within the band of triangle 3 but below its plane: not kept
    P3 = P.copy()
    P3[1] = [-0.002, -0.002, 0.0006]
    assert mesh.n[3][2] > 0 and float(mesh.n[3] @ (P3[1] - V[1])) < 0
    assert np.linalg.norm(P3[1] - np.array([0.0, -0.002, 0.0])) <= r_c + rob.delta
    assert collision.contact_set(solver.detect(rob, P3, prev=(prev, np.array([0.4])))) == \
        collision.contact_set(solver.detect(rob, P3))


def test_ambiguity_flag_marks_decisions_within_1e9_of_a_threshold():
    """Nodes whose detection decisions lie within AMBIG_TOL (1e-9 m) of a threshold are
    flagged - the parity tests exclude exactly those from the exact set comparison - and
    clear decisions are not."""
    m = one_triangle()
    rc, dl = 1.5e-3, 1e-3
    band = rc + dl
    base = np.array([0, 0, -1.0])

    def det(p):
        return collision.detect(np.array([base, p]), m, rc, dl)

    # clear face contact, well inside the face region and the band
    c = det(np.array([0.002, 0.003, band - 1e-6]))
    assert len(c) == 1 and c[0]["kind"] == 0 and not c[0]["ambiguous"]
    # just inside the band edge: a contact, flagged
    c = det(np.array([0.002, 0.003, band - 4e-10]))
    assert len(c) == 1 and c[0]["kind"] == 0 and c[0]["ambiguous"]
    # just outside the band edge: no contact, but a flagged placeholder (tri = -1)
    c = det(np.array([0.002, 0.003, band + 4e-10]))
    assert len(c) == 1 and c[0]["tri"] == -1 and c[0]["ambiguous"]
    assert collision.active(c) == [] and collision.contact_set(c) == ()
    # just behind the plane's lower threshold s = -r_c
    c = det(np.array([0.002, 0.003, -rc + 4e-10]))
    assert len(c) == 1 and c[0]["ambiguous"]
    # projection 4e-10 m inside edge AB (y = 0): face-region decision is near its boundary
    c = det(np.array([0.004, 4e-10, 2e-3]))
    assert len(c) == 1 and c[0]["kind"] == 0 and c[0]["ambiguous"]
    # and 1e-6 m inside: clear
    c = det(np.array([0.004, 1e-6, 2e-3]))
    assert len(c) == 1 and not c[0]["ambiguous"]


def test_ambiguity_flag_on_edge_fallback_ties():
    """Two triangles whose nearest edge points are equally far from the node (within
    1e-9 m) but distinct: the fallback's choice between them is flagged."""
    # two coplanar triangles (normal +z) with parallel edges at x = -a and x = +a
    a = 2e-3
    V = np.array([[-a, -0.01, 0], [-0.012, 0.0, 0], [-a, 0.01, 0],
                  [a, -0.01, 0], [a, 0.01, 0], [0.012, 0.0, 0]], float)
    T = np.array([[0, 2, 1], [3, 5, 4]])
    m = collision.Mesh(V, T)
    assert m.n[0][2] > 0 and m.n[1][2] > 0
    rc, dl = 1.5e-3, 1e-3
    z = 1.2e-3                     # distance to both edges sqrt(a^2 + z^2) = 2.33 mm < band
    c = collision.detect(np.array([[0, 0, -1.0], [0.0, 0.0, z]]), m, rc, dl)
    assert len(c) == 1 and c[0]["kind"] == 1 and c[0]["tri"] == 0 and c[0]["ambiguous"]
    c = collision.detect(np.array([[0, 0, -1.0], [1e-6, 0.0, z]]), m, rc, dl)
    assert len(c) == 1 and c[0]["kind"] == 1 and c[0]["tri"] == 1 and not c[0]["ambiguous"]
