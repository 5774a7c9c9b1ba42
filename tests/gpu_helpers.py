"""Shared drivers for the GPU parity tests: run the HIP library and the oracle on the
same seeded inputs and compare what the method fixes uniquely."""
import numpy as np

from oracle import solver, collision, beam, actuation
from workloads import make_config, load_schedule


def gpu_context(rb, V=None, T=None, **kw):
    from paper_2503_06922_amd import fem
    ctx = fem.Context(fem.params_from_batch(rb, **kw))
    if V is None:
        ctx.fem_set_lumen(np.zeros((0, 3)), np.zeros((0, 3), np.int32))
    else:
        ctx.fem_set_lumen(V, T)
    return ctx


def robot_slices(rb):
    off = rb.node_offset
    return [slice(int(off[b]), int(off[b + 1])) for b in range(rb.n_robots)]


def oracle_robots(rb, V=None, T=None):
    mesh = None if V is None or len(T) == 0 else collision.Mesh(V, T)
    return solver.robots_from_batch(rb, mesh), mesh


def displacement_error(P_gpu, P_orc, P_ref):
    """max_i |p_gpu - p_orc| / max_i |p_orc - p_ref|."""
    scale = np.max(np.linalg.norm(P_orc - P_ref, axis=1))
    return np.max(np.linalg.norm(P_gpu - P_orc, axis=1)) / max(scale, 1e-300)


def node_forces(contacts, n_nodes, ykey="force"):
    """Per-node contact force vectors sum_c y_c n_c (unique even when y is not); a contact
    along an element gives (1 - s) y n and s y n to its two nodes."""
    f = np.zeros((n_nodes, 3))
    for c in contacts:
        for i, w in collision.row_entries(c):
            f[i] += w * c[ykey] * np.asarray(c["n"])
    return f


_EDGE_VERTS = {collision.EDGE_AB: (0, 1), collision.EDGE_AC: (0, 2), collision.EDGE_BC: (1, 2)}
_VERT = {collision.VERT_A: 0, collision.VERT_B: 1, collision.VERT_C: 2}


def feature_key(c, P, mesh):
    """The mesh feature a contact constrains against: ("F", triangle) for a face contact; for an
    edge/vertex contact the edge (its two vertex indices) or the vertex that holds the node's
    nearest point on the contact's triangle.  Two triangles that share that edge or vertex give
    the same constraint (same nearest point, normal and gap), so the key is the feature, not the
    triangle whose index won the tie."""
    if c["kind"] == 0:
        return (c["node"], "F", c["tri"])
    tv = mesh.T[c["tri"]]
    if c["kind"] == collision.ELEMENT:
        # the feature that holds the nearest point of the chord point on the triangle
        reg = collision.element_contact_geometry(np.asarray(P[c["node"]], float),
                                                 np.asarray(P[c["node"] + 1], float), mesh, c["tri"])[4]
        if reg in _EDGE_VERTS:
            a, b = _EDGE_VERTS[reg]
            return (c["node"], "SE", int(min(tv[a], tv[b])), int(max(tv[a], tv[b])))
        if reg in _VERT:
            return (c["node"], "SV", int(tv[_VERT[reg]]))
        return (c["node"], "Sf", c["tri"])
    _, reg, _ = collision.closest_points(np.asarray(P[c["node"]], float), mesh, np.array([c["tri"]]))
    reg = int(reg[0])
    if reg in _EDGE_VERTS:
        a, b = _EDGE_VERTS[reg]
        return (c["node"], "E", int(min(tv[a], tv[b])), int(max(tv[a], tv[b])))
    if reg in _VERT:
        return (c["node"], "V", int(tv[_VERT[reg]]))
    return (c["node"], "f", c["tri"])   # a persisting fallback whose nearest point is now inside


def compare_contact_keys(gpu_contacts, orc_contacts, P_orc, rob, P_gpu=None):
    """Active contact sets equal, keyed by node and mesh feature, outside nodes with
    near-threshold decisions (element contacts: elements with near-threshold decisions);
    returns (n_compared, n_excluded)."""
    det = collision.detect(P_orc, rob.mesh, rob.r_c, rob.delta) if rob.mesh is not None else []
    amb = {c["node"] for c in det if c["ambiguous"]}
    if rob.mesh is not None and rob.elements:
        amb_e = {c["node"] for c in collision.detect_elements(P_orc, rob.mesh, rob.r_c, rob.delta)
                 if c["ambiguous"]}
    else:
        amb_e = set()
    skip = lambda c: (c["node"] in amb_e) if c["kind"] == collision.ELEMENT else (c["node"] in amb)
    Pg = P_orc if P_gpu is None else P_gpu
    g = {feature_key(c, Pg, rob.mesh) for c in gpu_contacts if c["force"] > 0 and not skip(c)}
    o = {feature_key(c, P_orc, rob.mesh) for c, y in orc_contacts if y > 0 and not skip(c)}
    assert g == o, (sorted(g ^ o), sorted(amb), sorted(amb_e))
    return len(o), len(amb) + len(amb_e)


def same_contacts(a, b):
    """Two fem_contacts lists are identical, field by field (bitwise)."""
    if len(a) != len(b):
        return False
    for x, y in zip(a, b):
        if {k: x[k] for k in x if k != "n"} != {k: y[k] for k in y if k != "n"}:
            return False
        if not np.array_equal(x["n"], y["n"]):
            return False
    return True


def check_equilibrium_state(rob, X, contacts, info, depth, act_values, act_kind=0, tol=1e-10,
                            stag_tol=1e-9):
    """What the oracle computes at any size about a GPU state that the GPU reports converged:
      * equilibrium (eq. 19): the oracle's FP64 out-of-balance force at the GPU state minus the
        GPU's contact forces vanishes over the free DOFs, to the Newton tolerance or the
        stagnation level, and equals the residual the GPU reported;
      * detection (Sec. III-C): the oracle's detection at the GPU state finds the GPU's contact
        set, keyed by node and mesh feature, outside nodes with near-threshold decisions; any
        other GPU entry is a persisting contact still within the band of its triangle (an
        edge/vertex one also on the triangle's inner side);
      * the contact conditions of eq. 12: forces >= 0, gaps >= -1e-9 m, force x gap = 0.
    Returns the number of contacts checked."""
    from paper_2503_06922_amd.fem import state_to_PR
    band = rob.r_c + rob.delta
    lim = max(tol, solver.stagnation_tol(rob, stag_tol))
    P, R = state_to_PR(X)
    guided = rob.guided(depth)
    F = solver.out_of_balance(rob, P, R, act_kind, act_values)
    y = np.array([c["force"] for c in contacts])
    rn = float(np.linalg.norm(solver.contact_residual(F, contacts, y, rob, guided)))
    assert rn <= lim * 1.001, ("residual", rn, lim)
    assert abs(rn - info["res_norm"]) <= 1e-9, ("reported residual", rn, info["res_norm"])
    det = collision.detect(P, rob.mesh, rob.r_c, rob.delta, skip=guided)
    amb = {c["node"] for c in det if c["ambiguous"]}
    orc = {feature_key(c, P, rob.mesh): c for c in det if c["tri"] >= 0 and c["node"] not in amb}
    gpu = {feature_key(c, P, rob.mesh): c for c in contacts if c["node"] not in amb}
    missing = sorted(set(orc) - set(gpu))
    assert not missing, ("detection", missing)
    for key in sorted(set(gpu) - set(orc)):
        # a persisting contact: the oracle's closest point of that triangle is within the band;
        # an edge/vertex one also has the node on the triangle's inner side
        c = gpu[key]
        node, tri = c["node"], c["tri"]
        cpt, _, _ = collision.closest_points(P[node], rob.mesh, np.array([tri]))
        assert np.linalg.norm(P[node] - cpt[0]) <= band + 1e-12, ("persisting", node, tri)
        if c["kind"] != 0:
            assert rob.mesh.n[tri] @ (P[node] - rob.mesh.v0[tri]) > 0.0, ("persisting", node, tri)
    for c in contacts:
        assert c["force"] >= 0.0
        assert c["gap"] >= -1e-9, ("gap", c)
        assert c["force"] * c["gap"] <= 1e-9 * max(c["force"], 1e-12) + 1e-15, ("complementarity", c)
    return len(contacts)
