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
    """Per-node contact force vectors sum_c y_c n_c (unique even when y is not)."""
    f = np.zeros((n_nodes, 3))
    for c in contacts:
        f[c["node"]] += c[ykey] * np.asarray(c["n"])
    return f


def compare_contact_keys(gpu_contacts, orc_contacts, P_orc, rob):
    """Active (node, tri, kind) sets equal outside ambiguous nodes; returns (n_compared, n_excluded)."""
    det = collision.detect(P_orc, rob.mesh, rob.r_c, rob.delta) if rob.mesh is not None else []
    amb = {c["node"] for c in det if c["ambiguous"]}
    g = {(c["node"], c["tri"], c["kind"]) for c in gpu_contacts if c["force"] > 0 and c["node"] not in amb}
    o = {(c["node"], c["tri"], c["kind"]) for c, y in orc_contacts if y > 0 and c["node"] not in amb}
    assert g == o, (sorted(g ^ o), sorted(amb))
    return len(o), len(amb)


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
