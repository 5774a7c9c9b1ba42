"""Contact along an element (Sec. II-C, eq. 3-7 at 0 < xi < l0) on the GPU against the oracle:
detection of chords against the wall's edges and vertices (brute force), the knife-edge
propped cantilever (a single element contact; beam theory pins the oracle there), stored
oracle trajectories of lumen robots with element contacts, and the calls that do not support
them."""
import glob
import os

import numpy as np
import pytest

from oracle import actuation, collision, solver
from workloads import load_schedule, make_config, robots_for_config, schedule_table
from tests.element_fixtures import knife_edge_case
from tests.gpu_helpers import (compare_contact_keys, displacement_error, gpu_context, node_forces,
                               oracle_robots)

pytestmark = pytest.mark.gpu

FIX = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "element_oracle")


def test_element_detection_matches_oracle():
    """Robots whose nodes are scattered near the wall of the lumen: the GPU's element contacts
    (node, triangle, kind 2) equal the oracle's outside elements with near-threshold
    decisions; s at 1e-12, gaps at 1e-15, normals at 1e-10."""
    rb, V, T = make_config(1)
    mesh = collision.Mesh(V, T)
    rng = np.random.default_rng(7)
    rb3 = robots_for_config(3, n_robots=6)
    rb3.n_elem[:] = 24
    rb3.guide_len = 0.0
    ctx = gpu_context(rb3, V, T, contact_capacity=512, contact_along_elements=1)
    ctx.fem_set_actuation(0, np.zeros(3 * rb3.n_robots), np.zeros(rb3.n_robots))
    robs, _ = oracle_robots(rb3)
    Xs, Ps = [], []
    for rob in robs:
        n = rob.n_elem + 1
        # pairs of nodes on either side of a wall vertex, so that chords pass by edges
        vid = rng.choice(len(V), size=n)
        nrm = mesh.n[rng.choice(len(T), size=n)]
        P = V[vid] + nrm * rng.uniform(1e-3, 3e-3, size=(n, 1)) + rng.normal(size=(n, 3)) * 2e-3
        q = np.tile([1.0, 0, 0, 0], (n, 1))
        Xs.append(np.concatenate([P, q], axis=1))
        Ps.append(P)
    ctx.fem_set_state(np.concatenate(Xs))
    print("GPU detection", flush=True)
    ctx.fem_eval()
    got = ctx.fem_contacts(-1)
    n_cmp = 0
    for b, (P, rob) in enumerate(zip(Ps, robs)):
        # the k-d-tree superset of the triangles that can reach the band (the same contacts
        # as every triangle: tests/test_oracle_element_contact.py)
        print("oracle detection, robot", b, flush=True)
        det = collision.detect_elements(P, mesh, rob.r_c, rob.delta, cull=True)
        amb = {c["node"] for c in det if c["ambiguous"]}
        o = {(c["node"], c["tri"]): c for c in det if c["tri"] >= 0 and c["node"] not in amb}
        g = {(c["node"], c["tri"]): c for c in got
             if c["robot"] == b and c["kind"] == collision.ELEMENT and c["node"] not in amb}
        assert set(g) == set(o), (b, sorted(set(g) ^ set(o)))
        for k, c in g.items():
            ref = o[k]
            assert abs(c["s"] - ref["s"]) <= 1e-12
            assert abs(c["gap"] - ref["gap"]) <= 1e-15
            # the normal turns with the chord point: a rounding difference ds of s (the closest
            # pair's 2x2 solve, amplified by up to 1/sin of the chord-edge angle) moves it by
            # l ds / |p - c|, up to a few 1e-12 here
            assert np.abs(c["n"] - ref["n"]).max() <= 1e-10
        n_cmp += len(o)
        # node contacts carry s = 0
        assert all(c["s"] == 0.0 for c in got if c["robot"] == b and c["kind"] != collision.ELEMENT)
    print("element contacts compared", n_cmp)
    assert n_cmp >= 10


def _knife_edge_gpu(u, elements, n_steps=1, **kw):
    from paper_2503_06922_amd import fem
    rb, V, T, a = knife_edge_case()
    ctx = gpu_context(rb, V, T, precision=fem.FEM_FP64, newton_tol=1e-13, stag_tol=1e-9,
                      max_newton=200, contact_along_elements=int(elements), **kw)
    for k in range(1, n_steps + 1):
        ctx.fem_set_actuation(fem.FEM_ACT_TIP_WRENCH_GLOBAL, np.asarray(u, float) * k / n_steps,
                              np.zeros(1))
        out = ctx.fem_solve(1)
    return ctx, out


@pytest.mark.parametrize("scale", [1e-4, 3e-3])
def test_knife_edge_matches_oracle(scale):
    """The propped cantilever (tip force towards the ridge, plus a sideways force and a twist
    at the larger load): GPU and oracle states agree to 1e-9 of the deflection, the element
    contact's s to 1e-9 and its force and the nodal contact forces to 1e-9."""
    rb, V, T, a = knife_edge_case()
    robs, mesh = oracle_robots(rb, V, T)
    rob = robs[0]
    rob.elements = True
    EI, L = rob.EI[0], rob.length
    P0 = scale * 3 * EI / L ** 2
    u = np.array([P0, 0.4 * P0, 0.0, 0.0, 0.0, 0.2 * P0 * L]) if scale > 1e-3 else np.array([P0, 0, 0, 0, 0, 0])
    n_steps = 2 if scale > 1e-3 else 1
    sched = lambda k: (0.0, u * k / n_steps)
    Po, Ro, traj = solver.solve_robot(rob, sched, n_steps, act_kind=actuation.TIP_GLOBAL, tol=1e-13,
                                      stag_tol=1e-9, max_iter=200)
    last = traj[-1]
    assert last["info"]["status"] == solver.OK
    ctx, out = _knife_edge_gpu(u, True, n_steps)
    assert out["info"][0]["status"] == 0
    Pg = out["state"][:, 0:3]
    Pref, _ = rob.reference()
    assert displacement_error(Pg, Po, Pref) <= 1e-9
    gc = ctx.fem_contacts(0)
    ge = [c for c in gc if c["force"] > 0]
    oe = [(c, y) for c, y in zip(last["contacts"], last["y"]) if y > 0]
    assert len(ge) == 1 and ge[0]["kind"] == collision.ELEMENT and ge[0]["node"] == 7
    assert len(oe) == 1
    assert abs(ge[0]["s"] - oe[0][0]["s"]) <= 1e-9
    assert ge[0]["force"] == pytest.approx(oe[0][1], rel=1e-9)
    fg = node_forces(gc, Pg.shape[0])
    fo = node_forces([dict(c, force=y) for c, y in zip(last["contacts"], last["y"])], Pg.shape[0])
    assert np.abs(fg - fo).max() <= 1e-9 * np.abs(fo).max()
    compare_contact_keys(gc, list(zip(last["contacts"], last["y"])), Po, rob, Pg)
    ctx.close()


def test_knife_edge_without_element_contacts_passes_through():
    """With node contacts only, GPU and oracle agree that the chord crosses the ridge."""
    rb, V, T, a = knife_edge_case()
    rob = oracle_robots(rb, V, T)[0][0]
    EI, L = rob.EI[0], rob.length
    u = np.array([1e-4 * 3 * EI / L ** 2, 0, 0, 0, 0, 0])
    Po, Ro, traj = solver.solve_robot(rob, lambda k: (0.0, u), 1, act_kind=actuation.TIP_GLOBAL,
                                      tol=1e-13, stag_tol=1e-9, max_iter=200)
    ctx, out = _knife_edge_gpu(u, False)
    Pg = out["state"][:, 0:3]
    Pref, _ = rob.reference()
    assert out["info"][0]["status"] == 0 and ctx.fem_contacts(0) == []
    assert displacement_error(Pg, Po, Pref) <= 1e-9
    s = 0.3
    assert (1 - s) * Pg[7, 0] + s * Pg[8, 0] > 1e-6
    ctx.close()


def test_adjoint_rejects_active_element_contacts():
    """fem_grad does not support a robot with an active contact along an element: NaN and
    FEM_E_NOCONV, as its declaration states."""
    from paper_2503_06922_amd import fem
    rb, V, T, a = knife_edge_case()
    rob = oracle_robots(rb, V, T)[0][0]
    EI, L = rob.EI[0], rob.length
    ctx, out = _knife_edge_gpu([1e-4 * 3 * EI / L ** 2, 0, 0, 0, 0, 0], True)
    assert any(c["kind"] == collision.ELEMENT and c["force"] > 0 for c in ctx.fem_contacts(0))
    g, st = ctx.fem_grad(np.array([-1], np.int32), np.ones(3))
    assert st == fem.FEM_E_NOCONV and np.all(np.isnan(g))
    assert "along an element" in fem.lib().fem_last_error(ctx._h).decode()
    ctx.close()


def test_element_contacts_need_the_exact_qp_method():
    from paper_2503_06922_amd import fem
    rb, V, T, a = knife_edge_case()
    with pytest.raises(fem.FemError):
        gpu_context(rb, V, T, qp_solver=fem.FEM_QP_ADMM, contact_along_elements=1)
    with pytest.raises(fem.FemError):
        gpu_context(rb, V, T, contact_along_elements=2)


C_MAX = 450.0   # m/N: a cantilever of the robot's length in its softest section, L^3 / 3 EI


def test_lumen_trajectories_with_element_contacts_match_oracle():
    """Robots of the batched workload whose oracle trajectories (their first 40 load steps,
    element contacts on, tests/golden/element_oracle/) meet element contacts: load step by
    load step, with equal status and equal active sets (keyed by node and mesh feature,
    outside near-threshold decisions), the GPU's node positions agree with the oracle's within
    1e-9 of the largest deformation (beyond the rigid insertion) plus C_MAX (r_gpu + r_oracle):
    a load step stops at a residual below 1e-13 N or at the stagnation level, and a residual r
    fixes the equilibrium only to within the robot's compliance times r.  Every robot is
    compared over at least 25 load steps and at least 3 compared load steps hold an active
    element contact."""
    from paper_2503_06922_amd import fem
    files = sorted(glob.glob(os.path.join(FIX, "robot_*.npz")))
    assert files, "run tests/golden/make_element_oracle.py"
    rb, V, T = make_config(3)
    mesh = collision.Mesh(V, T)
    n_elem_steps = 0
    for f in files:
        with np.load(f) as z:
            fx = {k: z[k] for k in z.files}
        b = int(fx["robot"])
        sub = rb.subset([b])
        rob = solver.robots_from_batch(sub, mesh)[0]
        rob.elements = True
        nsteps = int(fx["status"].shape[0])
        vals, deps = schedule_table(sub, nsteps)
        ctx = gpu_context(sub, V, T, precision=fem.FEM_FP64, newton_tol=1e-13, stag_tol=1e-9,
                          max_newton=100, contact_capacity=512, contact_along_elements=1)
        P0 = rob.reference()[0]
        unit = rob.base_dir / np.linalg.norm(rob.base_dir)
        rigid = lambda k: P0 + load_schedule(sub, k)[0][0] * unit
        d_scale = max(np.linalg.norm(fx["P"][k] - rigid(k + 1), axis=1).max() for k in range(nsteps))
        n_cmp = 0
        for k in range(nsteps):
            ctx.fem_set_actuation(0, vals[k].ravel(), deps[k])
            out = ctx.fem_solve(1)
            st = out["info"][0]["status"]
            if st != 0 or int(fx["status"][k]) != 0:
                print("robot", b, "load step", k + 1, "status gpu", st, "oracle", int(fx["status"][k]))
                assert (st == 0) == (int(fx["status"][k]) == 0)
                break
            Pg = out["state"][:, 0:3]
            Po = fx["P"][k]
            act = fx["act"][k]
            oc = [(dict(node=int(a_[0]), tri=int(a_[1]), kind=int(a_[2]), s=float(a_[3]), n=a_[4:7],
                        gap=0.0), float(a_[7])) for a_ in act[act[:, 0] >= 0]]
            gc = ctx.fem_contacts(0)
            compare_contact_keys(gc, oc, Po, rob, Pg)
            bound = max(1e-9 * d_scale, 1e-11) + C_MAX * (float(fx["res_norm"][k]) + out["info"][0]["res_norm"])
            err = np.linalg.norm(Pg - Po, axis=1).max()
            assert err <= bound, (b, k + 1, err, bound)
            n_cmp += 1
            n_elem_steps += any(c["kind"] == collision.ELEMENT and c["force"] > 0 for c in gc)
        print("robot", b, "load steps compared", n_cmp)
        assert n_cmp >= 25
        ctx.close()
    print("load steps with an active element contact:", n_elem_steps)
    assert n_elem_steps >= 3
