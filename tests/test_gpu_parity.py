"""GPU parity tests: the HIP path through the C ABI against the FP64 oracle."""
import numpy as np
import pytest

from oracle import solver, collision, beam, actuation
from workloads import make_config, load_schedule, robots_for_config
from tests.gpu_helpers import (gpu_context, robot_slices, oracle_robots, displacement_error,
                               node_forces, compare_contact_keys)

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


def _perturbed_states(rb, rng, scale_p=2e-3, scale_r=0.3):
    """Random smooth deformations of each robot's reference state (node-major [N,7])."""
    from paper_2503_06922_amd.fem import state_to_PR
    robs, _ = oracle_robots(rb)
    X = []
    PR = []
    for rob in robs:
        P, R = rob.reference()
        n = P.shape[0]
        s = np.linspace(0, 1, n)[:, None]
        dX = np.zeros((n, 6))
        dX[:, 0:3] = scale_p * np.sin(np.pi * s * rng.uniform(1, 3, size=3)) * rng.normal(size=3)
        dX[:, 3:6] = scale_r * np.sin(np.pi * s * rng.uniform(1, 3, size=3)) * rng.normal(size=3)
        P, R = beam.apply_increment(P, R, dX)
        q = np.array([_quat(Ri) for Ri in R])
        X.append(np.concatenate([P, q], axis=1))
        PR.append((P, R))
    return np.concatenate(X, axis=0), PR


def _quat(R):
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(R).as_quat()
    return np.array([w, x, y, z])


@pytest.mark.parametrize("mixed", [False, True])
def test_element_update_matches_oracle(mixed):
    """F, diagonal and coupling blocks of the QP tangent at deformed states (several robots).
    Plain FP64: F within 1e-12 and the blocks within 1e-13 of their largest entries.  Mixed
    precision far from convergence (the residual of a fresh load step is unknown, so above the
    FP32 level): element forces in FP32 with FP32 accumulation from FP64 geometry, within 1e-6
    of the largest force (a few FP32 roundings of the element forces, which here are of the
    size of the node forces); tangent blocks from the FP32 chord directions within 1e-6."""
    from paper_2503_06922_amd import fem
    rb = robots_for_config(3, n_robots=6)
    rng = np.random.default_rng(1)
    ctx = gpu_context(rb, precision=fem.FEM_MIXED if mixed else fem.FEM_FP64)
    T = rb.tensions
    ctx.fem_set_actuation(0, T.ravel(), np.zeros(rb.n_robots))
    X, PR = _perturbed_states(rb, rng)
    ctx.fem_set_state(X)
    F, KD, KS = ctx.fem_eval()
    robs, _ = oracle_robots(rb)
    for b, (sl, rob) in enumerate(zip(robot_slices(rb), robs)):
        P, R = PR[b]
        Fo = solver.out_of_balance(rob, P, R, actuation.CABLES, T[b])
        n = P.shape[0]
        Ko = beam.upper_banded_to_dense(beam.tangent_qp_upper_banded(P, R, rob.K12), 6 * n)
        KDo = np.array([Ko[6 * i:6 * i + 6, 6 * i:6 * i + 6] for i in range(n)])
        KSo = np.array([Ko[6 * i:6 * i + 6, 6 * i + 6:6 * i + 12] for i in range(n - 1)])
        fs = np.abs(Fo).max()
        ks = np.abs(Ko).max()
        tf, tk = (1e-6, 1e-6) if mixed else (1e-12, 1e-13)
        print("robot", b, "force error", np.abs(F[sl] - Fo).max() / fs, "block error",
              max(np.abs(KD[sl] - KDo).max(), np.abs(KS[sl][:-1] - KSo).max()) / ks)
        assert np.abs(F[sl] - Fo).max() <= tf * fs + 1e-13
        if mixed:
            assert np.abs(F[sl] - Fo).max() > 1e-12 * fs     # the FP32 path did run
        assert np.abs(KD[sl] - KDo).max() <= tk * ks
        assert np.abs(KS[sl][:-1] - KSo).max() <= tk * ks


def test_detection_matches_oracle_brute_force():
    rb, V, T = make_config(1)
    mesh = collision.Mesh(V, T)
    rng = np.random.default_rng(2)
    # short robots whose nodes are scattered near the wall (no guide)
    rb3 = robots_for_config(3, n_robots=6)
    rb3.n_elem[:] = 24
    rb3.guide_len = 0.0
    ctx = gpu_context(rb3, V, T, contact_capacity=256)
    ctx.fem_set_actuation(0, np.zeros(3 * rb3.n_robots), np.zeros(rb3.n_robots))
    Xs = []
    Ps = []
    robs, _ = oracle_robots(rb3)
    for rob in robs:
        n = rob.n_elem + 1
        # random points inside the bounding region of the mesh near vertices
        vid = rng.choice(len(V), size=n)
        cen = mesh.centroid[rng.choice(len(T), size=n)]
        P = 0.85 * V[vid] + 0.15 * cen + rng.normal(size=(n, 3)) * 3e-4
        q = np.tile([1.0, 0, 0, 0], (n, 1))
        Xs.append(np.concatenate([P, q], axis=1))
        Ps.append(P)
    ctx.fem_set_state(np.concatenate(Xs))
    ctx.fem_eval()
    got = ctx.fem_contacts(-1)
    n_cmp = 0
    for b, (P, rob) in enumerate(zip(Ps, robs)):
        det = collision.detect(P, mesh, rob.r_c, rob.delta, cull=False)
        amb = {c["node"] for c in det if c["ambiguous"]}
        o = {(c["node"], c["tri"], c["kind"]) for c in det if c["tri"] >= 0 and c["node"] not in amb}
        g = {(c["node"], c["tri"], c["kind"]) for c in got if c["robot"] == b and c["node"] not in amb}
        assert g == o
        n_cmp += len(o)
        og = {(c["node"], c["tri"], c["kind"]): c for c in det if c["tri"] >= 0}
        for c in got:
            if c["robot"] == b and c["node"] not in amb:
                ref = og[(c["node"], c["tri"], c["kind"])]
                assert abs(c["gap"] - ref["gap"]) <= 1e-15
                assert np.abs(c["n"] - ref["n"]).max() <= 1e-12
    assert n_cmp > 20


@pytest.fixture(scope="module")
def cfg0_oracle():
    rb, V, T = make_config(0)
    robs, mesh = oracle_robots(rb, V, T)
    rob = robs[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(rb, k))
    P, R, traj = solver.solve_robot(rob, sched, rb.n_load_steps, tol=1e-13, stag_tol=1e-9)
    return rb, V, T, rob, traj


def test_cfg0_trajectory_parity(cfg0_oracle):
    """20 tension-ramp load steps of the straight-tube workload, step by step."""
    rb, V, T, rob, traj = cfg0_oracle
    ctx = gpu_context(rb, V, T, newton_tol=1e-13, stag_tol=1e-9, max_newton=200)
    ctx.fem_set_actuation(0, rb.tensions.ravel(), rb.depth)
    Pref, _ = rob.reference()
    n_active = 0
    for k in range(1, rb.n_load_steps + 1):
        d, t = load_schedule(rb, k)
        ctx.fem_set_actuation(0, t.ravel(), d)
        out = ctx.fem_solve(1)
        info = out["info"][0]
        o = traj[k - 1]
        assert info["status"] == 0 and o["info"]["status"] == solver.OK
        P = out["state"][:, 0:3]
        err = displacement_error(P, o["P"], Pref)
        assert err <= 1e-9, (k, err)
        gc = ctx.fem_contacts(0)
        n_cmp, _ = compare_contact_keys(gc, list(zip(o["contacts"], o["y"])), o["P"], rob)
        n_active += n_cmp
        fg = node_forces(gc, P.shape[0])
        fo = node_forces([dict(c, force=y) for c, y in zip(o["contacts"], o["y"])], P.shape[0])
        assert np.abs(fg - fo).max() <= 1e-7 * max(np.abs(fo).max(), 1e-12) + 1e-13
    assert n_active > 0


def test_cfg1_one_step_parity_from_oracle_states():
    """Insertion into the branching lumen: from the oracle's state at several load steps,
    one GPU load step must reproduce the oracle's next converged equilibrium."""
    rb, V, T = make_config(1)
    robs, mesh = oracle_robots(rb, V, T)
    rob = robs[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(rb, k))
    ctx = gpu_context(rb, V, T, newton_tol=1e-10, stag_tol=1e-9, max_newton=100)
    P, R = rob.reference()
    Pref = P.copy()
    checked = 0
    for k in range(1, 31):
        d, t = sched(k)
        P1, R1, cont, y, info = solver.solve_load_step(rob, P, R, rob.base_target(d), 0, t,
                                                       tol=1e-10, stag_tol=1e-9, max_iter=100,
                                                       guided=rob.guided(d))
        if k % 3 == 0 and info["status"] == solver.OK:
            X = np.concatenate([P, np.array([_quat(Ri) for Ri in R])], axis=1)
            ctx.fem_set_state(X)
            dd, tt = sched(k - 1) if k > 1 else (0.0, np.zeros(3))
            ctx.fem_set_actuation(0, np.atleast_1d(tt), np.atleast_1d(dd))
            ctx.fem_solve(0)
            ctx.fem_set_actuation(0, np.atleast_1d(t), np.atleast_1d(d))
            out = ctx.fem_solve(1)
            assert out["info"][0]["status"] == 0
            err = displacement_error(out["state"][:, 0:3], P1, Pref)
            assert err <= 1e-9, (k, err)
            compare_contact_keys(ctx.fem_contacts(0), list(zip(cont, y)), P1, rob)
            checked += 1
        P, R = P1, R1
    assert checked >= 5


def test_cfg0_mixed_precision_matches_oracle(cfg0_oracle):
    """Mixed precision (FP32 tangent blocks and detection screen, FP64 residual and
    factorisation): same equilibria within 1e-5 relative tip error and the same active sets."""
    from paper_2503_06922_amd import fem
    rb, V, T, rob, traj = cfg0_oracle
    ctx = gpu_context(rb, V, T, precision=fem.FEM_MIXED, newton_tol=1e-13, stag_tol=1e-9,
                      max_newton=200)
    Pref, _ = rob.reference()
    worst = 0.0
    for k in range(1, rb.n_load_steps + 1):
        d, t = load_schedule(rb, k)
        ctx.fem_set_actuation(0, t.ravel(), d)
        out = ctx.fem_solve(1)
        o = traj[k - 1]
        assert out["info"][0]["status"] == 0
        P = out["state"][:, 0:3]
        tip = np.linalg.norm(P[-1] - o["P"][-1]) / rob.length
        worst = max(worst, tip)
        assert tip <= 1e-5
        assert displacement_error(P, o["P"], Pref) <= 1e-7
        compare_contact_keys(ctx.fem_contacts(0), list(zip(o["contacts"], o["y"])), o["P"], rob)
    print("mixed worst relative tip error", worst)


def test_batched_robots_match_oracle_per_robot():
    """A batch of robots of different lengths in one context: each robot equals its own
    oracle solve (several insertion load steps through the guide into the airway)."""
    rb, V, T = make_config(3)
    sub = rb.subset([0, 1, 2, 3, 5, 8])
    robs, mesh = oracle_robots(sub, V, T)
    ctx = gpu_context(sub, V, T, newton_tol=1e-10, stag_tol=1e-9, max_newton=100)
    n_steps = 6
    states = [r.reference() for r in robs]
    for k in range(1, n_steps + 1):
        d, t = load_schedule(sub, k)
        ctx.fem_set_actuation(0, t.ravel(), d)
        out = ctx.fem_solve(1)
        for b, (sl, rob) in enumerate(zip(robot_slices(sub), robs)):
            P, R = states[b]
            P1, R1, cont, y, info = solver.solve_load_step(rob, P, R, rob.base_target(d[b]), 0, t[b],
                                                           tol=1e-10, stag_tol=1e-9, max_iter=100,
                                                           guided=rob.guided(d[b]))
            states[b] = (P1, R1)
            assert out["info"][b]["status"] == (0 if info["status"] == solver.OK else 1)
            if info["status"] == solver.OK:
                Pref = rob.reference()[0]
                assert displacement_error(out["state"][sl, 0:3], P1, Pref) <= 1e-9


def test_edge_cases_single_element_and_no_lumen():
    """One element, no wall: a dead tip force gives the cantilever closed form of the element."""
    from paper_2503_06922_amd import fem
    rb = robots_for_config(0)
    rb.n_elem[:] = 1
    ctx = gpu_context(rb, None, None, newton_tol=1e-13, stag_tol=1e-9, max_newton=50)
    EI = np.pi / 4 * (rb.r_out**4 - rb.r_in**4) * rb.E
    L = rb.length[0]
    P = 1e-4 * 3 * EI / L**2
    ctx.fem_set_actuation(fem.FEM_ACT_TIP_WRENCH_GLOBAL, np.array([P, 0, 0, 0, 0, 0]), None)
    out = ctx.fem_solve(1)
    assert out["info"][0]["status"] == 0
    X = out["state"]
    assert X.shape == (2, 7)
    assert X[1, 0] == pytest.approx(P * L**3 / (3 * EI), rel=1e-6)
    assert ctx.fem_contacts(-1) == []


def test_invalid_calls_report_errors():
    from paper_2503_06922_amd import fem
    rb = robots_for_config(0)
    ctx = fem.Context(fem.params_from_batch(rb))
    with pytest.raises(fem.FemError) as e:
        ctx.fem_solve(1)
    assert e.value.status == fem.FEM_E_STATE
    with pytest.raises(fem.FemError) as e:
        ctx.fem_set_lumen(np.zeros((3, 3)), np.array([[0, 1, 5]], np.int32))
    assert e.value.status == fem.FEM_E_INVAL
    with pytest.raises(fem.FemError):
        ctx.fem_contacts(7)


def test_short_robots_match_oracle():
    """Robots of 2, 3, 4, 5 and 7 elements (the two-ended elimination with an empty tip side,
    one node per side, ...) pushed into the straight tube by a dead lateral tip force sized to
    deflect each free robot by 5 mm; every load step against the oracle per robot."""
    from paper_2503_06922_amd import fem
    rb0, V, T = make_config(0)
    ne = [2, 3, 4, 5, 7]
    rb = rb0.subset([0] * len(ne))
    rb.n_elem[:] = ne
    rb.length[:] = 0.015 * np.asarray(ne, float)
    EI = np.pi / 4 * (rb.r_out**4 - rb.r_in**4) * rb.E
    W = np.zeros((len(ne), 6))
    W[:, 1] = -3 * EI * 5e-3 / rb.length**3
    robs, mesh = oracle_robots(rb, V, T)
    ctx = gpu_context(rb, V, T, newton_tol=1e-12, stag_tol=1e-9, max_newton=100)
    n_steps = 5
    trajs = []
    for b, rob in enumerate(robs):
        _, _, traj = solver.solve_robot(rob, lambda k, b=b: (0.0, W[b] * k / n_steps), n_steps,
                                        act_kind=actuation.TIP_GLOBAL, tol=1e-12, stag_tol=1e-9)
        trajs.append(traj)
    n_active = 0
    for k in range(1, n_steps + 1):
        ctx.fem_set_actuation(fem.FEM_ACT_TIP_WRENCH_GLOBAL, (W * k / n_steps).ravel(), None)
        out = ctx.fem_solve(1)
        for b, (sl, rob) in enumerate(zip(robot_slices(rb), robs)):
            o = trajs[b][k - 1]
            assert out["info"][b]["status"] == 0 and o["info"]["status"] == solver.OK, (b, k)
            Pref = rob.reference()[0]
            assert displacement_error(out["state"][sl, 0:3], o["P"], Pref) <= 1e-9, (b, k)
            n_cmp, _ = compare_contact_keys(ctx.fem_contacts(b), list(zip(o["contacts"], o["y"])),
                                            o["P"], rob)
            n_active += n_cmp
    assert n_active > 0


@pytest.mark.parametrize("robot,n_elem,n_steps", [(2950, 116, 24), (1509, 240, 27)])
def test_contact_cycles_and_dependent_contacts_converge_like_oracle(robot, n_elem, n_steps):
    """Two robots of the batched workload: robot 2950, whose tip node at load step 24 used to
    alternate between a detected face and an edge fallback on every iteration (60 iterations,
    not converged; fixed by persisting edge/vertex contacts), and robot 1509, whose LCP at
    load step 27 meets a contact that depends linearly on the active ones (the active-set
    method used to give up; fixed by the exchange along a null direction of W).  The GPU and
    the oracle converge on every load step to the same state and active set."""
    rb, V, T = make_config(3)
    sub = rb.subset([robot])
    assert int(sub.n_elem[0]) == n_elem
    robs, mesh = oracle_robots(sub, V, T)
    rob = robs[0]
    ctx = gpu_context(sub, V, T, newton_tol=1e-10, stag_tol=1e-9, max_newton=60)
    P, R = rob.reference()
    Pref = P.copy()
    for k in range(1, n_steps + 1):
        d, t = load_schedule(sub, k)
        ctx.fem_set_actuation(0, t.ravel(), d)
        out = ctx.fem_solve(1)
        P, R, cont, y, info = solver.solve_load_step(rob, P, R, rob.base_target(d[0]), 0, t[0],
                                                     tol=1e-10, stag_tol=1e-9, max_iter=60,
                                                     guided=rob.guided(d[0]))
        assert info["status"] == solver.OK and out["info"][0]["status"] == 0, k
        assert displacement_error(out["state"][:, 0:3], P, Pref) <= 1e-9, k
        compare_contact_keys(ctx.fem_contacts(0), list(zip(cont, y)), P, rob)
    ctx.close()


@pytest.mark.parametrize("mixed,disp_tol", [(True, 1e-5), (False, 1e-9)])
def test_full_batch_in_bench_configuration_sampled_robots(mixed, disp_tol):
    """All 4096 robots of the batched insertion in the launch configuration of the benchmark
    (contact capacity 512, at most 60 Newton iterations; mixed precision as timed, and plain
    FP64) through its first 12 load steps, where the first contacts appear; six seeded robots
    against their own oracle solves at every load step: same status, displacement within
    1e-5 (mixed) / 1e-9 (FP64) and tip within 1e-5 of the robot length, identical active
    sets.  Plain FP64 follows the oracle's own iteration path, so both stop at the same
    iterate; the mixed path takes FP32 element forces while the residual is large, a
    different path to the same equilibrium, which the residual tolerance of 1e-10 N fixes
    only to about 2e-7 of the displacement here."""
    from paper_2503_06922_amd import fem
    rb, V, T = make_config(3)
    assert rb.n_robots == 4096
    pick = sorted(np.random.default_rng(2025).choice(rb.n_robots, size=6, replace=False).tolist())
    sub = rb.subset(pick)
    robs, mesh = oracle_robots(sub, V, T)
    ctx = gpu_context(rb, V, T, precision=fem.FEM_MIXED if mixed else fem.FEM_FP64,
                      newton_tol=1e-10, stag_tol=1e-9, max_newton=60, contact_capacity=512)
    states = [r.reference() for r in robs]
    slices = robot_slices(rb)
    n_active = 0
    for k in range(1, 13):
        d, t = load_schedule(rb, k)
        ctx.fem_set_actuation(0, t.ravel(), d)
        out = ctx.fem_solve(1)
        for j, (b, rob) in enumerate(zip(pick, robs)):
            P, R = states[j]
            P, R, cont, y, info = solver.solve_load_step(rob, P, R, rob.base_target(d[b]), 0, t[b],
                                                         tol=1e-10, stag_tol=1e-9, max_iter=60,
                                                         guided=rob.guided(d[b]))
            states[j] = (P, R)
            assert out["info"][b]["status"] == (0 if info["status"] == solver.OK else 1), (k, b)
            Pg = out["state"][slices[b], 0:3]
            assert displacement_error(Pg, P, rob.reference()[0]) <= disp_tol, (k, b)
            assert np.linalg.norm(Pg[-1] - P[-1]) / rob.length <= 1e-5, (k, b)
            n_cmp, _ = compare_contact_keys(ctx.fem_contacts(b), list(zip(cont, y)), P, rob)
            n_active += n_cmp
    ctx.close()
    assert n_active > 0
