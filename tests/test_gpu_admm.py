"""GPU tests of the ADMM variant of the linear step (qp_solver = FEM_QP_ADMM: the OSQP
iteration the paper uses, on the block-tridiagonal factor of K + sigma I + rho A^T A).

* Against the oracle's own ADMM Newton iteration (oracle/admm.py, the same iteration): the
  straight-tube robot through its tension ramp, every load step.
* Against the exact method (Schur complement + LCP) at equal tolerance: the same equilibria,
  on the straight tube and on robots of the batched insertion.
Both Newton iterations stop at a residual below the tolerance, which fixes positions only to
within the robot's compliance times the residuals (C_MAX = a cantilever of the robot's length
in its softest section)."""
import time

import numpy as np
import pytest

from oracle import solver
from workloads import make_config, load_schedule
from tests.gpu_helpers import gpu_context, oracle_robots, robot_slices

pytestmark = pytest.mark.gpu

RHO, EPS = 1.0, 1e-11


def _bound(rob, scale, res):
    C = rob.length ** 3 / (3.0 * float(np.min(rob.EI)))
    return 1e-9 * scale + C * res


def test_admm_trajectory_matches_oracle_admm():
    from paper_2503_06922_amd import fem
    rb, V, T = make_config(0)
    robs, _ = oracle_robots(rb, V, T)
    rob = robs[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(rb, k))
    _, _, traj = solver.solve_robot(rob, sched, 20, tol=1e-10, stag_tol=1e-9, max_iter=100,
                                    qp=dict(rho=RHO, eps=EPS))
    ctx = gpu_context(rb, V, T, newton_tol=1e-10, stag_tol=1e-9, max_newton=100,
                      qp_solver=fem.FEM_QP_ADMM, admm_rho=RHO, admm_eps=EPS)
    P0 = rob.reference()[0]
    scale = max(np.linalg.norm(s["P"] - P0, axis=1).max() for s in traj)
    qp_g = qp_o = 0
    for k in range(1, 21):
        d, t = load_schedule(rb, k)
        ctx.fem_set_actuation(fem.FEM_ACT_CABLES, t.ravel(), d)
        o = ctx.fem_solve(1)
        i = o["info"][0]
        s = traj[k - 1]
        assert i["status"] == 0 and s["info"]["status"] == solver.OK, k
        err = np.linalg.norm(o["state"][:, 0:3] - s["P"], axis=1).max()
        assert err <= _bound(rob, scale, i["res_norm"] + s["info"]["res_norm"]), (k, err)
        qp_o += s["info"]["qp_iters"]
    qp_g = o["info"][0]["qp_iters_total"]
    print("ADMM iterations over the ramp: GPU", qp_g, "oracle", qp_o)
    assert qp_g > 0 and abs(qp_g - qp_o) <= 0.05 * qp_o
    ctx.close()


@pytest.mark.parametrize("cfg,n_steps", [(0, 20), (3, 12)])
def test_admm_matches_exact_method_at_equal_tolerance(cfg, n_steps):
    """The same robots through the same load steps with the exact QP solution and with ADMM
    steps (both Newton iterations to 1e-10 N): the same statuses and equilibria within the
    residual bound; the time per Newton iteration of each is printed."""
    from paper_2503_06922_amd import fem
    rb, V, T = make_config(cfg)
    if cfg == 3:
        rb = rb.subset([527, 2767])
    robs, _ = oracle_robots(rb, V, T)
    kw = dict(newton_tol=1e-10, stag_tol=1e-9, max_newton=100, contact_capacity=512)
    ex = gpu_context(rb, V, T, **kw)
    ad = gpu_context(rb, V, T, qp_solver=fem.FEM_QP_ADMM, admm_rho=RHO, admm_eps=EPS, **kw)
    sl = robot_slices(rb)
    times = {}
    worst = 0.0
    n_cmp = 0
    P0 = [r.reference()[0] for r in robs]
    scale = [1e-3] * rb.n_robots
    for k in range(1, n_steps + 1):
        print("config", cfg, "load step", k, flush=True)
        d, t = load_schedule(rb, k)
        outs = []
        for name, ctx in (("exact", ex), ("admm", ad)):
            ctx.fem_set_actuation(fem.FEM_ACT_CABLES, t.ravel(), d)
            t0 = time.perf_counter()
            outs.append(ctx.fem_solve(1))
            times[name] = times.get(name, 0.0) + time.perf_counter() - t0
        oe, oa = outs
        for j, rob in enumerate(robs):
            ie, ia = oe["info"][j], oa["info"][j]
            assert ie["status"] == ia["status"], (k, j, ie["status"], ia["status"])
            if ie["status"] != 0:
                continue
            scale[j] = max(scale[j], np.linalg.norm(oe["state"][sl[j], 0:3] - P0[j], axis=1).max())
            err = np.linalg.norm(oe["state"][sl[j], 0:3] - oa["state"][sl[j], 0:3], axis=1).max()
            b = _bound(rob, scale[j], ie["res_norm"] + ia["res_norm"])
            worst = max(worst, err / b)
            n_cmp += 1
    it_e = sum(i["iters_total"] for i in oe["info"])
    it_a = sum(i["iters_total"] for i in oa["info"])
    qp = sum(i["qp_iters_total"] for i in oa["info"])
    print(f"config {cfg}: {n_cmp} load steps compared, worst error / bound {worst:.2e}; "
          f"exact {1e3 * times['exact'] / max(it_e, 1):.3f} ms per Newton iteration ({it_e} iterations), "
          f"ADMM {1e3 * times['admm'] / max(it_a, 1):.3f} ms ({it_a} iterations, {qp} ADMM iterations)")
    assert worst <= 1.0 and n_cmp >= 0.8 * n_steps * rb.n_robots
    ex.close()
    ad.close()
