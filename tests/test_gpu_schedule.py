"""GPU tests of the load-stepping loop: every robot advancing through an explicit schedule on
its own (fem_solve_schedule, graph-replayed passes) against one call per load step."""
import numpy as np
import pytest

from workloads import make_config, load_schedule, schedule_table
from tests.gpu_helpers import gpu_context, robot_slices, same_contacts

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mixed", [False, True])
def test_schedule_equals_one_call_per_load_step(mixed):
    """64 robots of the batched insertion, the first 24 load steps of its schedule (tensions
    ramped over 10, depth over 100): the robots run through the schedule on their own in one
    call, and give bit-identical per-step tips and statuses, final states, solve records and
    contacts as 24 calls of fem_set_actuation + fem_solve(1), where every robot waits for the
    slowest at every load step."""
    from paper_2503_06922_amd import fem
    rb, V, T = make_config(3)
    sub = rb.subset(np.arange(0, 4096, 64))
    n = 24
    kw = dict(precision=fem.FEM_MIXED if mixed else fem.FEM_FP64, newton_tol=1e-10, stag_tol=1e-9,
              max_newton=60, contact_capacity=512)
    a = gpu_context(sub, V, T, **kw)
    tips = np.empty((n, sub.n_robots, 3))
    stat = np.empty((n, sub.n_robots), np.int32)
    iters = np.empty((n, sub.n_robots), np.int32)
    sl = robot_slices(sub)
    for k in range(1, n + 1):
        d, t = load_schedule(sub, k)
        a.fem_set_actuation(fem.FEM_ACT_CABLES, t.ravel(), d)
        o = a.fem_solve(1)
        tips[k - 1] = np.array([o["state"][s][-1, 0:3] for s in sl])
        stat[k - 1] = [i["status"] for i in o["info"]]
        iters[k - 1] = [i["iters"] for i in o["info"]]
    b = gpu_context(sub, V, T, **kw)
    vals, deps = schedule_table(sub, n)
    ob = b.fem_solve_schedule(fem.FEM_ACT_CABLES, vals, deps)
    assert np.array_equal(ob["rec_status"], stat)
    assert np.array_equal(ob["rec_iters"], iters)
    assert np.array_equal(ob["rec_tip"], tips)
    assert np.array_equal(ob["state"], o["state"])
    assert ob["info"] == o["info"]
    assert same_contacts(a.fem_contacts(-1), b.fem_contacts(-1))
    assert (stat == 0).mean() > 0.8 and all(i["steps_total"] == n for i in ob["info"])
    # a later ramp starts from the schedule's last values: one more load step at the same load
    d, t = load_schedule(sub, n)
    a.fem_set_actuation(fem.FEM_ACT_CABLES, t.ravel(), d)
    b.fem_set_actuation(fem.FEM_ACT_CABLES, t.ravel(), d)
    assert np.array_equal(a.fem_solve(1)["state"], b.fem_solve(1)["state"])
    a.close()
    b.close()


def test_schedule_invalid_calls():
    from paper_2503_06922_amd import fem
    rb, V, T = make_config(0)
    ctx = gpu_context(rb, V, T)
    vals = np.zeros((3, 1, 3))
    with pytest.raises(fem.FemError) as e:
        ctx.fem_solve_schedule(fem.FEM_ACT_CABLES, np.zeros((0, 1, 3)))
    assert e.value.status == fem.FEM_E_INVAL
    ctx.fem_solve_schedule(fem.FEM_ACT_CABLES, vals)
    with pytest.raises(fem.FemError) as e:
        ctx.fem_solve_schedule(fem.FEM_ACT_TIP_WRENCH_LOCAL, np.zeros((3, 1, 6)))
    assert e.value.status == fem.FEM_E_INVAL
    ctx.close()


def test_autotuned_launch_shapes_give_identical_results():
    """A context created with autotune = 1 times the candidate launch shapes of the element
    update (64/128/256 threads per block) and of detection (4/8/16 lanes per node) during its
    first solve and keeps the fastest; the results are bit-identical to those of the default
    shapes (256, 8), on 64 robots of the batched insertion through 12 load steps (tuned at the
    end of the first call, which is shorter than the tuning point) and 12 more."""
    from paper_2503_06922_amd import fem
    rb, V, T = make_config(3)
    sub = rb.subset(np.arange(0, 4096, 64))
    kw = dict(precision=fem.FEM_MIXED, newton_tol=1e-10, stag_tol=1e-9, max_newton=60,
              contact_capacity=512)
    a = gpu_context(sub, V, T, **kw)
    b = gpu_context(sub, V, T, autotune=1, **kw)
    assert a.fem_tuning()[:2] == (256, 8) and np.all(np.isnan(a.fem_tuning()[2]))
    vals, deps = schedule_table(sub, 24)
    a.fem_solve_schedule(fem.FEM_ACT_CABLES, vals[:12], deps[:12])
    b.fem_solve_schedule(fem.FEM_ACT_CABLES, vals[:12], deps[:12])
    oa = a.fem_solve_schedule(fem.FEM_ACT_CABLES, vals[12:], deps[12:])
    ob = b.fem_solve_schedule(fem.FEM_ACT_CABLES, vals[12:], deps[12:])
    blk, lanes, t = b.fem_tuning()
    print("tuned shapes", blk, lanes, "times us", t)
    assert blk in (64, 128, 256) and lanes in (4, 8, 16) and np.all(np.isfinite(t)) and np.all(t > 0)
    assert np.array_equal(oa["state"], ob["state"])
    assert oa["info"] == ob["info"]
    assert np.array_equal(oa["rec_tip"], ob["rec_tip"])
    assert same_contacts(a.fem_contacts(-1), b.fem_contacts(-1))
    a.close()
    b.close()
