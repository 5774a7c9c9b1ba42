"""Full-size checks of the 1000-element robot inserted into the 200k-triangle lumen.

The oracle cannot follow this insertion (minutes per load step), so the GPU's converged states
are checked, at sampled load steps, against what the oracle computes at any size:
  * equilibrium (eq. 19): the oracle's FP64 out-of-balance force at the GPU state, minus the
    GPU's contact forces, vanishes over the free DOFs (to the Newton tolerance or the rounding
    floor of the stagnation test) and equals the residual the GPU reported;
  * detection (Sec. III-C): the oracle's brute-force (k-d-tree culled) detection at the GPU
    state finds the GPU's contact set, keyed by node and mesh feature (an edge/vertex contact
    constrains against the edge or vertex that holds the nearest point, whichever of the
    triangles sharing it carries the index), outside nodes with near-threshold decisions; any
    other GPU entry is a persisting contact still within the band of its triangle;
  * the contact conditions of eq. 12: forces >= 0, gaps >= 0 to the tolerance, force x gap = 0;
  * mixed precision against the FP64 GPU path: relative tip error <= 1e-5.
"""
import numpy as np
import pytest

from oracle import solver, collision
from workloads import make_config, load_schedule
from tests.gpu_helpers import gpu_context, oracle_robots, check_equilibrium_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def config2_runs():
    from paper_2503_06922_amd import fem
    rb, V, T = make_config(2)
    robs, mesh = oracle_robots(rb, V, T)
    kw = dict(newton_tol=1e-10, stag_tol=1e-9, max_newton=60, contact_capacity=256)
    ctx_m = gpu_context(rb, V, T, precision=fem.FEM_MIXED, **kw)
    ctx_d = gpu_context(rb, V, T, precision=fem.FEM_FP64, **kw)
    samples = []
    for k in range(1, rb.n_load_steps + 1):
        d, t = load_schedule(rb, k)
        outs = []
        for ctx in (ctx_m, ctx_d):
            ctx.fem_set_actuation(0, t.ravel(), d)
            outs.append(ctx.fem_solve(1))
        if k % 10 == 0:
            samples.append(dict(k=k, depth=float(d[0]), t=t[0].copy(),
                                info_m=outs[0]["info"][0], info_d=outs[1]["info"][0],
                                X_m=outs[0]["state"], X_d=outs[1]["state"],
                                contacts_m=ctx_m.fem_contacts(0)))
    ctx_m.close()
    ctx_d.close()
    return rb, robs[0], samples


def test_config2_mixed_matches_fp64(config2_runs):
    rb, rob, samples = config2_runs
    both = [s for s in samples if s["info_m"]["status"] == 0 and s["info_d"]["status"] == 0]
    assert len(both) >= 6
    for s in both:
        tip = np.linalg.norm(s["X_m"][-1, 0:3] - s["X_d"][-1, 0:3]) / rob.length
        assert tip <= 1e-5, (s["k"], tip)


def test_config2_equilibrium_detection_complementarity(config2_runs):
    rb, rob, samples = config2_runs
    checked = 0
    n_contacts = 0
    for s in samples:
        if s["info_m"]["status"] != 0:
            continue
        n_contacts += check_equilibrium_state(rob, s["X_m"], s["contacts_m"], s["info_m"], s["depth"],
                                              s["t"])
        checked += 1
    assert checked >= 6 and n_contacts > 0
