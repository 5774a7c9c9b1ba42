"""Benchmark: batched contact-FEM solves per second on one MI355X.

Workload (the batched configuration): 4096 robots with 50..400 elements
(L = 0.6 m, stiff shaft + 70 mm tube tip), tensions U(0,3) N ramped over 10
load steps and insertion depths U(0.1,0.5) m over 100 load steps, sharing one
50k-triangle branching lumen.  One bench step = the whole quasi-static
insertion (all load steps) of the whole batch from the straight reference
state, run as one explicit schedule in which every robot advances through its
load steps on its own; inputs (state, schedule tables, lumen) are resident on
the GPU.

value = solves per second that meet the metric: a solve is one load step of one
robot that converged in mixed precision AND in plain FP64 with the mixed-precision
tip within 1e-5 of the robot length of the FP64 tip at that load step.  The raw
rate of converged mixed-precision solves is reported beside it.

Prints one JSON line.  Extra fields: per-kernel HIP-event times, the roofline of
the dominant kernel (the step's algorithmic bytes of the scope table, plus this
design's own byte model), per-load-step tip error percentiles, the FP64 oracle
timed on the host's cores on a bounded sample, and the plain FP64 single-robot
GPU path on a sample of the same robots.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "contact-FEM solves/sec, batched+mixed vs plain FP64 at 1e-5 rel tip error"
HBM_PEAK_GBS = 8000.0
TIP_TOL = 1e-5

KERNELS = ["elem_kernel", "collide_kernel", "check_rhs_kernel", "factor_kernel", "subst_kernel",
           "update_kernel", "step_solve_kernel"]
KERNEL_SOURCE = {"elem_kernel": "elem.hip", "collide_kernel": "collide.hip", "check_rhs_kernel": "solve.hip",
                 "factor_kernel": "solve.hip", "subst_kernel": "solve.hip", "update_kernel": "solve.hip",
                 "step_solve_kernel": "solve.hip"}


def launch_units(info, n_nodes):
    """Work units of one schedule, summed over robots: node-iterations of the element update
    (every pass of a load step, the final check included), free node-steps of the Newton step
    (one per Newton iteration and free node), free-node right-hand sides, those swept forward
    inside the factorisation, free-node substitution passes (Newton steps with contacts only),
    and the contact products the substitution writes."""
    free = [int(n) - 1 for n in n_nodes]
    return dict(
        elem_node_iters=sum((i["iters_total"] + i["steps_total"]) * int(n_nodes[b]) for b, i in enumerate(info)),
        free_node_steps=sum(i["iters_total"] * free[b] for b, i in enumerate(info)),
        free_node_rhs=sum(i["rhs_total"] * free[b] for b, i in enumerate(info)),
        free_node_rhs_fused=sum(i["rhs_fused"] * free[b] for b, i in enumerate(info)),
        free_node_passes=sum(i["sweep_passes"] * free[b] for b, i in enumerate(info)),
        contact_products=sum(i["products_total"] for i in info),
        free_node_steps_with_contacts=sum(i["contact_steps_total"] * free[b] for b, i in enumerate(info)),
        # a Newton step without contacts has the one right-hand side b, swept in the factorisation
        free_node_rhs_with_contacts=sum((i["rhs_total"] - i["iters_total"] + i["contact_steps_total"]) * free[b]
                                        for b, i in enumerate(info)),
        free_node_rhs_fused_with_contacts=sum((i["rhs_fused"] - i["iters_total"] + i["contact_steps_total"])
                                              * free[b] for b, i in enumerate(info)),
    )


def byte_models(u, sb):
    """Algorithmic HBM bytes per schedule of the kernels with a per-node byte count.

    "scope": the minimum of the step itself (the hot-path scope table): the element update
    reads the node state (7 FP64) and writes its out-of-balance force (6 FP64) and tangent
    blocks D (21) and S (36) in the element precision, 560 B (FP64) / 280 B (FP32) per node;
    the block Cholesky reads and writes the 57 unique block values per free node (912 B);
    the multi-right-hand-side solve reads L twice per free node, shared by all right-hand
    sides of the step (912 B); so does the step's own solve after the LCP; the contact LCP
    (the update kernels) reads the contact products once, W and q (8 B per product).
    "design": what this design's kernels must move: the element update writes the chord
    direction (3 x sb) instead of D and S; the factorisation reads the element (3 x sb + 6
    FP64 constants) and column 0's right-hand side and writes L[i,i] and the coupling block,
    plus a checkpoint of 6 FP64 forward values per 6 nodes (8 B per node) for each of the first
    64 right-hand sides; the substitution stages L[i,i] and 7/6 coupling blocks per node and
    pass of 64 right-hand sides (624 B), reads column 0's right-hand side once per step (48 B),
    reads the checkpoints of every right-hand side (8 B per node), sweeps the right-hand sides
    beyond the first 64 forward (L[i,i] and the coupling block, 576 B per node and pass, and
    8 B of checkpoints per node and right-hand side) and writes 8 B per contact product (an
    upper bound: the backward sweeps stop at the outermost contact nodes).
    Returns {kernel: {"scope": (bytes_per_unit, unit, total), "design": (...)}}."""
    el_scope = 8 * (7 + 6) + (21 + 36) * (8 if sb == 8 else 4)
    el_design = 8 * (7 + 6) + 3 * sb
    fa_design = 3 * sb + 8 * 6 + 8 * (21 + 36) + 8 * 6
    extra_passes = u["free_node_passes"] - u["free_node_steps_with_contacts"]   # beyond the first
    return {
        "elem_kernel": {"scope": (el_scope, "node-iteration", el_scope * u["elem_node_iters"]),
                        "design": (el_design, "node-iteration", el_design * u["elem_node_iters"])},
        "factor_kernel": {"scope": (912, "free node-step", 912 * u["free_node_steps"]),
                          "design": ([fa_design, 8], "free node-step, fused rhs",
                                     fa_design * u["free_node_steps"] + 8 * u["free_node_rhs_fused"])},
        "subst_kernel": {"scope": (912, "free node-step", 912 * u["free_node_steps"]),
                         "design": ([624, 48, 8, 576, 8, 8],
                                    "free node-pass, node-step with contacts, node-rhs, node-pass "
                                    "beyond the first, node-rhs beyond 64, contact product",
                                    624 * u["free_node_passes"] + 48 * u["free_node_steps_with_contacts"]
                                    + 8 * u["free_node_rhs_with_contacts"] + 576 * extra_passes
                                    + 8 * (u["free_node_rhs_with_contacts"] - u["free_node_rhs_fused_with_contacts"])
                                    + 8 * u["contact_products"])},
        # W and q read once; the active-set iterations re-read columns of W from L2
        "update_kernel": {"scope": (8, "contact product", 8 * u["contact_products"]),
                          "design": (8, "contact product", 8 * u["contact_products"])},
        # forward and backward: the coupling block and the rows of L[i,i] (288 B each, whole
        # cache lines), the vector read and written (48 B each), per free node-step
        "step_solve_kernel": {"scope": (912, "free node-step", 912 * u["free_node_steps"]),
                              "design": (1344, "free node-step", 1344 * u["free_node_steps"])},
    }


def traffic_key(kernel, capacity):
    """What the counters of `kernel` depend on: its source, every device header and the
    contact capacity of the run (hashed together)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_06922_amd", "csrc")
    for path in [os.path.join(csrc, KERNEL_SOURCE[kernel])] + sorted(glob.glob(os.path.join(csrc, "*.h"))):
        with open(path, "rb") as f:
            h.update(f.read())
    h.update(b"capacity=%d" % capacity)
    return h.hexdigest()


def measured_traffic(kernel, capacity):
    """Per-launch HBM bytes of `kernel` from the committed rocprofv3 counter summary, if the
    kernel's source, the device header and the contact capacity are those the counters were
    taken with (else None)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel)
    if not rec or traffic_key(kernel, capacity) != rec.get("key_sha256"):
        return None
    return rec.get("bytes_per_launch")


def make_context(fem, rb, prec, args, V, T, **kw):
    """A context of the batch with inputs and outputs on the device; the launch shapes of the
    element update and detection are autotuned at its first solve."""
    import torch
    kw.setdefault("autotune", 1)
    ctx = fem.Context(fem.params_from_batch(rb, precision=prec, newton_tol=1e-10, stag_tol=1e-9,
                                            max_newton=args.max_newton,
                                            contact_capacity=args.capacity, io_on_device=1, **kw))
    ctx.fem_set_lumen(torch.tensor(V, device="cuda"), torch.tensor(T, dtype=torch.int32, device="cuda"))
    return ctx


def run_schedule(ctx, X0, vals, deps, records=False):
    """One insertion of the batch from X0: one explicit schedule, every robot on its own."""
    ctx.fem_set_state(X0)
    return ctx.fem_solve_schedule(0, vals, deps, state=False, info=True, records=records)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_worker(job):
    """One load step of one robot of the batched workload, re-solved by the FP64 oracle from the
    oracle's own converged state after the previous load step (stored with the oracle's
    trajectories under tests/golden/bench_oracle); a process of its own, one BLAS thread."""
    path, q = job
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import solver, collision
    from workloads import make_config, load_schedule
    from paper_2503_06922_amd.fem import state_to_PR
    with np.load(path) as z:
        b = int(z["robot"])
        k = int(z["restart_after"][q]) + 1
        X = z["restart_state"][q]
    rb, V, T = make_config(3)
    sub = rb.subset([b])
    rob = solver.robots_from_batch(sub, collision.Mesh(V, T))[0]
    d, t = load_schedule(sub, k)
    P, R = state_to_PR(X)
    t0 = time.perf_counter()
    _, _, _, _, info = solver.solve_load_step(rob, P, R, rob.base_target(d[0]), 0, t[0], tol=1e-10,
                                              stag_tol=1e-9, max_iter=60, guided=rob.guided(d[0]))
    return int(info["status"] == solver.OK), time.perf_counter() - t0, info["iters"]


def cpu_baseline(workers, total_solves_gpu):
    """The FP64 oracle on the host cores, on a bounded sample of the batched workload spread
    over its schedule: sixteen seeded robots (four per quarter of the element-count range), each
    re-solving load steps 25, 50, 75 and 100 from the oracle's own state after the previous load
    step, at the benchmark's tolerances; one process per solve in a pool of `workers`."""
    import glob
    import multiprocessing as mp
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "golden", "bench_oracle", "robot_*.npz")))
    if not files:
        return None
    jobs = [(f, q) for f in files for q in range(4)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_cpu_worker, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    conv = sum(r[0] for r in res)
    rate = conv / wall
    return dict(value=rate, unit="solves/s", cores=workers, kind="oracle", cpu=cpu_model(),
                sample=f"{len(files)} seeded robots of the batched workload (4 per quarter of the "
                       f"element-count range) x load steps 25, 50, 75, 100, each re-solved from "
                       f"the oracle's own state after the previous load step, one process per "
                       f"solve on {workers} cores: {conv} of {len(jobs)} converged in {wall:.1f} s "
                       f"wall ({sum(r[1] for r in res):.0f} s CPU, "
                       f"{sum(r[2] for r in res) / len(res):.1f} Newton iterations per solve)",
                extrapolated_batch_s=total_solves_gpu / rate if rate > 0 else None,
                extrapolation="time the oracle would take for the batch's converged solves at "
                              "the sample's rate (extrapolated, not measured)")


def config2(args):
    """The 1000-element robot inserted into the 200k-triangle lumen over 100 load steps, in
    mixed precision and in FP64: solves/s, converged load steps, Newton iterations and the
    mixed path's relative tip error against the FP64 one per load step."""
    from paper_2503_06922_amd import fem
    from workloads import make_config, schedule_table
    rb, V, T = make_config(2)
    out = {"workload": "1 robot x %d load steps, %d elements, %dk-triangle branching lumen"
                       % (rb.n_load_steps, int(rb.n_elem[0]), round(T.shape[0] / 1000))}
    vals, deps = schedule_table(rb)
    rec = {}
    for name, prec in (("mixed", fem.FEM_MIXED), ("fp64", fem.FEM_FP64)):
        ctx = fem.Context(fem.params_from_batch(rb, precision=prec, newton_tol=1e-10, stag_tol=1e-9,
                                                max_newton=args.max_newton,
                                                contact_capacity=args.capacity))
        ctx.fem_set_lumen(V, T)
        t0 = time.perf_counter()
        o = ctx.fem_solve_schedule(0, vals, deps, state=False, info=True, records=True)
        t_solve = time.perf_counter() - t0
        i = o["info"][0]
        ctx.close()
        rec[name] = o
        out[name] = {"solves_per_s": i["steps_converged"] / t_solve, "converged": i["steps_converged"],
                     "load_steps": i["steps_total"],
                     "newton_iters_per_solve": i["iters_total"] / max(i["steps_total"], 1)}
    ok = (rec["mixed"]["rec_status"][:, 0] == 0) & (rec["fp64"]["rec_status"][:, 0] == 0)
    e = np.linalg.norm(rec["mixed"]["rec_tip"][:, 0] - rec["fp64"]["rec_tip"][:, 0], axis=1) / rb.length[0]
    out["tip_err_mixed_vs_fp64"] = {"max": float(e[ok].max()) if ok.any() else None,
                                    "median": float(np.median(e[ok])) if ok.any() else None,
                                    "load_steps_compared": int(ok.sum())}
    return out


PHASES = ["element", "detection", "convergence+rhs", "factorisation", "substitution", "lcp", "step"]


def contact_sweep(args, n_nodes=(100, 200, 300, 400), per_size=2):
    """Time per Newton iteration against the number of active contacts, per phase, for single
    robots of 100/200/300/400 nodes (the speed claim of Sec. IV-A: how the cost of the
    element update, the factorisation and the contact solve grows with the contact count).

    Each robot (L = 0.6 m, shaft + tube tip, tensions and base frame of a robot of the
    batched workload, inserted 0.5 m over 100 load steps into the 50k-triangle lumen) runs in
    a context of its own in plain FP64 with HIP events around every kernel class; per load
    step the phase times divided by its Newton iterations give the time per iteration, binned
    by the active contacts (force > 0) at the end of that load step."""
    from paper_2503_06922_amd import fem
    from workloads import make_config, schedule_table
    rb3, V, T = make_config(3)
    edges = [0, 1, 6, 11, 21, 31, 41, 61, 10 ** 9]
    out = {"unit": "ms per Newton iteration", "phases": PHASES, "bins_active_contacts": edges[:-1],
           "sizes": {}}
    for nn in n_nodes:
        rows = []
        for j in range(per_size):
            sub = rb3.subset([j])
            sub.n_elem = np.array([nn - 1], np.int32)
            sub.depth = np.array([0.5])
            vals, deps = schedule_table(sub, 100)
            ctx = fem.Context(fem.params_from_batch(sub, precision=fem.FEM_FP64, newton_tol=1e-10,
                                                    stag_tol=1e-9, max_newton=args.max_newton,
                                                    contact_capacity=args.capacity, profile=1))
            ctx.fem_set_lumen(V, T)
            for k in range(len(KERNELS)):
                ctx.fem_profile(k, reset=True)
            for k in range(100):
                ctx.fem_set_actuation(0, vals[k].ravel(), deps[k])
                o = ctx.fem_solve(1, state=False)
                it = o["info"][0]["iters"]
                ms = [ctx.fem_profile(c, reset=True)[0] for c in range(len(KERNELS))]
                n_act = sum(1 for c in ctx.fem_contacts(0) if c["force"] > 0)
                if it > 0 and o["info"][0]["status"] == 0:
                    # element update, detection and convergence test run once more than the
                    # Newton steps (the final check of the load step)
                    rows.append((n_act, [m / (it + 1) for m in ms[:3]] + [m / it for m in ms[3:]]))
            ctx.close()
        bins = []
        for lo, hi in zip(edges[:-1], edges[1:]):
            sel = [r[1] for r in rows if lo <= r[0] < hi]
            if sel:
                bins.append([lo, len(sel)] + [float("%.4g" % v) for v in np.mean(sel, axis=0)])
        out["sizes"][str(nn)] = bins
    out["columns"] = ["active_contacts_from", "load_steps"] + PHASES
    return out


def element_variant(fem, rb, args, V, T, X0, vals, deps):
    """The same batched insertion (mixed precision) with contacts along elements as well
    (contact_along_elements = 1, eq. 3-7 at 0 < xi < l0): one timed schedule; converged
    solves per second, the converged fraction, Newton iterations per solve and the active
    element contacts at the end of the insertion."""
    import torch
    ce = make_context(fem, rb, fem.FEM_MIXED, args, V, T, contact_along_elements=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    oe = run_schedule(ce, X0, vals, deps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = oe["info"]
    conv = sum(i["steps_converged"] for i in info)
    total = sum(i["steps_total"] for i in info)
    iters = sum(i["iters_total"] for i in info)
    act = [c for c in ce.fem_contacts(-1) if c["kind"] == 2 and c["force"] > 0]
    ce.close()
    return {"ms_per_step": 1e3 * dt, "solves_converged_per_s": conv / dt,
            "converged_fraction": conv / max(total, 1), "newton_iters_per_solve": iters / max(total, 1),
            "active_element_contacts_at_end": len(act),
            "robots_with_active_element_contact_at_end": len({c["robot"] for c in act})}


def qp_variants(args):
    """The linear step's QP solved exactly (Schur complement + LCP) and by the paper's OSQP
    iteration (qp_solver = FEM_QP_ADMM, rho = 1 N/m, tolerance 1e-11) at the same Newton
    tolerance (1e-10 N): the straight-tube robot through its 20-step tension ramp and two
    robots of the batched workload through their first 12 load steps; time per Newton
    iteration (single-robot contexts are latency-bound), Newton and ADMM iteration counts."""
    from paper_2503_06922_amd import fem
    from workloads import make_config, load_schedule
    out = {}
    for name, cfg, pick, n_steps in (("straight tube, 20 elements", 0, None, 20),
                                     ("batched workload robots 527 and 2767", 3, [527, 2767], 12)):
        rb, V, T = make_config(cfg)
        if pick is not None:
            rb = rb.subset(pick)
        row = {}
        for qp, label in ((fem.FEM_QP_EXACT, "exact"), (fem.FEM_QP_ADMM, "admm")):
            ctx = fem.Context(fem.params_from_batch(rb, newton_tol=1e-10, stag_tol=1e-9, max_newton=100,
                                                    contact_capacity=args.capacity, qp_solver=qp,
                                                    admm_rho=1.0, admm_eps=1e-11))
            ctx.fem_set_lumen(V, T)
            t_tot = 0.0
            for k in range(1, n_steps + 1):
                d, t = load_schedule(rb, k)
                ctx.fem_set_actuation(0, t.ravel(), d)
                t0 = time.perf_counter()
                o = ctx.fem_solve(1, state=False)
                t_tot += time.perf_counter() - t0
            it = sum(i["iters_total"] for i in o["info"])
            row[label] = {"ms_per_newton_iter": 1e3 * t_tot / max(it, 1), "newton_iters": it,
                          "converged": sum(i["steps_converged"] for i in o["info"]),
                          "admm_iters": sum(i["qp_iters_total"] for i in o["info"])}
            ctx.close()
        row["admm_slowdown"] = row["admm"]["ms_per_newton_iter"] / row["exact"]["ms_per_newton_iter"]
        out[name] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--robots", type=int, default=4096)
    ap.add_argument("--load-steps", type=int, default=100)
    ap.add_argument("--max-newton", type=int, default=60)
    ap.add_argument("--capacity", type=int, default=512)
    ap.add_argument("--cpu-workers", type=int, default=0, help="0 = the host's cores, at most 16")
    ap.add_argument("--single-robots", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 reference schedule (value then counts every converged solve)")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel timing schedule")
    ap.add_argument("--no-config2", action="store_true",
                    help="skip the 1000-element robot on the 200k-triangle lumen")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the time-per-iteration against contact count sweep")
    ap.add_argument("--no-qp-variants", action="store_true",
                    help="skip the exact vs ADMM linear-step comparison")
    ap.add_argument("--no-elements", action="store_true",
                    help="skip the batched insertion with contacts along elements")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (robots are "
              "independent: a multi-GPU run would shard the batch, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_06922_amd import fem
    from workloads import make_config, schedule_table

    torch.cuda.init()
    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    rb_all, V, T = make_config(3)
    rb = rb_all.subset(np.arange(args.robots)) if args.robots < rb_all.n_robots else rb_all
    nls = args.load_steps
    vals_h, deps_h = schedule_table(rb, nls)
    vals = torch.tensor(vals_h, device="cuda")
    deps = torch.tensor(deps_h, device="cuda")

    ctx = make_context(fem, rb, fem.FEM_MIXED, args, V, T)
    X0 = ctx.fem_get_state()
    for _ in range(args.warmup):
        run_schedule(ctx, X0, vals, deps)
        print("bench: warmup schedule done", file=sys.stderr, flush=True)
    # timed region: whole-batch insertions; each call returns after its stream synchronises
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        out = run_schedule(ctx, X0, vals, deps, records=(s == args.steps - 1))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"bench: timed schedules done ({dt:.1f} s)", file=sys.stderr, flush=True)
    tb, tl, tt = ctx.fem_tuning()
    launch_shapes = {"elem_threads_per_block": tb, "detect_lanes_per_node": tl,
                     "tuning_us": {"elem_64_128_256": [round(float(v), 1) for v in tt[:3]],
                                   "detect_4_8_16": [round(float(v), 1) for v in tt[3:]]}}
    info = out["info"]                      # counters of the last schedule (fem_set_state resets)
    conv = sum(i["steps_converged"] for i in info)
    total = sum(i["steps_total"] for i in info)
    iters = sum(i["iters_total"] for i in info)
    st_m = out["rec_status"].cpu().numpy()
    tip_m = out["rec_tip"].cpu().numpy()

    it_m = out["rec_iters"].cpu().numpy()
    conv_it = it_m[st_m == 0]
    status_counts = {name: int(np.sum(st_m == k)) for k, name in
                     enumerate(("ok", "noconv", "lcpfail", "nonspd", "overflow"))}
    iters_hist = {"bins": [0, 5, 10, 15, 20, 30, 40, 50, 60],
                  "converged_solves": np.histogram(conv_it, bins=[0, 5, 10, 15, 20, 30, 40, 50, 60,
                                                                  10 ** 6])[0].tolist()}
    tip_err = None
    fp64 = {}
    if args.no_fp64:
        value = conv * args.steps / dt
    else:
        # the same schedule in plain FP64 (batched): throughput and the per-step reference tips
        c64 = make_context(fem, rb, fem.FEM_FP64, args, V, T)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        o64 = run_schedule(c64, X0, vals, deps, records=True)
        t64 = time.perf_counter() - t1
        print(f"bench: FP64 schedule done ({t64:.1f} s)", file=sys.stderr, flush=True)
        conv64 = sum(i["steps_converged"] for i in o64["info"])
        st_64 = o64["rec_status"].cpu().numpy()
        tip_64 = o64["rec_tip"].cpu().numpy()
        c64.close()
        err = np.linalg.norm(tip_m - tip_64, axis=2) / rb.length[None, :]      # [steps, robots]
        both = (st_m == 0) & (st_64 == 0)
        valid = both & (err <= TIP_TOL)
        value = int(valid.sum()) * args.steps / dt
        p50, p99, pmax = [], [], []
        for k in range(nls):
            e = err[k][both[k]]
            p50.append(float(np.median(e)) if e.size else None)
            p99.append(float(np.percentile(e, 99)) if e.size else None)
            pmax.append(float(e.max()) if e.size else None)
        apart = np.any(both & (err > TIP_TOL), axis=0)
        first_apart = [int(np.argmax(both[:, b] & (err[:, b] > TIP_TOL))) + 1 for b in np.nonzero(apart)[0]]
        tip_err = {
            "per_step_p50": [float("%.2g" % v) if v is not None else None for v in p50],
            "per_step_p99": [float("%.2g" % v) if v is not None else None for v in p99],
            "per_step_max": [float("%.2g" % v) if v is not None else None for v in pmax],
            "solves_compared": int(both.sum()), "solves_within_1e-5": int(valid.sum()),
            "robots_ever_apart": int(apart.sum()),
            "first_step_apart_quartiles": (np.percentile(first_apart, [25, 50, 75]).tolist()
                                           if first_apart else None),
        }
        fp64 = {"fp64_batched_solves_per_s": conv64 / t64,
                "mixed_vs_fp64_batched": (conv * args.steps / dt) / (conv64 / t64)}

    res = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 + f32 (f32 element forces far from convergence, f32 tangent storage and "
                 "detection screen)",
        "data": "synthetic",
        "config": {"workload": "batched insertion: %d robots x %d load steps, 50-400 elements "
                               "(Table I shaft + 70 mm tube tip), moment-only cable load (eq. 16), "
                               "rigid insertion guide, 50k-triangle branching lumen, mixed "
                               "precision" % (rb.n_robots, nls),
                   "robots": int(rb.n_robots), "load_steps": nls, "precision": "mixed",
                   "max_newton": args.max_newton, "contact_capacity": args.capacity,
                   "nodes": int(ctx.n_nodes)},
        "value_basis": ("converged mixed-precision solves (no FP64 reference run)" if args.no_fp64 else
                        "converged mixed-precision solves whose tip is within 1e-5 of the robot "
                        "length of the FP64 batch's tip at that load step (both converged)"),
        "solves_converged_per_s": conv * args.steps / dt,
        "converged_fraction": conv / max(total, 1),
        "newton_iters_per_solve": iters / max(total, 1),
        "newton_iters_histogram": iters_hist,
        "load_step_status": status_counts,
        "launch_shapes": launch_shapes,
        **fp64,
        "tip_err_mixed_vs_fp64": tip_err,
    }

    if not args.no_profile:
        # kernel times: one more schedule on a context that brackets every kernel class with
        # HIP events on its stream (outside the timed region: it synchronises every pass)
        cp = make_context(fem, rb, fem.FEM_MIXED, args, V, T, profile=1)
        op = run_schedule(cp, X0, vals, deps)
        print("bench: profiled schedule done", file=sys.stderr, flush=True)
        prof = [cp.fem_profile(k) for k in range(len(KERNELS))]
        cp.close()
        kern = {KERNELS[k]: dict(total_ms=prof[k][0], launches=prof[k][1],
                                 avg_us=1e3 * prof[k][0] / max(prof[k][1], 1)) for k in range(len(KERNELS))}
        dom = KERNELS[max(range(len(KERNELS)), key=lambda k: prof[k][0])]
        n_nodes = np.asarray(rb.n_elem, np.int64) + 1
        units = launch_units(op["info"], n_nodes)
        models = byte_models(units, 4)
        roofs = {}
        for name, m in models.items():
            k = KERNELS.index(name)
            launches = max(prof[k][1], 1)
            avg_s = prof[k][0] / 1e3 / launches
            r = {"bound": "hbm", "kernel": name, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                 "avg_launch_us": avg_s * 1e6, "launches": launches,
                 "traffic": measured_traffic(name, args.capacity)}
            for key in ("scope", "design"):
                per, unit, tot = m[key]
                gbs = tot / launches / avg_s / 1e9
                r[key] = dict(bytes_per_unit=per, unit_name=unit, bytes_per_launch=tot / launches,
                              achieved=gbs, frac=gbs / HBM_PEAK_GBS)
            r["achieved"] = r["scope"]["achieved"]
            r["frac"] = r["scope"]["frac"]
            roofs[name] = r
        res["units_per_schedule"] = units
        res["kernels"] = kern
        res["dominant_kernel"] = dom
        roof = roofs.get(dom) or max(roofs.values(), key=lambda r: r["avg_launch_us"])
        res["roofline"] = roof
        res["rooflines"] = roofs
    if not args.no_single:
        # plain FP64 path of configuration 0: one robot per context, run one after another
        t_single, conv_single = 0.0, 0
        for b in range(args.single_robots):
            sub = rb.subset([b])
            v1, d1 = schedule_table(sub, nls)
            c1 = fem.Context(fem.params_from_batch(sub, precision=fem.FEM_FP64, newton_tol=1e-10,
                                                   stag_tol=1e-9, max_newton=args.max_newton,
                                                   contact_capacity=args.capacity))
            c1.fem_set_lumen(V, T)
            t1 = time.perf_counter()
            o1 = c1.fem_solve_schedule(0, v1, d1, state=False, info=True, records=False)
            t_single += time.perf_counter() - t1
            conv_single += o1["info"][0]["steps_converged"]
            c1.close()
        res["fp64_single_solves_per_s"] = conv_single / t_single
        res["ratio_vs_fp64_single"] = value / res["fp64_single_solves_per_s"]
    ctx.close()
    if not args.no_config2:
        res["config2"] = config2(args)
        print("bench: 1000-element robot done", file=sys.stderr, flush=True)
    if not args.no_sweep:
        res["contact_sweep"] = contact_sweep(args)
        print("bench: contact sweep done", file=sys.stderr, flush=True)
    if not args.no_elements:
        res["element_contacts"] = element_variant(fem, rb, args, V, T, X0, vals, deps)
        print("bench: element-contact schedule done", file=sys.stderr, flush=True)
    if not args.no_qp_variants:
        res["qp_variants"] = qp_variants(args)
        print("bench: QP variants done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        res["cpu_baseline"] = cpu_baseline(workers, conv)
        print("bench: oracle sample done", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
