"""Benchmark: batched contact-FEM solves per second on one MI355X.

Workload (the batched configuration): 4096 robots with 50..400 elements
(L = 0.6 m, stiff shaft + 70 mm tube tip), tensions U(0,3) N ramped over 10
load steps and insertion depths U(0.1,0.5) m over 100 load steps, sharing one
50k-triangle branching lumen.  One bench step = the whole quasi-static
insertion (all load steps) of the whole batch from the straight reference
state, inputs resident on the GPU.  A solve = one converged load step of one
robot; value = converged solves / wall time of the timed steps.

Prints one JSON line (see --help).  Extra fields: per-kernel HIP-event times,
the roofline of the dominant kernel, the FP64 oracle timed on the host on a
bounded sample, and the plain FP64 single-robot GPU path on a sample of the
same robots (the configuration-0 design run one robot at a time).
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


KERNELS = ["elem_kernel", "collide_kernel", "check_rhs_kernel", "factor_kernel", "subst_kernel",
           "update_kernel"]
KERNEL_SOURCE = {"elem_kernel": "elem.hip", "collide_kernel": "collide.hip", "check_rhs_kernel": "solve.hip",
                 "factor_kernel": "solve.hip", "subst_kernel": "solve.hip", "update_kernel": "solve.hip"}


def algorithmic_bytes(info, n_nodes, sb, steps):
    """HBM bytes the kernels with a fixed per-node byte count must move over one schedule.

    sb = bytes of a stored chord-direction component (4 in mixed precision, 8 in FP64).
      elem_kernel   per active node: read the state (7 FP64), write F (6 FP64) and the chord
                    direction of its element (3 x sb)
      factor_kernel per free node and Newton step: read the node's two elements (direction
                    3 x sb and 6 FP64 constants each; the left one is shared with the previous
                    node, so one element per node), write the Cholesky blocks L[i,i] (21 unique
                    FP64) and L[i+1,i] (36 FP64) and read column 0's right-hand side (6 FP64);
                    its second wavefront sweeps the first 64 right-hand sides forward (the
                    contact columns are generated, not read): write y, 6 FP64 per node and
                    right-hand side
      subst_kernel  per free node and pass of 64 right-hand sides: read L[i,i] and L[i+1,i]
                    (57 FP64); per right-hand side read y and write x (2 x 6 FP64); those
                    beyond the first 64 are also swept forward here (write y, 6 FP64)
    Returns {kernel: (bytes per unit, total bytes)}.
    """
    per = {"elem_kernel": 8 * (7 + 6) + 3 * sb,
           "factor_kernel": (3 * sb + 8 * 6 + 8 * (21 + 36) + 8 * 6, 8 * 6),
           "subst_kernel": (8 * 57, 2 * 8 * 6, 8 * 6)}
    elem_nodes = sum((i["iters_total"] + i["steps_total"]) * int(n_nodes[b]) for b, i in enumerate(info))
    free = [int(n) - 1 for n in n_nodes]
    free_steps = sum(i["iters_total"] * free[b] for b, i in enumerate(info))
    free_rhs = sum(i["rhs_total"] * free[b] for b, i in enumerate(info))
    free_fused = sum(i["rhs_fused"] * free[b] for b, i in enumerate(info))
    free_passes = sum(i["sweep_passes"] * free[b] for b, i in enumerate(info))
    return {
        "elem_kernel": (per["elem_kernel"], per["elem_kernel"] * elem_nodes * steps),
        "factor_kernel": (per["factor_kernel"], (per["factor_kernel"][0] * free_steps
                                                + per["factor_kernel"][1] * free_fused) * steps),
        "subst_kernel": (per["subst_kernel"], (per["subst_kernel"][0] * free_passes
                                              + per["subst_kernel"][1] * free_rhs
                                              + per["subst_kernel"][2] * (free_rhs - free_fused)) * steps),
    }


def traffic_key(kernel, capacity):
    """What the counters of `kernel` depend on: its source, the shared device header and the
    contact capacity of the run (hashed together)."""
    import hashlib
    h = hashlib.sha256()
    for name in (KERNEL_SOURCE[kernel], "fem_device.h"):
        with open(os.path.join(ROOT, "paper_2503_06922_amd", "csrc", name), "rb") as f:
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


def run_schedule(ctx, rb, n_load_steps, X0):
    from workloads import load_schedule
    ctx.fem_set_state(X0)
    for k in range(1, n_load_steps + 1):
        d, t = load_schedule(rb, k)
        ctx.fem_set_actuation(0, t.ravel(), d)
        ctx.fem_solve(1, state=False, info=False)


def solves_of(ctx):
    out = ctx.fem_solve(0, state=False, info=True)
    info = out["info"]
    return (sum(i["steps_converged"] for i in info), sum(i["steps_total"] for i in info),
            sum(i["iters_total"] for i in info), info)


def config2(max_newton, capacity):
    """The 1000-element robot inserted into the 200k-triangle lumen over 100 load steps, in
    mixed precision and in FP64 (one context each): solves/s, converged load steps, Newton
    iterations and the mixed path's relative tip error against the FP64 one per load step."""
    from paper_2503_06922_amd import fem
    from workloads import make_config, load_schedule
    rb, V, T = make_config(2)
    out = {"workload": "1 robot x %d load steps, %d elements, %dk-triangle branching lumen"
                       % (rb.n_load_steps, int(rb.n_elem[0]), round(T.shape[0] / 1000))}
    tips = {}
    for name, prec in (("mixed", fem.FEM_MIXED), ("fp64", fem.FEM_FP64)):
        ctx = fem.Context(fem.params_from_batch(rb, precision=prec, newton_tol=1e-10, stag_tol=1e-9,
                                                max_newton=max_newton, contact_capacity=capacity))
        ctx.fem_set_lumen(V, T)
        ctx.fem_set_actuation(0, np.zeros(3), np.zeros(1))
        tip, t_solve = [], 0.0
        for k in range(1, rb.n_load_steps + 1):
            d, t = load_schedule(rb, k)
            ctx.fem_set_actuation(0, t.ravel(), d)
            t0 = time.perf_counter()
            o = ctx.fem_solve(1, state=True, info=True)
            t_solve += time.perf_counter() - t0
            tip.append((o["state"][-1, 0:3].copy(), o["info"][0]["status"]))
        conv, total, iters, _ = solves_of(ctx)
        ctx.close()
        tips[name] = tip
        out[name] = {"solves_per_s": conv / t_solve, "converged": conv, "load_steps": total,
                     "newton_iters_per_solve": iters / max(total, 1)}
    e = [np.linalg.norm(a[0] - b[0]) / rb.length[0]
         for a, b in zip(tips["mixed"], tips["fp64"]) if a[1] == 0 and b[1] == 0]
    out["tip_err_mixed_vs_fp64"] = {"max": float(max(e)) if e else None,
                                    "median": float(np.median(e)) if e else None,
                                    "load_steps_compared": len(e)}
    return out


def cpu_baseline(rb, V, T, n_robots, n_steps):
    """The FP64 oracle on a bounded sample: n_robots robots x n_steps load steps."""
    from oracle import solver, collision
    from workloads import load_schedule
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:
        lim = None
    mesh = collision.Mesh(V, T)
    sub = rb.subset(np.arange(n_robots))
    robs = solver.robots_from_batch(sub, mesh)
    t0 = time.perf_counter()
    conv = 0
    for b, rob in enumerate(robs):
        sched = lambda k, b=b: (lambda d, t: (d[b], t[b]))(*load_schedule(sub, k))
        _, _, traj = solver.solve_robot(rob, sched, n_steps, tol=1e-10, stag_tol=1e-9, max_iter=100)
        conv += sum(1 for s in traj if s["info"]["status"] == solver.OK)
    dt = time.perf_counter() - t0
    return dict(value=conv / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"{n_robots} robots x {n_steps} load steps of the batched workload "
                       f"({conv} converged solves in {dt:.1f} s, 1 BLAS thread)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--robots", type=int, default=4096)
    ap.add_argument("--load-steps", type=int, default=100)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--max-newton", type=int, default=60)
    ap.add_argument("--capacity", type=int, default=512)
    ap.add_argument("--cpu-robots", type=int, default=2)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--single-robots", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-config2", action="store_true",
                    help="skip the 1000-element robot on the 200k-triangle lumen")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (robots are "
              "independent: a multi-GPU run would shard the batch, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    from paper_2503_06922_amd import fem
    from workloads import make_config

    import torch
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
    prec = fem.FEM_MIXED if args.precision == "mixed" else fem.FEM_FP64
    ctx = fem.Context(fem.params_from_batch(rb, precision=prec, newton_tol=1e-10, stag_tol=1e-9,
                                            max_newton=args.max_newton,
                                            contact_capacity=args.capacity))
    ctx.fem_set_lumen(V, T)
    ctx.fem_set_actuation(0, np.zeros(3 * rb.n_robots), np.zeros(rb.n_robots))
    X0 = ctx.fem_get_state()

    for _ in range(args.warmup):
        run_schedule(ctx, rb, args.load_steps, X0)
        print("bench: warmup schedule done", file=sys.stderr, flush=True)
    # timed region: whole-batch insertions; each fem_solve returns after its stream synchronises
    ctx.fem_set_state(X0)  # resets the per-robot counters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_schedule(ctx, rb, args.load_steps, X0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"bench: timed schedules done ({dt:.1f} s)", file=sys.stderr, flush=True)
    # counters cover the last schedule only (fem_set_state resets them): scale to all steps
    conv, total, iters, info = solves_of(ctx)
    solves = conv * args.steps
    value = solves / dt

    # kernel times: one more schedule on a context that brackets every launch with HIP events
    # on its stream (outside the timed region: the event synchronisation slows the loop)
    cp = fem.Context(fem.params_from_batch(rb, precision=prec, newton_tol=1e-10, stag_tol=1e-9,
                                           max_newton=args.max_newton,
                                           contact_capacity=args.capacity, profile=1))
    cp.fem_set_lumen(V, T)
    cp.fem_set_actuation(0, np.zeros(3 * rb.n_robots), np.zeros(rb.n_robots))
    run_schedule(cp, rb, args.load_steps, X0)
    print("bench: profiled schedule done", file=sys.stderr, flush=True)
    prof = [cp.fem_profile(k) for k in range(6)]
    _, _, _, info_p = solves_of(cp)
    cp.close()
    kern = {KERNELS[k]: dict(total_ms=prof[k][0], launches=prof[k][1],
                             avg_us=1e3 * prof[k][0] / max(prof[k][1], 1)) for k in range(6)}
    dom = KERNELS[max(range(6), key=lambda k: prof[k][0])]
    # rooflines: algorithmic bytes per launch / average launch time
    sb = 4 if prec == fem.FEM_MIXED else 8
    n_nodes = np.asarray(rb.n_elem, np.int64) + 1
    alg = algorithmic_bytes(info_p, n_nodes, sb, 1)
    roofs = {}
    for name, (per_unit, total_bytes) in alg.items():
        k = KERNELS.index(name)
        launches = max(prof[k][1], 1)
        avg_s = prof[k][0] / 1e3 / launches
        gbs = total_bytes / launches / avg_s / 1e9
        tr = measured_traffic(name, args.capacity)
        roofs[name] = dict(bound="hbm", kernel=name, achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                           frac=gbs / HBM_PEAK_GBS, traffic=tr, bytes_per_unit=per_unit,
                           bytes_per_launch=total_bytes / launches, avg_launch_us=avg_s * 1e6)
    roof = roofs.get(dom) or max(roofs.values(), key=lambda r: r["avg_launch_us"])

    res = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 tangent+screen / f64" if prec == fem.FEM_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": "batched insertion: %d robots x %d load steps, 50-400 elements, "
                               "50k-triangle branching lumen" % (rb.n_robots, args.load_steps),
                   "robots": int(rb.n_robots), "load_steps": args.load_steps,
                   "precision": args.precision, "max_newton": args.max_newton,
                   "contact_capacity": args.capacity,
                   "nodes": int(ctx.n_nodes)},
        "converged_fraction": conv / max(total, 1),
        "newton_iters_per_solve": iters / max(total, 1),
        "kernels": kern, "dominant_kernel": dom,
        "roofline": roof, "rooflines": roofs,
    }
    if prec == fem.FEM_MIXED and not args.no_fp64:
        # the same batch in plain FP64 (batched): throughput and the mixed path's tip error
        c64 = fem.Context(fem.params_from_batch(rb, precision=fem.FEM_FP64, newton_tol=1e-10,
                                                stag_tol=1e-9, max_newton=args.max_newton,
                                                contact_capacity=args.capacity))
        c64.fem_set_lumen(V, T)
        c64.fem_set_actuation(0, np.zeros(3 * rb.n_robots), np.zeros(rb.n_robots))
        t1 = time.perf_counter()
        run_schedule(c64, rb, args.load_steps, X0)
        t64 = time.perf_counter() - t1
        print(f"bench: FP64 schedule done ({t64:.1f} s)", file=sys.stderr, flush=True)
        conv64, _, _, info64 = solves_of(c64)
        Xm = ctx.fem_get_state()
        X64 = c64.fem_get_state()
        tips = np.asarray(rb.node_offset[1:]) - 1
        both = np.array([i["status"] == 0 and j["status"] == 0 for i, j in zip(info, info64)])
        err = np.linalg.norm(Xm[tips, 0:3] - X64[tips, 0:3], axis=1) / rb.length
        res["fp64_batched_solves_per_s"] = conv64 / t64
        e = err[both]
        res["tip_err_mixed_vs_fp64"] = {"max": float(e.max()) if both.any() else None,
                                        "median": float(np.median(e)) if both.any() else None,
                                        "p99": float(np.percentile(e, 99)) if both.any() else None,
                                        "within_1e-5": int(np.sum(e <= 1e-5)),
                                        "robots_compared": int(both.sum())}
        # robots that converged on every load step in both precisions (no diverging restart
        # from a failed load step's last iterate on either side)
        every = np.array([i["steps_converged"] == i["steps_total"] and
                          j["steps_converged"] == j["steps_total"] for i, j in zip(info, info64)])
        ea = err[every]
        res["tip_err_mixed_vs_fp64"]["every_step_converged"] = {
            "robots": int(every.sum()), "within_1e-5": int(np.sum(ea <= 1e-5)),
            "p99": float(np.percentile(ea, 99)) if every.any() else None,
            "max": float(ea.max()) if every.any() else None}
        c64.close()
    if not args.no_single:
        # plain FP64 path of configuration 0: one robot per context, run one after another
        t_single = 0.0
        conv_single = 0
        for b in range(args.single_robots):
            sub = rb.subset([b])
            c1 = fem.Context(fem.params_from_batch(sub, precision=fem.FEM_FP64, newton_tol=1e-10,
                                                   stag_tol=1e-9, max_newton=args.max_newton,
                                                   contact_capacity=args.capacity))
            c1.fem_set_lumen(V, T)
            c1.fem_set_actuation(0, np.zeros(3), np.zeros(1))
            X1 = c1.fem_get_state()
            t1 = time.perf_counter()
            run_schedule(c1, sub, args.load_steps, X1)
            t_single += time.perf_counter() - t1
            conv_single += solves_of(c1)[0]
            c1.close()
        res["fp64_single_solves_per_s"] = conv_single / t_single
        res["ratio_vs_fp64_single"] = value / res["fp64_single_solves_per_s"]
    if not args.no_config2:
        res["config2"] = config2(args.max_newton, args.capacity)
        print("bench: 1000-element robot done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(rb, V, T, args.cpu_robots, args.cpu_steps)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
