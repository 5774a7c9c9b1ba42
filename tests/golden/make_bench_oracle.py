"""Write the oracle's trajectories of a seeded sample of the batched insertion's robots.

Calls only the oracle (oracle/) and the seeded input generators (workloads/): every stored
value is the oracle's.  Sixteen robots of the batched workload, four from each quarter of the
element-count range 50..400 (seeded choice), each run through all 100 load steps of its
insertion schedule (tensions ramped over 10, depth over 100) with the plain FP64 oracle at the
parity tolerance (residual 1e-13 N, or a stagnating residual below the stagnation level;
at most 100 Newton iterations per load step; a load step that does not converge keeps its last
iterate, as the method does).  The single robot of the realistic-size insertion (200 elements, 50k-triangle lumen) is run the
same way (bench_oracle/config1.npz).  Per robot a file bench_oracle/robot_<index>.npz holds, per load
step: status, Newton iterations, residual norm, tip position; the active contacts (node,
triangle, kind, force, normal); the nodes with near-threshold detection decisions at the
converged state (excluded from exact set comparison); the node positions at every tenth
load step; and the full node states (positions, unit quaternions) after load steps 24, 49, 74
and 99, from which a load step of the second to fourth quarter of the schedule can be re-solved.

Usage: python tests/golden/make_bench_oracle.py [workers]   (takes about an hour on 8 cores)
"""
from __future__ import annotations

import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")     # one BLAS thread per worker process
import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "bench_oracle")
N_STEPS = 100
TOL, STAG, MAX_ITER = 1e-13, 1e-9, 100
SAMPLE_EVERY = 10
RESTART_AFTER = (24, 49, 74, 99)


def mat_to_quat(R):
    """Unit quaternions (w, x, y, z) of rotation matrices [n, 3, 3] (Shepperd's method)."""
    q = np.empty((R.shape[0], 4))
    for i, M in enumerate(R):
        tr = M[0, 0] + M[1, 1] + M[2, 2]
        if tr > 0:
            s = 2.0 * np.sqrt(tr + 1.0)
            q[i] = (0.25 * s, (M[2, 1] - M[1, 2]) / s, (M[0, 2] - M[2, 0]) / s, (M[1, 0] - M[0, 1]) / s)
        elif M[0, 0] > M[1, 1] and M[0, 0] > M[2, 2]:
            s = 2.0 * np.sqrt(1.0 + M[0, 0] - M[1, 1] - M[2, 2])
            q[i] = ((M[2, 1] - M[1, 2]) / s, 0.25 * s, (M[0, 1] + M[1, 0]) / s, (M[0, 2] + M[2, 0]) / s)
        elif M[1, 1] > M[2, 2]:
            s = 2.0 * np.sqrt(1.0 + M[1, 1] - M[0, 0] - M[2, 2])
            q[i] = ((M[0, 2] - M[2, 0]) / s, (M[0, 1] + M[1, 0]) / s, 0.25 * s, (M[1, 2] + M[2, 1]) / s)
        else:
            s = 2.0 * np.sqrt(1.0 + M[2, 2] - M[0, 0] - M[1, 1])
            q[i] = ((M[1, 0] - M[0, 1]) / s, (M[0, 2] + M[2, 0]) / s, (M[1, 2] + M[2, 1]) / s, 0.25 * s)
    return q


def sample_robots():
    """Four seeded robots from each quarter of the element-count range of the batched
    workload."""
    sys.path.insert(0, ROOT)
    from workloads import make_config
    rb, _, _ = make_config(3)
    rng = np.random.default_rng([3, 11])
    picks = []
    for lo, hi in ((50, 137), (138, 225), (226, 313), (314, 400)):
        idx = np.nonzero((rb.n_elem >= lo) & (rb.n_elem <= hi))[0]
        picks += sorted(rng.choice(idx, size=4, replace=False).tolist())
    return picks


def out_name(cfg, b):
    return os.path.join(OUT, f"robot_{b:04d}.npz" if cfg == 3 else f"config{cfg}.npz")


def run_robot(job):
    cfg, b = job
    os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    from oracle import solver, collision
    from workloads import make_config, load_schedule
    rb, V, T = make_config(cfg)
    sub = rb.subset([b])
    mesh = collision.Mesh(V, T)
    rob = solver.robots_from_batch(sub, mesh)[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(sub, k))
    t0 = time.time()
    _, _, traj = solver.solve_robot(rob, sched, N_STEPS, tol=TOL, stag_tol=STAG, max_iter=MAX_ITER)
    rec = dict(robot=np.int64(b), n_elem=np.int64(rob.n_elem), tol=TOL, stag_tol=STAG,
               max_iter=np.int64(MAX_ITER))
    rec["status"] = np.array([s["info"]["status"] for s in traj], np.int32)
    rec["iters"] = np.array([s["info"]["iters"] for s in traj], np.int32)
    rec["res_norm"] = np.array([s["info"]["res_norm"] for s in traj])
    rec["tip"] = np.array([s["P"][-1] for s in traj])
    ptr, node, tri, kind, y, nrm = [0], [], [], [], [], []
    aptr, anode = [0], []
    for k, s in enumerate(traj):
        for c, yy in zip(s["contacts"], s["y"]):
            if yy > 0:
                node.append(c["node"]); tri.append(c["tri"]); kind.append(c["kind"])
                y.append(yy); nrm.append(np.asarray(c["n"], float))
        ptr.append(len(node))
        depth = sched(k + 1)[0]
        det = collision.detect(s["P"], rob.mesh, rob.r_c, rob.delta, skip=rob.guided(depth))
        amb = sorted({c["node"] for c in det if c["ambiguous"]})
        anode += amb
        aptr.append(len(anode))
    rec.update(act_ptr=np.array(ptr, np.int64), act_node=np.array(node, np.int32),
               act_tri=np.array(tri, np.int32), act_kind=np.array(kind, np.int32),
               act_y=np.array(y), act_n=np.array(nrm).reshape(-1, 3),
               amb_ptr=np.array(aptr, np.int64), amb_node=np.array(anode, np.int32))
    steps = np.arange(SAMPLE_EVERY, N_STEPS + 1, SAMPLE_EVERY)
    rec["sample_steps"] = steps.astype(np.int32)
    rec["P_sampled"] = np.stack([traj[k - 1]["P"] for k in steps])
    rec["restart_after"] = np.array(RESTART_AFTER, np.int32)
    rec["restart_state"] = np.stack([np.concatenate([traj[k - 1]["P"], mat_to_quat(traj[k - 1]["R"])],
                                                    axis=1) for k in RESTART_AFTER])
    os.makedirs(OUT, exist_ok=True)
    np.savez_compressed(out_name(cfg, b), **rec)
    return cfg, b, int(rob.n_elem), time.time() - t0, int((rec["status"] == 0).sum())


def main():
    import multiprocessing as mp
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else min(8, os.cpu_count() or 1)
    jobs = [(1, 0)] + [(3, b) for b in sample_robots()]
    todo = [j for j in jobs if not os.path.exists(out_name(*j))]
    print("jobs", jobs, "to run", todo, flush=True)
    with mp.get_context("spawn").Pool(workers) as pool:
        for cfg, b, ne, dt, conv in pool.imap_unordered(run_robot, todo):
            print(f"config {cfg} robot {b} ({ne} elements): {conv}/{N_STEPS} load steps converged, "
                  f"{dt:.0f} s", flush=True)


if __name__ == "__main__":
    main()
