"""Write the oracle's trajectories of robots of the batched workload with contacts along
elements enabled (Sec. II-C, eq. 3-7 at 0 < xi < l0), for the GPU parity test of that option.

Calls only the oracle (oracle/) and the seeded input generators (workloads/): every stored
value is the oracle's.  Each listed robot runs its first load steps at the parity tolerance
(residual 1e-13 N, or a stagnating residual below the stagnation level; at most 100 Newton
iterations per load step), stopping after the first load step that does not converge.  Per
robot a file element_oracle/robot_<index>.npz holds per load step the status, the residual
norm at which it stopped, the node positions and the active contacts (node, triangle, kind,
s, normal, force; rows of -1 pad).

Usage: python tests/golden/make_element_oracle.py [workers]
"""
from __future__ import annotations

import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")     # one BLAS thread per worker process
import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "element_oracle")
# robots (index into the batched workload) and their load steps: element contacts become
# active on the way (found by running the oracle)
ROBOTS = {15: 40, 38: 40, 47: 40, 473: 40}
TOL, STAG, MAX_ITER = 1e-13, 1e-9, 100
MAXACT = 64


def run_robot(b):
    os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    from oracle import solver, collision
    from workloads import make_config, load_schedule
    rb, V, T = make_config(3)
    sub = rb.subset([b])
    rob = solver.robots_from_batch(sub, collision.Mesh(V, T))[0]
    rob.elements = True
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(sub, k))
    t0 = time.time()
    P, R = rob.reference()
    status, Ps, acts, res = [], [], [], []
    for k in range(1, ROBOTS[b] + 1):
        depth, vals = sched(k)
        P, R, cont, y, info = solver.solve_load_step(rob, P, R, rob.base_target(depth), 0, vals, tol=TOL,
                                                     stag_tol=STAG, max_iter=MAX_ITER, guided=rob.guided(depth))
        a = np.full((MAXACT, 8), -1.0)
        rows = [(c["node"], c["tri"], c["kind"], c.get("s", 0.0), *c["n"], yy)
                for c, yy in zip(cont, y) if yy > 0]
        a[:len(rows)] = np.array(rows, float).reshape(-1, 8)
        status.append(info["status"])
        res.append(info["res_norm"])
        Ps.append(P.copy())
        acts.append(a)
        if info["status"] != solver.OK:
            break
    os.makedirs(OUT, exist_ok=True)
    np.savez_compressed(os.path.join(OUT, f"robot_{b:04d}.npz"), robot=np.int64(b),
                        status=np.array(status, np.int32), res_norm=np.array(res), P=np.array(Ps),
                        act=np.array(acts))
    return b, time.time() - t0, len(status)


def main():
    import multiprocessing as mp
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 2
    todo = [b for b in ROBOTS if not os.path.exists(os.path.join(OUT, f"robot_{b:04d}.npz"))]
    print("robots to run", todo, flush=True)
    with mp.get_context("spawn").Pool(workers) as pool:
        for b, dt, n in pool.imap_unordered(run_robot, todo):
            print(f"robot {b}: {n} load steps, {dt:.0f} s", flush=True)


if __name__ == "__main__":
    main()
