"""Write the oracle's solutions and adjoint gradients for a seeded sample of the differentiation
workload (1024 robots x 300 elements inserted into the 50k-triangle lumen, loss = squared
distance of the two tip sensors to seeded targets).

Calls only the oracle (oracle/) and the seeded input generators (workloads/): every stored
value is the oracle's.  Four seeded robots, each run through all 100 load steps of its
insertion schedule at the parity tolerance (residual 1e-13 N, or a stagnating residual below
the stagnation level; at most 100 Newton iterations per load step); at the final state the
oracle's adjoint gives dL/dT for the three cable tensions.  Per robot a file
config4_oracle/robot_<index>.npz holds the per-step status and tip position, the final node
state (positions, unit quaternions), the active contacts of the final load step, the loss and
its gradient.

Usage: python tests/golden/make_config4_oracle.py [workers]
"""
from __future__ import annotations

import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")     # one BLAS thread per worker process
import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "config4_oracle")
N_STEPS = 100
TOL, STAG, MAX_ITER = 1e-13, 1e-9, 100


def sample_robots():
    return sorted(np.random.default_rng([4, 5]).choice(1024, size=4, replace=False).tolist())


def run_robot(b):
    os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    sys.path.insert(0, HERE)
    from oracle import solver, collision, adjoint
    from workloads import make_config, load_schedule, sensor_nodes, sensor_targets
    from make_bench_oracle import mat_to_quat
    rb, V, T = make_config(4)
    targets = sensor_targets(rb)[b]
    sub = rb.subset([b])
    rob = solver.robots_from_batch(sub, collision.Mesh(V, T))[0]
    sched = lambda k: (lambda d, t: (d[0], t[0]))(*load_schedule(sub, k))
    t0 = time.time()
    P, R, traj = solver.solve_robot(rob, sched, N_STEPS, tol=TOL, stag_tol=STAG, max_iter=MAX_ITER)
    last = traj[-1]
    depth, tens = sched(N_STEPS)
    n = rob.n_elem + 1
    sens = [n + int(i) for i in sensor_nodes(sub, 0)]
    loss, dLdp = adjoint.sensor_loss(P, sens, targets)
    grad = adjoint.tension_gradient(rob, P, R, last["contacts"], last["y"], tens, sens, dLdp,
                                    guided=rob.guided(depth))
    act = [(c["node"], c["tri"], c["kind"], y, *c["n"]) for c, y in zip(last["contacts"], last["y"]) if y > 0]
    rec = dict(robot=np.int64(b), status=np.array([s["info"]["status"] for s in traj], np.int32),
               tip=np.array([s["P"][-1] for s in traj]),
               state=np.concatenate([P, mat_to_quat(R)], axis=1), targets=targets,
               sensors=np.array(sens, np.int32), loss=loss, grad=np.asarray(grad, float),
               act=np.array(act, float).reshape(-1, 7))
    os.makedirs(OUT, exist_ok=True)
    np.savez_compressed(os.path.join(OUT, f"robot_{b:04d}.npz"), **rec)
    return b, time.time() - t0, int((rec["status"] == 0).sum())


def main():
    import multiprocessing as mp
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    todo = [b for b in sample_robots() if not os.path.exists(os.path.join(OUT, f"robot_{b:04d}.npz"))]
    print("robots to run", todo, flush=True)
    with mp.get_context("spawn").Pool(workers) as pool:
        for b, dt, conv in pool.imap_unordered(run_robot, todo):
            print(f"robot {b}: {conv}/{N_STEPS} load steps converged, {dt:.0f} s", flush=True)


if __name__ == "__main__":
    main()
