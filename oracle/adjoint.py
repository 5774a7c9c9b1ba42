"""Gradient of a tip-sensor loss with respect to the cable tensions (oracle).  TEST INFRASTRUCTURE ONLY.

At a converged equilibrium of a load step (Sec. III-A, eq. 19),
    R(x, T) = F(x) - F_a(x, T) - A^T y = 0,   A_act dx = 0 for the active contacts,
so a perturbation dT moves the equilibrium by dx with
    J dx - A_act^T dy = dF_a/dT dT,   A_act dx = 0,   J = d(F - F_a)/dx
(the consistent Jacobian: material + geometric stiffness of the elements and the
load stiffness of the follower moment).  For a loss L(x) with gradient g, the
adjoint pair solves  J^T lam + A_act^T mu = g,  A_act lam = 0,  and then
    dL/dT_j = lam . dF_a/dT_j.
A face contact is a plane, so its constraint has no curvature.  An edge/vertex
fallback contact constrains the distance rho = |p - q| from the node to the
nearest point q of a fixed edge line or vertex (gap rho - r_c), whose normal
n = (p - q)/rho turns with the node: dn/dp = (I - n n^T - t t^T)/rho for an edge
of unit direction t, (I - n n^T)/rho for a vertex, so the contact force -y n
adds -y dn/dp to the node's translation block of J (the constraint curvature).
A contact along element i constrains the distance from the chord point p(s*) to the fixed
edge line or vertex (s* its nearest point on the chord); its row is (1 - s*) n, s* n on the
two nodes' translations (element_gap_gradient) and its curvature, the 6x6 Hessian of that
distance, is taken by central differences of the gradient.
Fixed DOFs (base node, guided lateral DOFs) are removed.  J is taken by central
finite differences of the out-of-balance force (banded, Richardson-extrapolated), the KKT system is
solved densely.  Independent check: central differences of complete re-solves.
The same function serves the tip-wrench actuations with u the wrench.
"""
from __future__ import annotations

import numpy as np

from . import beam, actuation, solver, collision


def free_mask(robot, n_nodes, guided):
    """Boolean mask over the 6N DOFs: True where the DOF is an unknown."""
    m = np.ones(6 * n_nodes, bool)
    m[0:6] = False
    if guided is not None and np.any(guided):
        ax = int(np.argmax(np.abs(robot.base_dir)))
        for i in np.nonzero(guided)[0]:
            for k in range(3):
                if k != ax:
                    m[6 * i + k] = False
    return m


def jacobian(robot, P, R, act_kind, act_values, h=1e-6):
    """Dense consistent Jacobian d(F - F_a)/dx [6N, 6N] by banded central differences with
    one Richardson step, (4 J(h) - J(2h)) / 3.

    The geometric nonlinearity of an element varies on the scale of its length l0, so a
    plain central difference errs by about (h/l0)^2 relative; for the 1.7 mm elements of a
    350-element robot and h = 1e-7 that reached 2.5e-6 in the gradient.  The Richardson
    step leaves O((h/l0)^4) and lets h stay large enough for rounding to be negligible.
    """
    resid = lambda P_, R_: solver.out_of_balance(robot, P_, R_, act_kind, act_values)
    N = P.shape[0]
    J1 = beam.banded_to_dense(beam.fd_jacobian_banded(resid, P, R, h=h), 6 * N)
    J2 = beam.banded_to_dense(beam.fd_jacobian_banded(resid, P, R, h=2 * h), 6 * N)
    return (4.0 * J1 - J2) / 3.0


def normal_derivative(p, mesh, tri):
    """dn/dp [3, 3] of an edge/vertex contact's normal n = (p - q)/|p - q|, q the nearest
    point of triangle `tri` to p on the edge or vertex that holds it."""
    cpt, region, _ = collision.closest_points(np.asarray(p, float), mesh, np.array([tri]))
    d = np.asarray(p, float) - cpt[0]
    rho = float(np.linalg.norm(d))
    n = d / rho
    H = np.eye(3) - np.outer(n, n)
    reg = int(region[0])
    if reg == collision.FACE:
        return np.zeros((3, 3))        # nearest point inside the face: a plane
    ends = {collision.EDGE_AB: (mesh.v0, mesh.v1), collision.EDGE_AC: (mesh.v0, mesh.v2),
            collision.EDGE_BC: (mesh.v1, mesh.v2)}
    if reg in ends:
        a, b = ends[reg]
        t = b[tri] - a[tri]
        t = t / np.linalg.norm(t)
        H -= np.outer(t, t)
    return H / rho


def element_gap_gradient(xa, xb, q1, q2=None):
    """Gradient [6] of the distance from the chord xa-xb to the line through q1, q2 (or the
    point q1) with respect to (xa, xb): (1 - s) n, s n, where s is the chord parameter of the
    closest pair (unclamped) and n the unit vector from the line (point) to the chord point."""
    d1 = xb - xa
    a = float(d1 @ d1)
    if q2 is None:
        s = float((q1 - xa) @ d1) / a
        q = q1
    else:
        d2 = q2 - q1
        r = xa - q1
        e, b, c, f = float(d2 @ d2), float(d1 @ d2), float(d1 @ r), float(d2 @ r)
        s = (b * f - c * e) / (a * e - b * b)
        q = q1 + ((b * s + f) / e) * d2
    p = xa + s * d1
    n = (p - q) / np.linalg.norm(p - q)
    return np.concatenate([(1.0 - s) * n, s * n])


def element_curvature(xa, xb, mesh, tri, h=1e-7):
    """Hessian [6, 6] of the element contact's distance at (xa, xb) by central differences
    of element_gap_gradient, against the edge line or vertex of triangle `tri` that holds
    the nearest point of the chord point (zero when that point lies inside the face: a
    plane, whose distance is linear in the nodes at fixed s)."""
    s, p, _, _, region, _, _, _ = collision.element_contact_geometry(xa, xb, mesh, tri)
    if region == collision.FACE:
        return np.zeros((6, 6))
    vs = {collision.VERT_A: (mesh.v0,), collision.VERT_B: (mesh.v1,), collision.VERT_C: (mesh.v2,),
          collision.EDGE_AB: (mesh.v0, mesh.v1), collision.EDGE_AC: (mesh.v0, mesh.v2),
          collision.EDGE_BC: (mesh.v1, mesh.v2)}[region]
    feat = tuple(v[tri] for v in vs)
    x = np.concatenate([xa, xb])
    H = np.zeros((6, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        gp = element_gap_gradient((x + e)[0:3], (x + e)[3:6], *feat)
        gm = element_gap_gradient((x - e)[0:3], (x - e)[3:6], *feat)
        H[:, k] = (gp - gm) / (2.0 * h)
    return 0.5 * (H + H.T)


def loss_gradient_x(P, sensor_nodes, dL_dp):
    """Scatter dL/dp of the sensor nodes [n_s, 3] into a 6N vector."""
    g = np.zeros(6 * P.shape[0])
    for s, i in enumerate(sensor_nodes):
        g[6 * i:6 * i + 3] += dL_dp[s]
    return g


def tension_gradient(robot, P, R, contacts, y, act_values, sensor_nodes, dL_dp, guided=None,
                     act_kind=actuation.CABLES, active_tol=0.0):
    """dL/du [n_values] (cable tensions, or the tip wrench) at a converged state, for the
    loss gradient dL_dp [n_sensors, 3] at the sensor nodes."""
    N = P.shape[0]
    J = jacobian(robot, P, R, act_kind, act_values)
    for c, yy in zip(contacts, y):
        if yy > active_tol and c["kind"] == collision.ELEMENT:
            i = c["node"]
            H = element_curvature(P[i], P[i + 1], robot.mesh, c["tri"])
            idx = np.r_[6 * i:6 * i + 3, 6 * i + 6:6 * i + 9]
            J[np.ix_(idx, idx)] -= yy * H
        elif yy > active_tol and c["kind"] != 0:
            i = c["node"]
            J[6 * i:6 * i + 3, 6 * i:6 * i + 3] -= yy * normal_derivative(P[i], robot.mesh, c["tri"])
    m = free_mask(robot, N, guided)
    Jf = J[np.ix_(m, m)]
    g = loss_gradient_x(P, sensor_nodes, dL_dp)[m]
    act = [c for c, yy in zip(contacts, y) if yy > active_tol]
    idx_free = np.cumsum(m) - 1
    A = np.zeros((len(act), int(m.sum())))
    for k, c in enumerate(act):
        for i, wgt in collision.row_entries(c):
            for d in range(3):
                A[k, idx_free[6 * i + d]] += wgt * c["n"][d]
    nf = Jf.shape[0]
    na = A.shape[0]
    K = np.zeros((nf + na, nf + na))
    K[:nf, :nf] = Jf.T
    K[:nf, nf:] = A.T
    K[nf:, :nf] = A
    # least squares: the KKT matrix is singular in mu when two active normals of a node
    # coincide (the two triangles of a flat quad); lam is still unique
    sol = np.linalg.lstsq(K, np.concatenate([g, np.zeros(na)]), rcond=None)[0]
    lam = np.zeros(6 * N)
    lam[m] = sol[:nf]
    return lam[6 * (N - 1):6 * N] @ load_gradient(robot, R[-1], act_kind)


def load_gradient(robot, R_tip, act_kind):
    """dF_a/du [6, n_values] of the tip load (eq. 18) for the actuation values u."""
    if act_kind in (actuation.CABLES, actuation.CABLE_WRENCH):
        return actuation.tension_gradient(R_tip, robot.cable_radius, robot.cable_angle, act_kind)
    if act_kind == actuation.TIP_LOCAL:
        G = np.zeros((6, 6))
        G[0:3, 0:3] = R_tip
        G[3:6, 3:6] = R_tip
        return G
    return np.eye(6)


def sensor_loss(P, sensor_nodes, targets):
    """L = sum_s |p_s - p*_s|^2 and its gradient with respect to the sensor positions."""
    d = P[np.asarray(sensor_nodes)] - targets
    return float(np.sum(d * d)), 2.0 * d
