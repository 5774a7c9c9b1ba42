"""Newton iteration of the contact-constrained quasi-static problem (oracle).  TEST INFRASTRUCTURE ONLY.

Sec. III-A: the equilibrium F(x) - F_ext(x) = 0 (eq. 1) with the external force
split of eq. 2, the contact forces of eq. 11-13, the fixed-node constraint of
eq. 14-15 and the cable wrench of eq. 18 form a nonlinear complementarity
problem (eq. 19).  Linearising the internal force about the current state
(eq. 20-21) gives a linear complementarity problem (eq. 22), which is the
optimality system of the quadratic program of eq. 23.  Sec. III-D limits the
step size and scales the multipliers by the same factor (eq. 25-27).

This oracle solves every linearised problem exactly:
  1. K = the QP tangent of eq. 23, the co-rotated constant local stiffness
     (symmetric positive definite once the base is fixed), assembled banded;
  2. the base node is prescribed (position = base target, triad fixed): its
     increment moves to the right-hand side (eq. 14);
  3. dx_free = -K^-1 r and Z = K^-1 A^T by LAPACK's banded Cholesky (scipy
     cholesky_banded / cho_solve_banded), W = A Z, q = g + A dx_free;
  4. contact forces y from Lemke's method on LCP(q, W) (eq. 12-13); dx = dx_free + Z y;
  5. step limit: if max_i |dp_i| > beta0, dx and y are scaled by beta0 / max_i |dp_i|.
The iteration repeats until the residual norm (free DOFs, SI units) falls below
tol - or stops improving once below stag_tol - with an unlimited last step, an
unchanged contact set and no gap below -1e-9 m.  Quasi-static load steps ramp the
insertion depth and the tensions; each starts from the previous equilibrium.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.linalg

from . import beam, actuation, collision, lcp

OK, NOCONV, LCPFAIL = 0, 1, 2


@dataclass
class Robot:
    """One robot: geometry, per-element rigidities EA, EI, GJ [n_e], cables, contact rule."""
    n_elem: int
    length: float
    base_pos: np.ndarray
    base_dir: np.ndarray
    base_up: np.ndarray
    EA: np.ndarray
    EI: np.ndarray
    GJ: np.ndarray
    cable_radius: float
    cable_angle: np.ndarray
    r_c: float
    delta: float
    beta0: float
    guide_len: float = 0.0
    mesh: collision.Mesh | None = None
    elements: bool = False            # contacts along elements (collision.detect_elements)
    l0: float = field(init=False)
    K12: np.ndarray = field(init=False)
    K7: np.ndarray = field(init=False)

    def __post_init__(self):
        self.l0 = self.length / self.n_elem
        ones = np.ones(self.n_elem)
        self.EA, self.EI, self.GJ = (np.asarray(v, float) * ones for v in (self.EA, self.EI, self.GJ))
        self.K12, self.K7 = beam.element_stiffness(self.l0, self.EA, self.EI, self.GJ)

    def reference(self):
        return beam.reference_state(self.n_elem, self.length, self.base_pos, self.base_dir,
                                    self.base_up)

    def guided(self, depth):
        """Nodes still inside the straight insertion guide at this depth (base excluded)."""
        s = np.arange(self.n_elem + 1) * self.l0 + depth
        g = s < self.guide_len
        g[0] = False
        return g

    def base_target(self, depth):
        d = np.asarray(self.base_dir, float)
        return np.asarray(self.base_pos, float) + depth * d / np.linalg.norm(d)


def element_rigidities(rb, b):
    """Per-element (EA, EI, GJ) of robot b: the tube section, with a stiffer shaft
    proximal to the distal bending section when the batch defines one."""
    n_e = int(rb.n_elem[b])
    EA, EI, GJ = beam.section_stiffness(rb.r_out, rb.r_in, rb.E, rb.nu)
    EA, EI, GJ = np.full(n_e, EA), np.full(n_e, EI), np.full(n_e, GJ)
    if rb.tip_len > 0.0:
        l0 = rb.length[b] / n_e
        mid = (np.arange(n_e) + 0.5) * l0
        shaft = mid < rb.length[b] - rb.tip_len
        G = rb.shaft_E / (2.0 * (1.0 + rb.nu))
        EA[shaft] = rb.shaft_E * rb.shaft_A
        EI[shaft] = rb.shaft_E * rb.shaft_I
        GJ[shaft] = G * 2.0 * rb.shaft_I
    return EA, EI, GJ


def robots_from_batch(rb, mesh=None):
    return [Robot(int(rb.n_elem[b]), float(rb.length[b]), rb.base_pos[b], rb.base_dir[b],
                  rb.base_up[b], *element_rigidities(rb, b), rb.cable_radius,
                  np.asarray(rb.cable_angle),
                  rb.contact_radius, rb.contact_margin, rb.beta0,
                  rb.guide_len, mesh)
            for b in range(rb.n_robots)]


def out_of_balance(robot, P, R, act_kind, act_values):
    """F(x) - F_a(x) at every node [N,6] (contact and base reaction excluded)."""
    return (beam.internal_forces(P, R, robot.l0, robot.K7)
            - actuation.load_vector(R, act_kind, act_values, robot.cable_radius,
                                    robot.cable_angle))


def detect(robot, P, guided=None, prev=None):
    """Contacts of the current iterate.  With prev = (contacts, y) of the previous Newton
    iterate, its active contacts that were not detected again persist (a face as its plane,
    an edge/vertex contact as the direction from the triangle's nearest point) while the
    node stays within the detection band of that triangle and no detected contact at the
    node lies on the same plane (see persist_faces)."""
    if robot.mesh is None:
        return []
    det = collision.active(collision.detect(P, robot.mesh, robot.r_c, robot.delta, skip=guided))
    if robot.elements:
        det = det + collision.active(collision.detect_elements(P, robot.mesh, robot.r_c, robot.delta,
                                                               skip=guided))
        det.sort(key=lambda c: (c["node"], c["kind"], c["tri"]))
    if prev is None:
        return det
    return persist_faces(robot, P, det, *prev)


PLANE_TOL = 1e-9


def persist_faces(robot, P, det, cont_prev, y_prev):
    """Detected contacts plus the persisting ones, ordered by (node, kind, triangle).

    Within a Newton loop the iterate can cross from one triangle's face region into the
    neighbouring edge or vertex region and back on every step, so that the detected set
    never settles (a 2-cycle between a face contact and the edge/vertex fallback, which is
    only detected while the node has no detected face contact).  A contact that carried
    force (y > 0) in the previous iterate and is not detected again with the same triangle
    and kind therefore stays, as long as the node's distance to the triangle is at most
    r_c + delta:
      * a face contact as its plane, gap n_t . (p - v0_t) - r_c;
      * an edge/vertex contact as the direction from the triangle's nearest point q,
        n = (p - q) / |p - q|, gap |p - q| - r_c, while the node is on the triangle's inner
        side (n_t . (p - v0_t) > 0, the fallback's own condition).
    It is dropped when a detected contact at the node has the same plane (normals and gaps
    equal within PLANE_TOL: coplanar neighbours).  A contact along element i (kind 2) is
    re-evaluated against its triangle with the chord's current position: it stays while
    0 < s* < 1, the chord point p(s*) lies in front of the triangle and within r_c + delta of
    it (normal and gap from the triangle's nearest point to p), unless a detected contact of
    the same element has the same normal, gap and s within PLANE_TOL.
    """
    mesh = robot.mesh
    band = robot.r_c + robot.delta
    keys = {(c["node"], c["tri"], c["kind"]) for c in det}
    by_node = {}
    for c in det:
        by_node.setdefault(c["node"], []).append(c)
    extra = []
    for c, y in zip(cont_prev, y_prev):
        key = (c["node"], c["tri"], c["kind"])
        if not (y > 0.0) or key in keys:
            continue
        i, t = c["node"], c["tri"]
        if c["kind"] == collision.ELEMENT:
            s, p, _, cp, _, _, front, dist = collision.element_contact_geometry(P[i], P[i + 1], mesh, t)
            if not (0.0 < s < 1.0 and front > 0.0 and 0.0 < dist <= band):
                continue
            n, gap = (p - cp) / dist, dist - robot.r_c
            if any(o["kind"] == collision.ELEMENT and abs(float(n @ o["n"]) - 1.0) <= PLANE_TOL
                   and abs(o["gap"] - gap) <= PLANE_TOL and abs(o["s"] - s) <= PLANE_TOL
                   for o in by_node.get(i, [])):
                continue
            amb = any(o.get("ambiguous", False) for o in by_node.get(i, []))
            extra.append(dict(node=i, tri=t, kind=c["kind"], s=float(s), n=n, gap=gap, ambiguous=amb))
            continue
        p = P[i]
        cpt, _, _ = collision.closest_points(p, mesh, np.array([t]))
        dist = float(np.linalg.norm(p - cpt[0]))
        if not (dist <= band):
            continue
        s_t = float(mesh.n[t] @ (p - mesh.v0[t]))
        if c["kind"] == collision.FACE:
            n, gap = mesh.n[t].copy(), s_t - robot.r_c
        else:
            if not (s_t > 0.0) or dist == 0.0:
                continue
            n, gap = (p - cpt[0]) / dist, dist - robot.r_c
        if any(abs(float(n @ o["n"]) - 1.0) <= PLANE_TOL and abs(o["gap"] - gap) <= PLANE_TOL
               for o in by_node.get(i, [])):
            continue
        amb = any(o.get("ambiguous", False) for o in by_node.get(i, []))
        extra.append(dict(node=i, tri=t, kind=c["kind"], n=n, gap=gap, ambiguous=amb))
    return sorted(det + extra, key=lambda c: (c["node"], c["kind"], c["tri"]))


def guide_dofs(robot, P, guided):
    """Prescribed lateral increments of guided nodes: {free-DOF index: increment}.

    The insertion guide is a straight rigid channel along the base direction
    (which must be a coordinate axis); inside it a node's two lateral
    coordinates are held on the channel axis (fixed-node constraints, eq. 14-15).
    """
    pres = {}
    if guided is None or not np.any(guided):
        return pres
    d = np.asarray(robot.base_dir, float)
    ax = int(np.argmax(np.abs(d)))
    lat = [k for k in range(3) if k != ax]
    for i in np.nonzero(guided)[0]:
        for k in lat:
            pres[6 * (i - 1) + k] = float(robot.base_pos[k] - P[i, k])
    return pres


def _sym_band_matvec(ab, x, ku=11):
    n = x.size
    y = np.zeros(n)
    for j in range(n):
        for i in range(max(0, j - ku), j + 1):
            a = ab[ku + i - j, j]
            y[i] += a * x[j]
            if i != j:
                y[j] += a * x[i]
    return y


def linear_step(robot, P, R, F, ab, base_target, contacts, guided=None, beta=None):
    """Exact solution of the QP of eq. 23 about (P, R); returns (dX, y, limited).

    ab is the QP tangent of all nodes in upper band storage (ku = 11).  Node 0 and
    the lateral DOFs of guided nodes have prescribed increments (eq. 14-15).
    """
    N = P.shape[0]
    nf = 6 * (N - 1)
    dx0 = np.zeros(6)
    dx0[0:3] = base_target - P[0]
    K01 = np.array([[ab[11 + i - j, j] for j in range(6, 12)] for i in range(6)])
    rhs = -F[1:].ravel().copy()
    rhs[0:6] -= K01.T @ dx0
    Kf = ab[:, 6:].copy()
    pres = guide_dofs(robot, P, guided)
    if pres:
        xp = np.zeros(nf)
        for j, v in pres.items():
            xp[j] = v
        rhs -= _sym_band_matvec(Kf, xp)
        for j, v in pres.items():
            Kf[:, j] = 0.0
            for k in range(j + 1, min(nf, j + 12)):
                Kf[11 + j - k, k] = 0.0
            Kf[11, j] = 1.0
            rhs[j] = v
    A, g = contact_rows(contacts, nf)
    cb = scipy.linalg.cholesky_banded(Kf, lower=False)
    sol = scipy.linalg.cho_solve_banded((cb, False), np.column_stack([rhs, A.T]))
    dxf = sol[:, 0]
    Z = sol[:, 1:]
    W = A @ Z
    q = g + A @ dxf
    y = lcp.lemke(W, q)
    dx = dxf + Z @ y
    dX = np.vstack([dx0[None, :], dx.reshape(N - 1, 6)])
    beta = robot.beta0 if beta is None else beta
    nrm = float(np.max(np.linalg.norm(dX[:, 0:3], axis=1)))
    limited = nrm > beta
    if limited:
        f = beta / nrm
        dX = dX * f
        y = y * f
    return dX, y, limited


def contact_rows(contacts, nf):
    """The rows A (eq. 9) and gaps g of the contacts over the nf free DOFs: n^T on the
    translations of each node of the contact's row (collision.row_entries), times its weight."""
    nc = len(contacts)
    A = np.zeros((nc, nf))
    g = np.zeros(nc)
    for c, ct in enumerate(contacts):
        for i, wgt in collision.row_entries(ct):
            A[c, 6 * (i - 1):6 * (i - 1) + 3] += wgt * np.asarray(ct["n"])
        g[c] = ct["gap"]
    return A, g


def contact_residual(F, contacts, y, robot=None, guided=None):
    """Residual over the free DOFs: F - F_a - A^T y, with guided lateral DOFs zeroed
    (their out-of-balance is the guide's reaction)."""
    r = F[1:].copy()
    for c, ct in enumerate(contacts):
        for i, wgt in collision.row_entries(ct):
            r[i - 1, 0:3] -= wgt * y[c] * ct["n"]
    if guided is not None and np.any(guided):
        ax = int(np.argmax(np.abs(robot.base_dir)))
        lat = [k for k in range(3) if k != ax]
        for k in lat:
            r[guided[1:], k] = 0.0
    return r


BETA_HALVING = 10      # contact-set changes between halvings of the step limit
BETA_MIN_FRAC = 1.0 / 64.0


def step_limit(beta0, n_switch):
    """Step limit after n_switch changes of the detected contact set within the
    current load step: beta0, halved every BETA_HALVING changes down to
    beta0 * BETA_MIN_FRAC, so that an iteration that keeps switching contact
    sets takes ever shorter steps while contact-free iterations keep beta0."""
    return beta0 * max(BETA_MIN_FRAC, 0.5 ** (n_switch // BETA_HALVING))


def stagnation_tol(robot, stag_tol):
    """Residual level below which a stagnating residual is accepted: stag_tol, raised to ten
    times the rounding floor of the out-of-balance force, eps * max(EA)/l0 * (1 m) *
    sqrt(DOFs) - node coordinates of order 1 m carry eps m of rounding, which the axial
    stiffness turns into force."""
    floor = np.finfo(float).eps * float(np.max(robot.EA)) / robot.l0 * np.sqrt(6.0 * (robot.n_elem + 1))
    return max(stag_tol, 10.0 * floor)


def solve_load_step(robot, P, R, base_target, act_kind, act_values, tol=1e-10,
                    stag_tol=1e-9, max_iter=200, guided=None, qp=None):
    """Newton iteration of one quasi-static load step from (P, R).

    qp = None solves each QP of eq. 23 exactly; qp = dict(rho=..., eps=..., max_iter=...)
    solves it with the ADMM iteration of oracle.admm (the paper's OSQP variant).
    Returns (P, R, contacts, y, info) with info = dict(status, iters, n_limited, res_norm)
    (plus qp_iters, the ADMM iterations summed over the load step, with qp).
    """
    stag_tol = stagnation_tol(robot, stag_tol)
    resid = lambda P_, R_: out_of_balance(robot, P_, R_, act_kind, act_values)
    prev = None
    rn_prev = np.inf
    n_lim = 0
    n_switch = 0
    rn = np.inf
    qp_iters = 0
    for it in range(max_iter + 1):
        F = resid(P, R)
        contacts = detect(robot, P, guided, None if prev is None else (prev[1], prev[0]))
        if prev is not None:
            y_p, cont_p, lim_p = prev
            rn = float(np.linalg.norm(contact_residual(F, cont_p, y_p, robot, guided)))
            same = collision.contact_set(contacts) == collision.contact_set(cont_p)
            n_switch += int(not same)
            gmin = min([ct["gap"] for ct in contacts], default=np.inf)
            if (same and not lim_p and gmin >= -1e-9
                    and (rn <= tol or (rn <= stag_tol and rn > 0.5 * rn_prev))):
                info = dict(status=OK, iters=it, n_limited=n_lim, res_norm=rn)
                if qp is not None:
                    info["qp_iters"] = qp_iters
                return P, R, cont_p, y_p, info
            rn_prev = rn
        if it == max_iter:
            break
        ab = beam.tangent_qp_upper_banded(P, R, robot.K12)
        if qp is not None:
            from . import admm
            dX, y, limited, qit = admm.linear_step_admm(robot, P, R, F, ab, base_target, contacts,
                                                        guided, step_limit(robot.beta0, n_switch), **qp)
            qp_iters += qit
        else:
            try:
                dX, y, limited = linear_step(robot, P, R, F, ab, base_target, contacts, guided,
                                             step_limit(robot.beta0, n_switch))
            except lcp.LCPFailure:
                return P, R, contacts, np.zeros(len(contacts)), dict(
                    status=LCPFAIL, iters=it, n_limited=n_lim, res_norm=rn)
        n_lim += int(limited)
        P, R = beam.apply_increment(P, R, dX)
        prev = (y, contacts, limited)
    y_p, cont_p, _ = prev
    info = dict(status=NOCONV, iters=max_iter, n_limited=n_lim, res_norm=rn)
    if qp is not None:
        info["qp_iters"] = qp_iters
    return P, R, cont_p, y_p, info


def solve_robot(robot, schedule, n_steps, act_kind=actuation.CABLES, state=None,
                record=True, stop_on_failure=False, **kw):
    """Quasi-static load stepping: schedule(k) -> (depth, act_values) for k = 1..n_steps.

    A load step that does not converge keeps its last iterate and the next load
    step starts from it (its status records the failure).
    """
    P, R = robot.reference() if state is None else state
    traj = []
    for k in range(1, n_steps + 1):
        depth, vals = schedule(k)
        P, R, cont, y, info = solve_load_step(robot, P, R, robot.base_target(depth), act_kind,
                                              vals, guided=robot.guided(depth), **kw)
        info["step"] = k
        if record:
            traj.append(dict(P=P.copy(), R=R.copy(), contacts=cont, y=y.copy(), info=info))
        if stop_on_failure and info["status"] != OK:
            break
    return P, R, traj
