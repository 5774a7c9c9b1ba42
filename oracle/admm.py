"""ADMM solution of the linear step's QP (oracle).  TEST INFRASTRUCTURE ONLY.

Sec. III-B solves the QP of eq. 23 with OSQP, an operator-splitting (ADMM) method.  This is
the OSQP iteration (Stellato et al., "OSQP: an operator splitting solver for quadratic
programs", Math. Prog. Comp. 2020, Algorithm 1), without its problem scaling and with a fixed
penalty, applied to the QP of a Newton iteration written as

    min 1/2 x^T K x - b^T x   subject to   A x + g >= 0,

with K the QP tangent over the free DOFs (prescribed DOFs: identity rows, b = their
increments), b the right-hand side of the exact step (minus the out-of-balance force, the
base coupling and the prescribed increments moved over), A the contact rows n_c^T on the
contact nodes' translations and g the gaps.  In OSQP's form l <= A x <= u with l = -g,
u = +inf, and OSQP's multiplier y_o equals minus the contact force.  Per iteration:

    (K + sigma I + rho A^T A) xt = sigma x - q + A^T (rho z - y_o),   q = -b
    zt = A xt
    x <- alpha xt + (1 - alpha) x
    z_new = max(alpha zt + (1 - alpha) z + y_o / rho, l)
    y_o <- y_o + rho (alpha zt + (1 - alpha) z - z_new),   z <- z_new

stopping when the primal residual |A x - z|_inf and the dual residual
|K x + q + A^T y_o|_inf (both over the free DOFs) are below eps_abs + eps_rel times the
scale OSQP uses.  The matrix K + sigma I + rho A^T A stays block tridiagonal (every contact row
lies on one node, or two adjacent ones), so it is factored once (banded Cholesky) and every iteration is one
solve.  The prescribed DOFs keep identity rows and their increments throughout.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import solver

SIGMA = 1e-6
ALPHA = 1.6


def _band_matvec(ab, x):
    """y = K x for K symmetric in upper band storage (ku = 11)."""
    n = x.shape[0]
    y = np.zeros(n)
    for d in range(12):
        diag = ab[11 - d, d:]
        y[: n - d] += diag * x[d:]
        if d:
            y[d:] += diag * x[: n - d]
    return y


def qp_data(robot, P, R, F, ab, base_target, contacts, guided=None):
    """The free-DOF QP of the linear step: (Kf banded, b, A, g, prescribed index list, dx0)."""
    N = P.shape[0]
    nf = 6 * (N - 1)
    dx0 = np.zeros(6)
    dx0[0:3] = base_target - P[0]
    K01 = np.array([[ab[11 + i - j, j] for j in range(6, 12)] for i in range(6)])
    b = -F[1:].ravel().copy()
    b[0:6] -= K01.T @ dx0
    Kf = ab[:, 6:].copy()
    pres = solver.guide_dofs(robot, P, guided)
    if pres:
        xp = np.zeros(nf)
        for j, v in pres.items():
            xp[j] = v
        b -= _band_matvec(Kf, xp)
        for j, v in pres.items():
            Kf[:, j] = 0.0
            for k in range(j + 1, min(nf, j + 12)):
                Kf[11 + j - k, k] = 0.0
            Kf[11, j] = 1.0
            b[j] = v
    A, g = solver.contact_rows(contacts, nf)
    for j in pres:
        A[:, j] = 0.0
    return Kf, b, A, g, sorted(pres), dx0


def admm_qp(Kf, b, A, g, fixed, rho, eps_abs=1e-10, eps_rel=1e-10, max_iter=10000):
    """OSQP iterations on min 1/2 x^T K x - b^T x, A x + g >= 0.  Returns (x, force, iters,
    converged) with force = -y_o >= 0 the contact forces."""
    nf = b.shape[0]
    nc = A.shape[0]
    free = np.ones(nf, bool)
    free[list(fixed)] = False
    M = Kf.copy()
    M[11, :] += np.where(free, SIGMA, 0.0)
    # rho A^T A: every contact row lies on the translations of one node or of two adjacent
    # ones (a contact along an element), inside the band
    AtA = rho * (A.T @ A)
    for d in range(12):
        M[11 - d, d:] += np.diagonal(AtA, offset=d)
    cb = scipy.linalg.cholesky_banded(M, lower=False)
    q = -b
    l = -g
    x = np.where(free, 0.0, b)
    z = np.zeros(nc)
    y = np.zeros(nc)
    for it in range(1, max_iter + 1):
        rhs = SIGMA * x - q + A.T @ (rho * z - y)
        rhs[~free] = b[~free]
        xt = scipy.linalg.cho_solve_banded((cb, False), rhs)
        zt = A @ xt
        x = ALPHA * xt + (1.0 - ALPHA) * x
        zr = ALPHA * zt + (1.0 - ALPHA) * z
        zn = np.maximum(zr + y / rho, l)
        y = y + rho * (zr - zn)
        z = zn
        Ax = A @ x
        Kx = _band_matvec(Kf, x)
        Aty = A.T @ y
        rp = np.abs(Ax - z).max(initial=0.0)
        rd_v = (Kx + q + Aty)[free]
        rd = np.abs(rd_v).max(initial=0.0)
        ep = eps_abs + eps_rel * max(np.abs(Ax).max(initial=0.0), np.abs(z).max(initial=0.0))
        ed = eps_abs + eps_rel * max(np.abs(Kx[free]).max(initial=0.0), np.abs(Aty[free]).max(initial=0.0),
                                     np.abs(q[free]).max(initial=0.0))
        if rp <= ep and rd <= ed:
            return x, -y, it, True
    return x, -y, max_iter, False


def linear_step_admm(robot, P, R, F, ab, base_target, contacts, guided=None, beta=None, rho=1.0,
                     eps=1e-11, max_iter=20000):
    """The linear step of a Newton iteration with the QP of eq. 23 solved by the iteration
    above instead of exactly; returns (dX, y, limited, iters) like solver.linear_step plus
    the ADMM iteration count (the step limit of eq. 25-27 as there)."""
    N = P.shape[0]
    Kf, b, A, g, fixed, dx0 = qp_data(robot, P, R, F, ab, base_target, contacts, guided)
    x, y, iters, _ = admm_qp(Kf, b, A, g, fixed, rho, eps_abs=eps, eps_rel=eps, max_iter=max_iter)
    dX = np.vstack([dx0[None, :], x.reshape(N - 1, 6)])
    beta = robot.beta0 if beta is None else beta
    nrm = float(np.max(np.linalg.norm(dX[:, 0:3], axis=1)))
    limited = nrm > beta
    if limited:
        f = beta / nrm
        dX = dX * f
        y = y * f
    return dX, y, limited, iters
