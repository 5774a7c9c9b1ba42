"""Co-rotational 3D beam element (oracle, FP64, numpy).  TEST INFRASTRUCTURE ONLY.

The paper discretises the robot into M equal beam elements with six DOF per node
(Sec. II-B) and updates the tangent stiffness with a co-rotational formulation:
element motion is split into a rigid part and a pure deformation whose local
stiffness is constant and linear-elastic (Sec. III-A, text after eq. 20).  The
paper names no particular co-rotational element, so this oracle uses the
following reading (the GPU path implements the same reading independently):

* node state: position p_i and triad R_i (columns: tangent, section y, section z);
  increments are (dp_i, dtheta_i) with dtheta a *spatial* spin, R <- exp(dtheta^) R.
* element frame (Battini & Pacoste 2002): e1 along the chord, e3 normal to e1
  and the mean of the two nodal y-axes, e2 = e3 x e1.
* local deformation d = (theta_a, l - l0, theta_b): the axial stretch and the
  nodal rotations relative to the element frame, theta = log(R_e^T R_node).
* strain energy U = 1/2 d^T K7 d, where K7 is the Euler-Bernoulli space-frame
  stiffness (Przemieniecki 1968) restricted to those seven local DOFs.
* element internal force = exact gradient of U with respect to the nodal
  increments (so every element is self-equilibrated and conservative).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation


# --------------------------------------------------------------------------- section
def section_stiffness(r_out, r_in, E, nu):
    """Axial, bending and torsional rigidities (EA, EI, GJ) of a circular tube."""
    A = np.pi * (r_out**2 - r_in**2)
    I = np.pi / 4.0 * (r_out**4 - r_in**4)
    J = 2.0 * I
    G = E / (2.0 * (1.0 + nu))
    return E * A, E * I, G * J


def local_stiffness_12(l0, EA, EI, GJ):
    """12x12 Euler-Bernoulli space-frame element stiffness in local coordinates.

    DOF order: (u1 v1 w1 rx1 ry1 rz1  u2 v2 w2 rx2 ry2 rz2), I_y = I_z = I.
    """
    K = np.zeros((12, 12))
    a = EA / l0
    t = GJ / l0
    K[np.ix_([0, 6], [0, 6])] = a * np.array([[1, -1], [-1, 1]])
    K[np.ix_([3, 9], [3, 9])] = t * np.array([[1, -1], [-1, 1]])
    L = l0
    kb = EI / L**3
    # bending in the local x-y plane: (v1, rz1, v2, rz2)
    Bz = kb * np.array([[12, 6 * L, -12, 6 * L],
                        [6 * L, 4 * L * L, -6 * L, 2 * L * L],
                        [-12, -6 * L, 12, -6 * L],
                        [6 * L, 2 * L * L, -6 * L, 4 * L * L]])
    K[np.ix_([1, 5, 7, 11], [1, 5, 7, 11])] = Bz
    # bending in the local x-z plane: (w1, ry1, w2, ry2)
    By = kb * np.array([[12, -6 * L, -12, -6 * L],
                        [-6 * L, 4 * L * L, 6 * L, 2 * L * L],
                        [-12, 6 * L, 12, 6 * L],
                        [-6 * L, 2 * L * L, 6 * L, 4 * L * L]])
    K[np.ix_([2, 4, 8, 10], [2, 4, 8, 10])] = By
    return K


K7_INDEX = np.array([3, 4, 5, 6, 9, 10, 11])


def local_stiffness_7(l0, EA, EI, GJ):
    """K_l restricted to d = (rx1, ry1, rz1, u2, rx2, ry2, rz2) with the other local DOFs zero."""
    return local_stiffness_12(l0, EA, EI, GJ)[np.ix_(K7_INDEX, K7_INDEX)]


def element_stiffness(l0, EA, EI, GJ):
    """Per-element (K12 [n_e,12,12], K7 [n_e,7,7]) from per-element rigidities [n_e]."""
    K12 = np.stack([local_stiffness_12(l0, a, b, c) for a, b, c in zip(EA, EI, GJ)])
    return K12, K12[:, K7_INDEX][:, :, K7_INDEX]


# --------------------------------------------------------------------------- SO(3)
def hat(v):
    v = np.asarray(v)
    z = np.zeros(v.shape[:-1])
    return np.stack([np.stack([z, -v[..., 2], v[..., 1]], -1),
                     np.stack([v[..., 2], z, -v[..., 0]], -1),
                     np.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def expm_so3(w):
    return Rotation.from_rotvec(np.atleast_2d(w)).as_matrix().reshape(np.shape(w)[:-1] + (3, 3))


def logm_so3(R):
    R = np.asarray(R)
    return Rotation.from_matrix(R.reshape(-1, 3, 3)).as_rotvec().reshape(R.shape[:-2] + (3,))


def _beta(th):
    """beta(theta) = 1/theta^2 - (1 + cos theta) / (2 theta sin theta), with its series near 0."""
    th = np.asarray(th, dtype=float)
    out = np.empty_like(th)
    small = th < 1e-2
    t2 = th[small] ** 2
    out[small] = 1.0 / 12.0 + t2 / 720.0 + t2 * t2 / 30240.0
    tb = th[~small]
    out[~small] = 1.0 / tb**2 - (1.0 + np.cos(tb)) / (2.0 * tb * np.sin(tb))
    return out


def jl_inv(theta):
    """Inverse left Jacobian of SO(3): log(exp(w^) exp(theta^)) = theta + jl_inv(theta) w + O(w^2)."""
    th = np.linalg.norm(theta, axis=-1)
    Th = hat(theta)
    return np.eye(3) - 0.5 * Th + _beta(th)[..., None, None] * (Th @ Th)


# --------------------------------------------------------------------------- reference state
def reference_state(n_elem, length, base_pos, base_dir, base_up):
    """Straight initial configuration S_0 of one robot: positions [N,3], triads [N,3,3]."""
    t = np.asarray(base_dir, float); t = t / np.linalg.norm(t)
    u = np.asarray(base_up, float); u = u - t * (u @ t); u = u / np.linalg.norm(u)
    l0 = length / n_elem
    P = np.asarray(base_pos, float)[None, :] + np.arange(n_elem + 1)[:, None] * l0 * t[None, :]
    R0 = np.stack([t, u, np.cross(t, u)], axis=1)
    R = np.repeat(R0[None], n_elem + 1, axis=0)
    return P, R


# --------------------------------------------------------------------------- element kinematics
def element_frame(pa, Ra, pb, Rb):
    """Chord length, element triad R_e = [e1 e2 e3] and the helper vectors of its spin."""
    c = pb - pa
    l = np.linalg.norm(c, axis=-1)
    e1 = c / l[..., None]
    qa = Ra[..., :, 1]
    qb = Rb[..., :, 1]
    q = 0.5 * (qa + qb)
    r = np.cross(e1, q)
    e3 = r / np.linalg.norm(r, axis=-1)[..., None]
    e2 = np.cross(e3, e1)
    Re = np.stack([e1, e2, e3], axis=-1)
    return dict(l=l, e1=e1, e2=e2, e3=e3, Re=Re, qa=qa, qb=qb, q=q)


def element_deformation(pa, Ra, pb, Rb, l0):
    """Local deformation d = (theta_a, l - l0, theta_b) [.., 7] and the element frame."""
    fr = element_frame(pa, Ra, pb, Rb)
    Re_T = np.swapaxes(fr["Re"], -1, -2)
    tha = logm_so3(Re_T @ Ra)
    thb = logm_so3(Re_T @ Rb)
    d = np.concatenate([tha, (fr["l"] - l0)[..., None], thb], axis=-1)
    return d, fr


def element_energy(pa, Ra, pb, Rb, l0, K7):
    d, _ = element_deformation(pa, Ra, pb, Rb, l0)
    return 0.5 * np.einsum("...i,...ij,...j->...", d, K7, d)


def element_forces(pa, Ra, pb, Rb, l0, K7):
    """Element internal force vector [.., 12] = dU/d(dp_a, dtheta_a, dp_b, dtheta_b).

    From dU = s . dd with s = K7 d, the chain rule through the element-frame spin
    and the log map gives forces on the chord, moments from the nodal rotations
    and the moment needed to turn the element frame.
    """
    d, fr = element_deformation(pa, Ra, pb, Rb, l0)
    s = np.einsum("...ij,...j->...i", K7, d)
    tha, thb = d[..., 0:3], d[..., 4:7]
    N = s[..., 3]
    # local end moments through the inverse left Jacobian of the log map
    ma = np.einsum("...ji,...j->...i", jl_inv(tha), s[..., 0:3])
    mb = np.einsum("...ji,...j->...i", jl_inv(thb), s[..., 4:7])
    m = ma + mb
    e1, e2, e3, l, Re = fr["e1"], fr["e2"], fr["e3"], fr["l"], fr["Re"]
    q1 = np.einsum("...i,...i->...", fr["q"], e1)
    q2 = np.einsum("...i,...i->...", fr["q"], e2)
    fpb = (N[..., None] * e1
           + ((m[..., 0] * q1 / q2 + m[..., 1]) / l)[..., None] * e3
           - (m[..., 2] / l)[..., None] * e2)
    c1 = (m[..., 0] / (2.0 * q2))[..., None]
    fta = np.einsum("...ij,...j->...i", Re, ma) - c1 * np.cross(fr["qa"], e3)
    ftb = np.einsum("...ij,...j->...i", Re, mb) - c1 * np.cross(fr["qb"], e3)
    return np.concatenate([-fpb, fta, fpb, ftb], axis=-1)


def internal_forces(P, R, l0, K7):
    """Assembled internal force vector F(x) [N,6] of one robot (eq. 1)."""
    fe = element_forces(P[:-1], R[:-1], P[1:], R[1:], l0, K7)
    F = np.zeros((P.shape[0], 6))
    F[:-1] += fe[:, 0:6]
    F[1:] += fe[:, 6:12]
    return F


def total_energy(P, R, l0, K7):
    return float(np.sum(element_energy(P[:-1], R[:-1], P[1:], R[1:], l0, K7)))


# --------------------------------------------------------------------------- state update
def apply_increment(P, R, dX):
    """x <- x (+) dx: translate positions, rotate triads by the spatial spin exp(dtheta^)."""
    return P + dX[:, 0:3], expm_so3(dX[:, 3:6]) @ R


def fd_jacobian_banded(resid, P, R, h=1e-7):
    """Central finite-difference Jacobian of resid(P, R) -> [N,6], banded (11, 11) LAPACK storage.

    Nodes interact only with their neighbours, so nodes three apart are perturbed
    together; each column of d(resid)/d(dx) is recovered from its unique neighbour.
    Returns ab with ab[11 + i - j, j] = J[i, j] for |i - j| <= 11.
    """
    N = P.shape[0]
    n = 6 * N
    ab = np.zeros((23, n))
    for c in range(3):
        nodes = np.arange(c, N, 3)
        for k in range(6):
            dX = np.zeros((N, 6))
            dX[nodes, k] = h
            Pp, Rp = apply_increment(P, R, dX)
            Pm, Rm = apply_increment(P, R, -dX)
            dF = (resid(Pp, Rp) - resid(Pm, Rm)) / (2.0 * h)
            for j in nodes:
                col = 6 * j + k
                for i in range(max(0, j - 1), min(N, j + 2)):
                    for a in range(6):
                        row = 6 * i + a
                        ab[11 + row - col, col] = dF[i, a]
    return ab


def banded_to_dense(ab, n, kl=11, ku=11):
    J = np.zeros((n, n))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            J[i, j] = ab[ku + i - j, j]
    return J


def element_tangent_qp(Re, K12):
    """QP tangent of one element, K_e = Rcal K_l Rcal^T with Rcal = blockdiag(R_e x 4).

    This is the stiffness of eq. 20-23 as the paper uses it: the constant local
    stiffness of the co-rotational element turned into the current element frame,
    symmetric positive semi-definite (rigid motions in its null space).
    """
    Rc = np.kron(np.eye(4), Re)
    return Rc @ K12 @ Rc.T


def tangent_qp_upper_banded(P, R, K12):
    """Assembled QP tangent of one robot in LAPACK upper band storage (ku = 11).

    K12 [n_e,12,12] are the elements' local stiffnesses.
    ab[11 + i - j, j] = K[i, j] for j - 11 <= i <= j.
    """
    N = P.shape[0]
    fr = element_frame(P[:-1], R[:-1], P[1:], R[1:])
    ab = np.zeros((12, 6 * N))
    for e in range(N - 1):
        Ke = element_tangent_qp(fr["Re"][e], K12[e])
        for a in range(12):
            for b in range(a, 12):
                i, j = 6 * e + a, 6 * e + b
                ab[11 + i - j, j] += Ke[a, b]
    return ab


def upper_banded_to_dense(ab, n, ku=11):
    K = np.zeros((n, n))
    for j in range(n):
        for i in range(max(0, j - ku), j + 1):
            K[i, j] = K[j, i] = ab[ku + i - j, j]
    return K
