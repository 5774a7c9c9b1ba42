"""Cable actuation carried to the tip node (oracle).  TEST INFRASTRUCTURE ONLY.

Sec. II-E: every cable tension F_j is moved to the centre of the distal section
as the force F_j plus the moment M_j = d_j x F_j (eq. 16), both expressed in the
tip node's local frame, and then rotated to global coordinates by the tip triad
T_M (eq. 17, eq. 18).  The wrench therefore follows the tip (a follower load).

Readings of what the paper leaves unstated:
* cable j is attached at d_j = r_c (0, cos phi_j, sin phi_j) in the tip section
  and pulls toward the base, F_j = -T_j e_x (local), so that
  M_j = d_j x F_j = T_j r_c (0, -sin phi_j, cos phi_j);
* two kinds of cable load are provided.  CABLE_WRENCH is eq. 17-18 as
  printed: the tip node receives the summed cable force sum_j F_j and the
  moments sum_j M_j, both turned by the tip triad.  CABLES (the default of the
  insertion workloads) keeps only the moments: the cable runs inside the tube
  from the tip back to the actuators at the base, so the tube carries the
  cable's pull as internal compression and the pair exerts no net axial force
  on the beam.  Applying sum_j F_j as an external compressive follower force
  gives loads of ~10^3 Euler loads at the configured tensions, where the
  paper's symmetric tangent iteration diverges and the linearised contact
  problems lose their P-matrix property; with CABLE_WRENCH the iteration
  converges only at small tensions (a few Euler loads).
Tip-wrench test modes apply an arbitrary given force and moment instead.
"""
from __future__ import annotations

import numpy as np

CABLES = 0          # values = tensions [n_cables]
TIP_LOCAL = 1       # values = (F, M) in the tip frame (follower)
TIP_GLOBAL = 2      # values = (F, M) in global coordinates (dead load)
CABLE_WRENCH = 3    # values = tensions [n_cables]; force and moment of eq. 17 (follower)


def cable_wrench_local(tensions, cable_radius, cable_angle):
    """Sum over cables of (F_j, d_j x F_j) in the tip frame (eq. 16)."""
    T = np.asarray(tensions, float)
    F = np.array([-T.sum(), 0.0, 0.0])
    M = np.zeros(3)
    for Tj, phi in zip(T, cable_angle):
        d = cable_radius * np.array([0.0, np.cos(phi), np.sin(phi)])
        M += np.cross(d, np.array([-Tj, 0.0, 0.0]))
    return F, M


def tip_wrench(R_tip, kind, values, cable_radius=None, cable_angle=None):
    """Global 6-vector (force, moment) applied at the tip node (eq. 18)."""
    v = np.asarray(values, float)
    if kind == CABLES:
        _, M = cable_wrench_local(v, cable_radius, cable_angle)
        return np.concatenate([np.zeros(3), R_tip @ M])
    if kind == CABLE_WRENCH:
        F, M = cable_wrench_local(v, cable_radius, cable_angle)
        return np.concatenate([R_tip @ F, R_tip @ M])
    if kind == TIP_LOCAL:
        return np.concatenate([R_tip @ v[0:3], R_tip @ v[3:6]])
    if kind == TIP_GLOBAL:
        return v[0:6].copy()
    raise ValueError(kind)


def load_vector(R, kind, values, cable_radius=None, cable_angle=None):
    """Assembled actuation load F_a [N,6]: non-zero on the last node only."""
    F = np.zeros((R.shape[0], 6))
    F[-1] = tip_wrench(R[-1], kind, values, cable_radius, cable_angle)
    return F


def literal_cable_wrench(R_tip, tensions, cable_radius, cable_angle):
    """Tip wrench of eq. 17-18 as printed (the CABLE_WRENCH kind): the summed cable force
    applied as an external follower force together with the cable moments."""
    return tip_wrench(R_tip, CABLE_WRENCH, tensions, cable_radius, cable_angle)


def tension_gradient(R_tip, cable_radius, cable_angle, kind=CABLES):
    """d(tip wrench)/d(T_j) [6, n_cables] in global coordinates: the follower moment of
    cable j, plus its follower force -e_x for the CABLE_WRENCH kind."""
    out = np.zeros((6, len(cable_angle)))
    for j, phi in enumerate(cable_angle):
        M = cable_radius * np.array([0.0, -np.sin(phi), np.cos(phi)])
        out[3:6, j] = R_tip @ M
        if kind == CABLE_WRENCH:
            out[0:3, j] = -R_tip[:, 0]
    return out
