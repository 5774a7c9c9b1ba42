"""Fixtures of contact along an element (shared by the oracle pins and the GPU parity tests):
a straight cantilever (the 20-element, 0.3 m robot of the small configuration, base at the
origin along +z) beside a knife-edge ridge of the wall.

The ridge is the common edge of two triangles at x = r_c, parallel to y, at the height
z = a = (k + s) l0 inside element k; the faces recede from the robot (towards +x), one
downwards and one upwards, so that every node is farther than the detection band from both
faces and from the ridge, while the chord of element k touches the ridge at its fraction s
(gap 0 in the reference state)."""
import numpy as np

from workloads import robots_for_config


def ridge_mesh(a, x0, w=5e-3, d=20e-3, h=2e-3):
    """Vertices and triangles of the ridge: common edge (x0, -w..w, a); inward normals (into
    the lumen, towards -x)."""
    V = np.array([[x0, -w, a], [x0, w, a], [x0 + d, 0.0, a - h], [x0 + d, 0.0, a + h]], float)
    T = np.array([[0, 1, 2], [1, 0, 3]], np.int32)
    return V, T


def knife_edge_case(k=7, s=0.3):
    """(robot batch, V, T, a): the small configuration's robot with the ridge at element k,
    fraction s."""
    rb = robots_for_config(0)
    l0 = float(rb.length[0]) / int(rb.n_elem[0])
    a = (k + s) * l0
    V, T = ridge_mesh(a, rb.contact_radius)
    return rb, V, T, a


def cantilever_influence(x, c, EI):
    """Deflection at x of an Euler-Bernoulli cantilever (clamped at 0) under a unit transverse
    force at c."""
    return x * x * (3 * c - x) / (6 * EI) if x <= c else c * c * (3 * x - c) / (6 * EI)
