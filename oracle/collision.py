"""Node-versus-triangle contact detection (oracle, brute force, FP64).  TEST INFRASTRUCTURE ONLY.

Sec. III-C matches every robot node against every triangle of the cavity mesh
and builds, for each detected contact, the constraint of eq. 3: with the wall
normal n_i oriented away from the robot and a point X_I of the triangle's plane,
the node must stay on the robot's side of that plane.  Stacking the contacts
gives the rows A_c and the gaps b_c of eq. 8-10.

Reading of the unstated detection rule (the GPU path implements the same rule):
* triangle normal n_t = unit((v1 - v0) x (v2 - v0)) points into the lumen, so
  the paper's n_i is -n_t; signed wall distance s = n_t . (p - v0); the
  closest point c of the triangle to the node and its Voronoi region (face,
  edge or vertex) follow Ericson 2005, Real-Time Collision Detection, Sec. 5.1.5;
* face contacts: every triangle whose closest point lies in its face region
  and with -r_c <= s <= r_c + delta (r_c = robot radius, delta = detection
  margin).  A node may carry several: near a concave facet edge a single
  constraint would let the node slide along one plane into its neighbour's
  half-space and the Newton iterates would cycle.  Row: n_t on the node's
  translations (the node-only case of the shape functions of eq. 4-6); gap
  g = s - r_c (b_c, eq. 10);
* edge/vertex fallback: a node with no face contact that lies in front of a
  triangle (s > 0) within r_c + delta of its closest edge or vertex point gets
  one contact, the nearest such point (ties to the lowest triangle index),
  with normal (p - c)/|p - c| and gap |p - c| - r_c.  Without it a node whose
  centre sits r_c off a convex ridge of the wall lies in neither face region
  and slips through the wedge between them;
* the clamped base node and nodes held by the insertion guide are never
  contact nodes.  Contacts are ordered by node, then triangle index;
* contacts along an element (eq. 3-7 at 0 < xi < l0, optional): see
  detect_elements below.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

AMBIG_TOL = 1e-9   # metres: decisions closer than this to a threshold are flagged


class Mesh:
    """Triangle soup with per-triangle planes and altitudes (precomputed once)."""

    def __init__(self, verts, tris):
        self.V = np.asarray(verts, float)
        self.T = np.asarray(tris, np.int64)
        self.v0 = self.V[self.T[:, 0]]
        self.v1 = self.V[self.T[:, 1]]
        self.v2 = self.V[self.T[:, 2]]
        nrm = np.cross(self.v1 - self.v0, self.v2 - self.v0)
        area2 = np.linalg.norm(nrm, axis=1)
        self.n = nrm / area2[:, None]
        # altitude from each vertex to its opposite edge, for barycentric -> metres
        e_opp = [np.linalg.norm(self.v2 - self.v1, axis=1),
                 np.linalg.norm(self.v2 - self.v0, axis=1),
                 np.linalg.norm(self.v1 - self.v0, axis=1)]
        self.alt = np.stack([area2 / e for e in e_opp], axis=1)
        cen = (self.v0 + self.v1 + self.v2) / 3.0
        self.centroid = cen
        self.circum = np.max(np.stack([np.linalg.norm(self.v0 - cen, axis=1),
                                       np.linalg.norm(self.v1 - cen, axis=1),
                                       np.linalg.norm(self.v2 - cen, axis=1)], 1), axis=1)
        self._tree = None
        self._sharp = None

    @property
    def sharp(self):
        """Sharp convex features, [T, 6] booleans: edges ab, ac, bc, then vertices a, b, c
        (see sharp_features)."""
        if self._sharp is None:
            self._sharp = sharp_features(self)
        return self._sharp

    @property
    def tree(self):
        if self._tree is None:
            self._tree = cKDTree(self.centroid)
        return self._tree


FACE, EDGE_AB, EDGE_AC, EDGE_BC, VERT_A, VERT_B, VERT_C = range(7)


def closest_points(p, mesh, idx):
    """Closest point of each triangle idx to p, its Voronoi region, and the smallest
    distance (m) of p's classification quantities to a region boundary."""
    a, b, c = mesh.v0[idx], mesh.v1[idx], mesh.v2[idx]
    ab = b - a
    ac = c - a
    bc = c - b
    lab = np.linalg.norm(ab, axis=1)
    lac = np.linalg.norm(ac, axis=1)
    lbc = np.linalg.norm(bc, axis=1)
    dot = lambda u, v: np.einsum("ij,ij->i", u, v)
    ap = p[None, :] - a
    bp = p[None, :] - b
    cp = p[None, :] - c
    d1, d2 = dot(ab, ap), dot(ac, ap)
    d3, d4 = dot(ab, bp), dot(ac, bp)
    d5, d6 = dot(ab, cp), dot(ac, cp)
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    n = len(idx)
    region = np.full(n, FACE)
    cpt = np.empty((n, 3))
    done = np.zeros(n, bool)

    def take(mask, reg, pts):
        m = mask & ~done
        region[m] = reg
        cpt[m] = pts[m]
        done[m] = True

    take((d1 <= 0) & (d2 <= 0), VERT_A, a)
    take((d3 >= 0) & (d4 <= d3), VERT_B, b)
    with np.errstate(divide="ignore", invalid="ignore"):
        v = d1 / (d1 - d3)
        take((vc <= 0) & (d1 >= 0) & (d3 <= 0), EDGE_AB, a + v[:, None] * ab)
        take((d6 >= 0) & (d5 <= d6), VERT_C, c)
        w = d2 / (d2 - d6)
        take((vb <= 0) & (d2 >= 0) & (d6 <= 0), EDGE_AC, a + w[:, None] * ac)
        w2 = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        take((va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0), EDGE_BC, b + w2[:, None] * bc)
        den = 1.0 / (va + vb + vc)
        vf = (vb * den)[:, None]
        wf = (vc * den)[:, None]
        take(np.ones(n, bool), FACE, a + ab * vf + ac * wf)
        area2 = np.linalg.norm(np.cross(ab, ac), axis=1)
        margin = np.min(np.abs(np.stack([
            d1 / lab, d2 / lac, d3 / lab, (d4 - d3) / lbc, d6 / lac, (d5 - d6) / lbc,
            va / (area2 * lbc), vb / (area2 * lac), vc / (area2 * lab)])), axis=0)
    return cpt, region, margin


def detect(P, mesh, r_c, delta, cull=True, first_node=1, skip=None):
    """Contacts of one robot: list of dicts (node, tri, kind, n, gap, ambiguous).

    kind is 0 for a face contact and 1 for the edge/vertex fallback.  Brute force
    over all triangles, or over the k-d-tree superset of triangles whose
    circumscribing ball can reach the detection band when cull=True (same result).
    A node whose decisions lie within AMBIG_TOL metres of a threshold gets
    ambiguous=True on its entries (and an entry with tri=-1 if it has none).
    """
    out = []
    band = r_c + delta
    reach = band + float(np.max(mesh.circum)) + 1e-6
    for i in range(first_node, P.shape[0]):
        if skip is not None and skip[i]:
            continue
        p = P[i]
        if cull:
            idx = np.asarray(mesh.tree.query_ball_point(p, reach), dtype=np.int64)
            idx.sort()
        else:
            idx = np.arange(mesh.T.shape[0])
        if idx.size == 0:
            continue
        s = np.einsum("ij,ij->i", mesh.n[idx], p[None, :] - mesh.v0[idx])
        cpt, region, margin = closest_points(p, mesh, idx)
        dist = np.linalg.norm(p[None, :] - cpt, axis=1)
        face = (region == FACE) & (s >= -r_c) & (s <= band)
        # decisions within AMBIG_TOL of a threshold, for triangles that can matter
        near = (dist <= band + AMBIG_TOL) & (s >= -r_c - AMBIG_TOL)
        amb = bool(np.any(near & (margin <= AMBIG_TOL)))
        amb |= bool(np.any((region == FACE) & ((np.abs(s + r_c) <= AMBIG_TOL)
                                               | (np.abs(s - band) <= AMBIG_TOL))))
        node_out = []
        for k in np.nonzero(face)[0]:
            t = int(idx[k])
            node_out.append(dict(node=i, tri=t, kind=0, n=mesh.n[t].copy(),
                                 gap=float(s[k] - r_c)))
        if not node_out:
            feat = (region != FACE) & (s > 0.0) & (dist <= band)
            amb |= bool(np.any((region != FACE) & (np.abs(dist - band) <= AMBIG_TOL)))
            amb |= bool(np.any((region != FACE) & (np.abs(s) <= AMBIG_TOL) & (dist <= band)))
            if np.any(feat):
                ks = np.nonzero(feat)[0]
                order = np.lexsort((idx[ks], dist[ks]))
                k = ks[order[0]]
                if order.size > 1:
                    k2 = ks[order[1]]
                    if (abs(dist[k2] - dist[k]) <= AMBIG_TOL
                            and np.linalg.norm(cpt[k2] - cpt[k]) > AMBIG_TOL):
                        amb = True
                t = int(idx[k])
                node_out.append(dict(node=i, tri=t, kind=1, n=(p - cpt[k]) / dist[k],
                                     gap=float(dist[k] - r_c)))
        for c in node_out:
            c["ambiguous"] = amb
        if not node_out and amb:
            node_out.append(dict(node=i, tri=-1, kind=-1, n=None, gap=np.nan, ambiguous=True))
        out.extend(node_out)
    return out


def contact_set(contacts):
    """The (node, triangle, kind) keys of the detected contacts (ambiguous misses dropped)."""
    return tuple((c["node"], c["tri"], c["kind"]) for c in contacts if c["tri"] >= 0)


def active(contacts):
    return [c for c in contacts if c["tri"] >= 0]


# ---------------------------------------------------------------- contact along an element
# Eq. 3-7 put the contact point anywhere on an element, at xi in [0, l0] from its base-side
# node, with N_i(xi) interpolating the two nodes' positions (B_i extracts their translations).
# Reading: N_i acts in the element's chord frame, where both nodes lie on the axis, so its
# Hermite transverse blend P3 + P4 = 1 returns their common transverse coordinate and the
# point is the chord point p(s) = (1 - s) x_i + s x_{i+1}, s = xi / l0.  Node contacts are the
# cases s = 0 and s = 1; on a triangle mesh the chord's interior comes closest to a convex
# edge or vertex of the wall (against a plane the gap is linear in s, so the nearest point of
# the chord to it is an end), which is what the element contacts below detect:
#  * for every element whose two nodes are both contact nodes (not the clamped base, not held
#    by the insertion guide) and every triangle t: the closest points of the chord and each
#    of t's three edges (segment-segment, Ericson 2005, Real-Time Collision Detection, Sec.
#    5.1.9), the nearest edge giving s* and the chord point p = p(s*);
#  * a candidate when 0 < s* < 1, p lies in front of t (n_t . (p - v0) > 0), the closest
#    point c of t to p lies on its boundary (edge or vertex region), on a sharp convex feature
#    of the wall (sharp_features), and |p - c| <= r_c + delta;
#    an edge (nearly) parallel to the chord, sin^2 of their angle below SEG_PARALLEL, gives
#    none (the closest pair is not unique; the nodes' own contacts hold such a chord);
#  * the element's contact is its nearest candidate (ties to the lowest triangle index):
#    kind 2, stored at its base-side node i with s = s*, normal n = (p - c)/|p - c|, gap
#    |p - c| - r_c; its constraint row is (1 - s) n^T on node i's translations and s n^T on
#    node i+1's (the derivative of the gap of p(s) at fixed s), so that the contact force
#    (eq. 11) acts as (1 - s) y n and s y n on the two nodes, statically equivalent to y n
#    at p.
SEG_PARALLEL = 1e-6
ELEMENT = 2
SHARP_FOLD_COS = float(np.cos(np.radians(10.0)))


def sharp_features(mesh):
    """Which edges and vertices of each triangle are sharp convex features of the wall, where a
    contact along an element is made: an edge shared by two triangles whose far vertex of the
    neighbour lies behind the triangle's plane (convex seen from the lumen) and whose normals
    are at least 10 degrees apart (cos <= SHARP_FOLD_COS); an edge of one triangle only (the rim
    of an opening) or of more than two; a vertex on such an edge.  At a shallower fold the
    nodes' own face contacts hold a chord to within (l / 2) tan(fold / 2) of the wall, and a
    contact there would be nearly parallel to them (W close to singular).  [T, 6] booleans:
    edges ab, ac, bc, vertices a, b, c."""
    T = mesh.T
    owners = {}
    for t in range(T.shape[0]):
        for e, (i, j) in enumerate(((0, 1), (0, 2), (1, 2))):
            u, v = int(T[t, i]), int(T[t, j])
            owners.setdefault((min(u, v), max(u, v)), []).append((t, e))
    sharp = np.zeros((T.shape[0], 6), bool)
    for (u, v), own in owners.items():
        if len(own) == 2:
            (t, e), (t2, _) = own
            far = [w for w in T[t2] if w != u and w != v]
            far2 = [w for w in T[t] if w != u and w != v]
            convex = (float(mesh.n[t] @ (mesh.V[far[0]] - mesh.V[u])) < 0.0
                      and float(mesh.n[t2] @ (mesh.V[far2[0]] - mesh.V[u])) < 0.0)
            flag = convex and float(mesh.n[t] @ mesh.n[t2]) <= SHARP_FOLD_COS
        else:
            flag = True
        for t, e in own:
            sharp[t, e] = flag
    # vertices: on any sharp edge of any triangle
    vsharp = np.zeros(mesh.V.shape[0], bool)
    for (u, v), own in owners.items():
        if sharp[own[0][0], own[0][1]]:
            vsharp[u] = vsharp[v] = True
    sharp[:, 3:6] = vsharp[T]
    return sharp


_FEATURE_COL = {EDGE_AB: 0, EDGE_AC: 1, EDGE_BC: 2, VERT_A: 3, VERT_B: 4, VERT_C: 5}


def segment_closest(p1, p2, q1, q2):
    """Closest points of the segments p1p2 and q1q2 (both of positive length): parameters
    (s, u) in [0, 1]^2 of p1 + s (p2 - p1) and q1 + u (q2 - q1), their distance and the
    squared sine of the segments' angle.  The unconstrained minimiser of the squared distance
    (a 2x2 linear system) is clamped to the square, one parameter at a time."""
    d1 = p2 - p1
    d2 = q2 - q1
    r = p1 - q1
    a = float(d1 @ d1)
    e = float(d2 @ d2)
    b = float(d1 @ d2)
    c = float(d1 @ r)
    f = float(d2 @ r)
    den = a * e - b * b
    sin2 = den / (a * e)
    s = min(max((b * f - c * e) / den, 0.0), 1.0) if den > 0.0 else 0.0
    u = (b * s + f) / e
    if u < 0.0:
        u = 0.0
        s = min(max(-c / a, 0.0), 1.0)
    elif u > 1.0:
        u = 1.0
        s = min(max((b - c) / a, 0.0), 1.0)
    dist = float(np.linalg.norm(p1 + s * d1 - (q1 + u * d2)))
    return s, u, dist, sin2


def element_contact_geometry(xa, xb, mesh, t):
    """Chord xa-xb against triangle t: (s*, p, sin2 of the nearest edge, closest point c of t
    to p, its region, the region margin, the signed distance n_t . (p - v0), |p - c|)."""
    verts = (mesh.v0[t], mesh.v1[t], mesh.v2[t])
    best = None
    for ea, eb in ((0, 1), (0, 2), (1, 2)):
        s, u, dist, sin2 = segment_closest(xa, xb, verts[ea], verts[eb])
        if best is None or dist < best[2]:
            best = (s, u, dist, sin2)
    s, _, _, sin2 = best
    p = xa + s * (xb - xa)
    cpt, region, margin = closest_points(p, mesh, np.array([t]))
    front = float(mesh.n[t] @ (p - mesh.v0[t]))
    d = float(np.linalg.norm(p - cpt[0]))
    return s, p, sin2, cpt[0], int(region[0]), float(margin[0]), front, d


def detect_elements(P, mesh, r_c, delta, cull=True, first_node=1, skip=None):
    """Element contacts of one robot (kind 2, node = the element's base-side node, s = the
    contact point's position along the element), ordered by node; entries flagged ambiguous
    when a decision lies within AMBIG_TOL metres of a threshold."""
    out = []
    band = r_c + delta
    reach = band + float(np.max(mesh.circum)) + 1e-6
    for i in range(first_node, P.shape[0] - 1):
        if skip is not None and (skip[i] or skip[i + 1]):
            continue
        xa, xb = P[i], P[i + 1]
        ln = float(np.linalg.norm(xb - xa))
        if cull:
            idx = np.asarray(mesh.tree.query_ball_point(0.5 * (xa + xb), reach + 0.5 * ln), dtype=np.int64)
            idx.sort()
        else:
            idx = np.arange(mesh.T.shape[0])
        cands = []
        amb = False
        for t in idx:
            s, p, sin2, c, region, margin, front, d = element_contact_geometry(xa, xb, mesh, int(t))
            ok = (sin2 >= SEG_PARALLEL and 0.0 < s < 1.0 and front > 0.0 and region != FACE
                  and d <= band and bool(mesh.sharp[int(t), _FEATURE_COL[region]]))
            near = d <= band + AMBIG_TOL and front >= -AMBIG_TOL
            if near and (abs(sin2 - SEG_PARALLEL) <= 1e-9 or min(s, 1.0 - s) * ln <= AMBIG_TOL
                         or abs(front) <= AMBIG_TOL or margin <= AMBIG_TOL or abs(d - band) <= AMBIG_TOL):
                amb = True
            if ok:
                cands.append((d, int(t), s, p, c))
        if cands:
            cands.sort(key=lambda x: (x[0], x[1]))
            d, t, s, p, c = cands[0]
            if len(cands) > 1 and abs(cands[1][0] - d) <= AMBIG_TOL and (
                    abs(cands[1][2] - s) * ln > AMBIG_TOL or np.linalg.norm(cands[1][4] - c) > AMBIG_TOL):
                amb = True
            out.append(dict(node=i, tri=t, kind=ELEMENT, s=float(s), n=(p - c) / d,
                            gap=float(d - r_c), ambiguous=amb))
        elif amb:
            out.append(dict(node=i, tri=-1, kind=-1, n=None, gap=np.nan, s=0.0, ambiguous=True))
    return out


def row_entries(ct):
    """The constraint row of a contact as (node, weight) pairs: (node, 1) for a node contact,
    (i, 1 - s) and (i + 1, s) for a contact along element i."""
    s = float(ct.get("s", 0.0))
    if ct["kind"] == ELEMENT and s > 0.0:
        return [(ct["node"], 1.0 - s), (ct["node"] + 1, s)]
    return [(ct["node"], 1.0)]
