"""Synthetic lumen meshes standing in for the paper's MRI-reconstructed cavity.

The paper matches robot nodes against a triangle mesh of the bronchial cavity
reconstructed from pre-operative MRI (Sec. II-C, Sec. III-C, Sec. IV-A).  Those
meshes are not available, so two seeded generators produce meshes of the same
kind: a straight faceted tube, and a bifurcating airway tree of tapering tubes
with a perturbed wall, open junctions and a straight introducer tube in front.

Every triangle is wound so that (v1 - v0) x (v2 - v0) points into the lumen
(toward the centreline).  Output: vertices float64 [V,3], triangles int32 [T,3].
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter


def _orient_inward(verts, tris, centre_of_tri):
    """Flip any triangle whose winding normal points away from its centreline point."""
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    nrm = np.cross(v1 - v0, v2 - v0)
    cen = (v0 + v1 + v2) / 3.0
    bad = np.einsum("ij,ij->i", nrm, centre_of_tri - cen) < 0
    tris = tris.copy()
    tris[bad, 1], tris[bad, 2] = tris[bad, 2].copy(), tris[bad, 1].copy()
    return tris


def _tube(rings, n_theta):
    """Triangles of a tube whose vertices are laid out ring-major, n_theta per ring."""
    n_r = rings
    j, k = np.meshgrid(np.arange(n_r - 1), np.arange(n_theta), indexing="ij")
    j = j.ravel(); k = k.ravel()
    a = j * n_theta + k
    b = j * n_theta + (k + 1) % n_theta
    c = (j + 1) * n_theta + k
    d = (j + 1) * n_theta + (k + 1) % n_theta
    t1 = np.stack([a, c, b], axis=1)
    t2 = np.stack([b, c, d], axis=1)
    return np.concatenate([t1, t2], axis=0).astype(np.int64)


def straight_cylinder_mesh(radius=4e-3, axis_xy=(0.0, 1e-3), z0=-0.02, z1=0.34,
                           n_theta=16, n_quads=16):
    """Straight faceted tube with axis parallel to z: 2*n_theta*n_quads triangles."""
    zs = np.linspace(z0, z1, n_quads + 1)
    ang = 2 * np.pi * np.arange(n_theta) / n_theta
    V = np.zeros(((n_quads + 1) * n_theta, 3))
    for j, z in enumerate(zs):
        V[j * n_theta:(j + 1) * n_theta, 0] = axis_xy[0] + radius * np.cos(ang)
        V[j * n_theta:(j + 1) * n_theta, 1] = axis_xy[1] + radius * np.sin(ang)
        V[j * n_theta:(j + 1) * n_theta, 2] = z
    T = _tube(n_quads + 1, n_theta)
    cen = (V[T[:, 0]] + V[T[:, 1]] + V[T[:, 2]]) / 3.0
    axis_pt = np.stack([np.full(len(T), axis_xy[0]), np.full(len(T), axis_xy[1]), cen[:, 2]], 1)
    T = _orient_inward(V, T, axis_pt)
    return V, T.astype(np.int32)


def _rot(axis, ang):
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def _perp(t):
    a = np.array([1.0, 0.0, 0.0]) if abs(t[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    v = a - t * (a @ t)
    return v / np.linalg.norm(v)


def _airway_tree(levels, rng, root_len=0.12, r0=8e-3, r_end=3e-3):
    segs = []
    root = dict(level=0, P0=np.zeros(3), T0=np.array([0.0, 0.0, 1.0]),
                P1=np.array([0.0, 0.0, root_len]), T1=np.array([0.0, 0.0, 1.0]),
                L=root_len, plane=np.array([1.0, 0.0, 0.0]), parent=-1, sibling=-1)
    segs.append(root)
    frontier = [0]
    while frontier:
        nxt = []
        for si in frontier:
            s = segs[si]
            if s["level"] >= levels:
                continue
            t = s["T1"]
            plane = _rot(t, np.deg2rad(90.0 + rng.uniform(-20.0, 20.0))) @ s["plane"]
            plane = plane - t * (plane @ t)
            plane /= np.linalg.norm(plane)
            kids = []
            for sgn in (+1.0, -1.0):
                half = np.deg2rad(30.0 + rng.uniform(-5.0, 5.0))
                d = _rot(plane, sgn * half) @ t
                L = 0.8 * s["L"]
                kids.append(len(segs))
                segs.append(dict(level=s["level"] + 1, P0=s["P1"].copy(), T0=t.copy(),
                                 P1=s["P1"] + L * d, T1=d, L=L, plane=plane, parent=si,
                                 sibling=-1))
            segs[kids[0]]["sibling"] = kids[1]
            segs[kids[1]]["sibling"] = kids[0]
            nxt.extend(kids)
        frontier = nxt
    for s in segs:
        s["radius"] = r0 * (r_end / r0) ** (s["level"] / max(levels, 1))
    return segs


def _hermite(s, u):
    u = u[:, None]
    h00 = 2 * u**3 - 3 * u**2 + 1
    h10 = u**3 - 2 * u**2 + u
    h01 = -2 * u**3 + 3 * u**2
    h11 = u**3 - u**2
    return h00 * s["P0"] + h10 * (s["L"] * s["T0"]) + h01 * s["P1"] + h11 * (s["L"] * s["T1"])


def _centreline(s, n_fine=400):
    u = np.linspace(0.0, 1.0, n_fine)
    P = _hermite(s, u)
    ds = np.linalg.norm(np.diff(P, axis=0), axis=1)
    arc = np.concatenate([[0.0], np.cumsum(ds)])
    return P, arc


def _ring_frames(P):
    """Rotation-minimising frames along a polyline by the double-reflection method."""
    T = np.gradient(P, axis=0)
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    Nn = np.zeros_like(P)
    Nn[0] = _perp(T[0])
    for i in range(len(P) - 1):
        v1 = P[i + 1] - P[i]
        c1 = v1 @ v1
        rL = Nn[i] - (2.0 / c1) * (v1 @ Nn[i]) * v1
        tL = T[i] - (2.0 / c1) * (v1 @ T[i]) * v1
        v2 = T[i + 1] - tL
        c2 = v2 @ v2
        Nn[i + 1] = rL - (2.0 / c2) * (v2 @ rL) * v2 if c2 > 0 else rL
        Nn[i + 1] -= T[i + 1] * (Nn[i + 1] @ T[i + 1])
        Nn[i + 1] /= np.linalg.norm(Nn[i + 1])
    Bn = np.cross(T, Nn)
    return T, Nn, Bn


def _polyline_dist(X, P):
    """Distance from points X [n,3] to the polyline P [m,3] (segment-clamped)."""
    best = np.full(len(X), np.inf)
    A = P[:-1]; D = P[1:] - P[:-1]
    dd = np.einsum("ij,ij->i", D, D)
    for c0 in range(0, len(X), 4096):
        x = X[c0:c0 + 4096]
        w = x[:, None, :] - A[None, :, :]
        t = np.clip(np.einsum("nmj,mj->nm", w, D) / dd[None, :], 0.0, 1.0)
        r = w - t[..., None] * D[None, :, :]
        best[c0:c0 + 4096] = np.sqrt(np.min(np.einsum("nmj,nmj->nm", r, r), axis=1))
    return best


def _build_tree_mesh(segs, h, n_theta, noise):
    Vs, Ts, Cs = [], [], []
    nv = 0
    cl = [_centreline(s) for s in segs]
    ang = 2 * np.pi * np.arange(n_theta) / n_theta
    for si, s in enumerate(segs):
        P, arc = cl[si]
        n_r = max(2, int(round(arc[-1] / h)) + 1)
        at = np.linspace(0.0, arc[-1], n_r)
        R = np.stack([np.interp(at, arc, P[:, d]) for d in range(3)], axis=1)
        _, Nn, Bn = _ring_frames(R)
        rad = s["radius"] + noise[si](n_r, h)
        V = (R[:, None, :] + rad[..., None] * (np.cos(ang)[None, :, None] * Nn[:, None, :]
                                                + np.sin(ang)[None, :, None] * Bn[:, None, :]))
        V = V.reshape(-1, 3)
        T = _tube(n_r, n_theta)
        cen_axis = np.repeat(R[:-1] * 0.5 + R[1:] * 0.5, n_theta, axis=0)
        cen_axis = np.concatenate([cen_axis, cen_axis], axis=0)
        T = _orient_inward(V, T, cen_axis)
        # open junctions: drop triangles whose centroid lies inside the parent or sibling tube
        cen = (V[T[:, 0]] + V[T[:, 1]] + V[T[:, 2]]) / 3.0
        keep = np.ones(len(T), bool)
        for other in (s["parent"], s["sibling"]):
            if other >= 0:
                keep &= _polyline_dist(cen, cl[other][0]) >= segs[other]["radius"]
        T = T[keep]
        Vs.append(V); Ts.append(T + nv); nv += len(V)
    return np.concatenate(Vs), np.concatenate(Ts)


def branching_lumen_mesh(levels=3, target_tris=50_000, seed=(1, 0), n_theta=32,
                         sigma=0.3e-3, corr_len=4e-3, introducer_len=0.0, introducer_rings=16):
    """Bifurcating airway tree (levels of bifurcation) tessellated to ~target_tris (+-1%).

    The tree's root runs along +z from the origin (8 mm radius, 0.12 m); each child
    is 0.8x its parent's length, branches at 30 +- 5 deg in a plane turned 90 +- 20 deg
    from its parent's plane, and radii taper to 3 mm at the last level.  Centrelines are
    tangent-continuous cubic Hermite curves, rings carry n_theta vertices with a
    radial perturbation drawn as a Gaussian random field (std sigma, correlation
    length corr_len along and around the wall, clipped at +-3 sigma), and an
    optional straight rigid introducer tube (8 mm, z in [-introducer_len, 0])
    leads into the root.
    """
    rng = np.random.default_rng(list(seed))
    segs = _airway_tree(levels, rng)
    noise_seed = rng.integers(0, 2**31 - 1, size=len(segs))

    def noise_fns():
        fns = []
        for si in range(len(segs)):
            g = np.random.default_rng([int(noise_seed[si])])
            circ = 2 * np.pi * segs[si]["radius"] / n_theta

            def field(n_r, h, g=g, circ=circ):
                w = g.normal(0.0, 1.0, size=(n_r, n_theta))
                f = gaussian_filter(w, sigma=(corr_len / h, corr_len / circ), mode=("nearest", "wrap"))
                f *= sigma / max(np.std(f), 1e-30)
                return np.clip(f, -3 * sigma, 3 * sigma)
            fns.append(field)
        return fns

    # optional introducer: straight, unperturbed, coarse rings
    r0 = segs[0]["radius"]
    if introducer_len <= 0.0:
        introducer_rings = 0
    zs = np.linspace(-introducer_len, 0.0, introducer_rings + 1) if introducer_rings else np.zeros(0)
    ang = 2 * np.pi * np.arange(n_theta) / n_theta
    VI = np.zeros((len(zs) * n_theta, 3))
    for j, z in enumerate(zs):
        VI[j * n_theta:(j + 1) * n_theta] = np.stack(
            [r0 * np.cos(ang), r0 * np.sin(ang), np.full(n_theta, z)], 1)
    if introducer_rings:
        TI = _tube(len(zs), n_theta)
        cI = (VI[TI[:, 0]] + VI[TI[:, 1]] + VI[TI[:, 2]]) / 3.0
        TI = _orient_inward(VI, TI, np.stack([np.zeros(len(TI)), np.zeros(len(TI)), cI[:, 2]], 1))
    else:
        TI = np.zeros((0, 3), np.int64)

    budget = target_tris - len(TI)
    total_len = sum(_centreline(s)[1][-1] for s in segs)
    h = 2 * n_theta * total_len / budget
    for _ in range(30):
        V, T = _build_tree_mesh(segs, h, n_theta, noise_fns())
        if abs(len(T) - budget) <= 0.005 * target_tris:
            break
        h *= len(T) / budget
    Vall = np.concatenate([VI, V])
    Tall = np.concatenate([TI, T + len(VI)])
    return Vall, Tall.astype(np.int32)


def lumen_for_config(cfg: int):
    """Lumen mesh of configuration `cfg`, seeded with default_rng([cfg, 0])."""
    if cfg == 0:
        return straight_cylinder_mesh()
    if cfg in (1, 3, 4):
        return branching_lumen_mesh(levels=3, target_tris=50_000, seed=(1, 0))
    if cfg == 2:
        return branching_lumen_mesh(levels=5, target_tris=200_000, seed=(2, 0))
    raise ValueError(f"unknown configuration {cfg}")
