"""Brute-force Voronoi cells for tiny inputs (numpy, independent of any clipping).

A cell of seed p is the intersection of the box with the half-spaces
{x : n.x <= c} of all bisectors (n = q - p, c = |n|^2/2 in seed-relative
coordinates).  Its vertices are found by solving every triple of planes and
keeping the feasible solutions; a face is a plane that holds at least three
distinct vertices; the volume is sum(area_f * dist_f) / 3 with dist_f the
distance from the seed (origin) to plane f; the centroid is the volume-weighted
mean of the centroids of the pyramids from the seed over each face, each
pyramid split into tetrahedra from the mean of its face's vertices.  No
incremental clipping, no certificate: this pins the oracle, it is not the
oracle.
"""
from __future__ import annotations

import itertools

import numpy as np

WALL_IDS = (-1, -2, -3, -4, -5, -6)


def halfspaces(points: np.ndarray, i: int, lo, hi, subset=None):
    """Planes (n, c, id) of cell i in coordinates relative to points[i]."""
    p = points[i]
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    ns, cs, ids = [], [], []
    for a in range(3):
        e = np.zeros(3)
        e[a] = -1.0
        ns.append(e.copy()); cs.append(p[a] - lo[a]); ids.append(-(2 * a + 1))
        e[a] = 1.0
        ns.append(e.copy()); cs.append(hi[a] - p[a]); ids.append(-(2 * a + 2))
    others = [j for j in range(len(points)) if j != i] if subset is None else list(subset)
    for j in others:
        n = points[j] - p
        ns.append(n); cs.append(0.5 * float(n @ n)); ids.append(j)
    return np.array(ns), np.array(cs), np.array(ids)


def cell(ns: np.ndarray, cs: np.ndarray, ids: np.ndarray, tol: float = 1e-11, return_moment: bool = False):
    """Vertices, faces {id: area}, volume (and first moment about the origin)
    of {x : ns @ x <= cs} (bounded, origin inside)."""
    m = len(cs)
    tri = np.array(list(itertools.combinations(range(m), 3)))
    A = ns[tri]                       # (T,3,3)
    b = cs[tri]                       # (T,3)
    det = np.linalg.det(A)
    ok = np.abs(det) > 1e-14
    A, b = A[ok], b[ok]
    x = np.linalg.solve(A, b[..., None])[..., 0]
    scale = np.linalg.norm(ns, axis=1)
    feas = np.all(x @ ns.T <= cs + tol * np.maximum(scale, 1e-300), axis=1)
    x = x[feas]
    # merge coincident solutions (degenerate vertices solve several triples)
    verts = []
    for v in x:
        if not any(np.max(np.abs(v - w)) < 1e-10 for w in verts):
            verts.append(v)
    V = np.array(verts)
    tight = np.abs(V @ ns.T - cs) <= 1e-10 * np.maximum(scale, 1e-300)  # (nv, m)
    faces = {}
    vol = 0.0
    mom = np.zeros(3)
    for f in range(m):
        on = np.nonzero(tight[:, f])[0]
        if len(on) < 3:
            continue
        P = V[on]
        cen = P.mean(axis=0)
        nrm = ns[f] / scale[f]
        u = P[0] - cen
        u -= nrm * (u @ nrm)
        u /= np.linalg.norm(u)
        w = np.cross(nrm, u)
        ang = np.arctan2((P - cen) @ w, (P - cen) @ u)
        Q = P[np.argsort(ang)]
        av = 0.5 * np.sum(np.cross(Q - cen, np.roll(Q, -1, axis=0) - cen), axis=0)
        area = float(np.abs(av @ nrm))
        faces[int(ids[f])] = area
        vol += area * (cs[f] / scale[f]) / 3.0
        Q1 = np.roll(Q, -1, axis=0)
        tv = np.einsum("ij,ij->i", np.broadcast_to(cen, Q.shape), np.cross(Q, Q1)) / 6.0  # tets (0, cen, q, q')
        mom += (tv[:, None] * (cen + Q + Q1)).sum(axis=0) / 4.0
    vplanes = [tuple(sorted(int(ids[f]) for f in np.nonzero(tight[k])[0])) for k in range(len(V))]
    if return_moment:
        return V, vplanes, faces, vol, mom
    return V, vplanes, faces, vol


def brute_cells(points: np.ndarray, lo=(0, 0, 0), hi=(1, 1, 1), geometry: bool = False):
    """All cells: (volumes, neighbour sets, vertices per cell as {triple: xyz});
    with ``geometry`` also the neighbour face areas per cell ({j: area}) and
    the centroids [n,3]."""
    points = np.asarray(points, float)
    vols, nbrs, verts, areas, cents = [], [], [], [], []
    for i in range(len(points)):
        ns, cs, ids = halfspaces(points, i, lo, hi)
        V, vp, faces, vol, mom = cell(ns, cs, ids, return_moment=True)
        vols.append(vol)
        nbrs.append(sorted(j for j, a in faces.items() if j >= 0 and a > 1e-14))
        verts.append({t: V[k] + points[i] for k, t in enumerate(vp)})
        areas.append({j: faces[j] for j in nbrs[-1]})
        cents.append(points[i] + mom / vol)
    if geometry:
        return np.array(vols), nbrs, verts, areas, np.array(cents)
    return np.array(vols), nbrs, verts
