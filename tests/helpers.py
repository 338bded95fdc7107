"""Shared helpers of the GPU parity tests (comparison against the oracle)."""
from __future__ import annotations

import sys

import numpy as np

# Parity bars.  FP64 path: neighbour sets bit-exact, volumes 1e-12 relative
# to the oracle's long-double volume (oracle.tessellate(volume_ld=True): each
# cell's vertices re-solved from their planes in long double; the oracle's
# double volume, interpolated by the primal clip from box-scale vertices, is
# off by up to ~1e-11 on cells far smaller than the box).  FP32 path:
# neighbour sets bit-exact, volumes 1e-5 relative.
VOL_RTOL = {"f64": 1e-12, "f32": 1e-5}


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def csr_rows(row_ptr, col):
    rp = np.asarray(row_ptr)
    c = np.asarray(col)
    return [c[rp[i]:rp[i + 1]] for i in range(len(rp) - 1)]


def compare_rows(gpu_rp, gpu_col, orc, rows=None):
    """Indices of rows whose neighbour lists differ."""
    grp, gcol = np.asarray(gpu_rp), np.asarray(gpu_col)
    orp, ocol = orc["row_ptr"], orc["col"]
    rows = range(len(orp) - 1) if rows is None else rows
    bad = []
    for i in rows:
        if not np.array_equal(gcol[grp[i]:grp[i + 1]], ocol[orp[i]:orp[i + 1]]):
            bad.append(int(i))
    return bad


class VolumeCheck(tuple):
    """(viol, rel), and how many cells the oracle's double volume itself was
    off its long-double volume by more than 1e-12 (``oracle_off``)."""

    def __new__(cls, viol, rel, oracle_off=0):
        t = super().__new__(cls, (viol, rel))
        t.viol, t.rel, t.oracle_off = viol, rel, oracle_off
        return t


def volume_errors(gpu_vol, orc: dict, prec: str, rows=None):
    """Violations of the volume bar and relative errors, against the oracle's
    long-double volume (``orc["volume_ld"]``, required for FP64) or its
    double volume.  ``rows`` selects cells (indices into both arrays)."""
    if prec == "f64" and "volume_ld" not in orc:
        raise ValueError("the FP64 volume bar needs oracle.tessellate(..., volume_ld=True)")
    ref = orc.get("volume_ld", orc["volume"])
    idx = slice(None) if rows is None else np.asarray(rows)
    g = np.asarray(gpu_vol, dtype=np.float64)[idx]
    o = np.asarray(ref, dtype=np.float64)[idx]
    err = np.abs(g - o)
    rel = err / np.maximum(np.abs(o), 1e-300)
    off = 0
    if "volume_ld" in orc:
        od = np.asarray(orc["volume"], dtype=np.float64)[idx]
        off = int((np.abs(od - o) > VOL_RTOL["f64"] * np.abs(o)).sum())
    return VolumeCheck(err > VOL_RTOL[prec] * np.abs(o), rel, off)


def ld_volumes(P, cells, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Volumes of the given cells in long double (64-bit mantissa) from the
    combinatorics the oracle reports, computed independently of its own
    long-double volume: each vertex is re-solved from its three planes
    (triple_vertices), each face is the vertices naming its plane, ordered by
    angle about their mean, and the volume is the sum of the tetrahedra
    (generator, face mean, v_i, v_i+1)."""
    import oracle
    P = np.asarray(P, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.int64)
    o = oracle.tessellate(P, lo, hi, vertices=True, cells=cells)
    out = np.zeros(len(cells), dtype=np.float64)
    for t, i in enumerate(cells):
        a, b = int(o["vrow_ptr"][i]), int(o["vrow_ptr"][i + 1])
        vpl = o["vplanes"][a:b]
        rel, _ = triple_vertices(P, np.full(b - a, i), vpl, lo, hi, relative_ld=True)
        vol = np.longdouble(0)
        for f in np.unique(vpl):
            on = np.nonzero((vpl == f).any(axis=1))[0]
            if len(on) < 3:
                continue
            V = rel[on]
            m = V.mean(axis=0)
            # order by angle about the face mean, in the face's own plane
            nrm = np.cross((V[0] - m).astype(np.float64), (V[1] - m).astype(np.float64))
            if np.linalg.norm(nrm) == 0:
                nrm = np.cross((V[0] - m).astype(np.float64), (V[2] - m).astype(np.float64))
            e1 = (V[0] - m).astype(np.float64)
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(nrm / np.linalg.norm(nrm), e1)
            d = (V - m).astype(np.float64)
            order = np.argsort(np.arctan2(d @ e2, d @ e1))
            V = V[order]
            W = np.roll(V, -1, axis=0)
            det = (m[0] * (V[:, 1] * W[:, 2] - V[:, 2] * W[:, 1]) - m[1] * (V[:, 0] * W[:, 2] - V[:, 2] * W[:, 0])
                   + m[2] * (V[:, 0] * W[:, 1] - V[:, 1] * W[:, 0]))
            vol += np.abs(det.sum()) / 6
        out[t] = float(vol)
    return out


def vertex_map(vrow_ptr, vxyz, vplanes, i):
    a, b = int(vrow_ptr[i]), int(vrow_ptr[i + 1])
    return {tuple(sorted(int(x) for x in vplanes[k])): np.asarray(vxyz[k]) for k in range(a, b)}


def triple_vertices(P, owner, vplanes, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), relative_ld=False):
    """Each vertex as the meeting point of its three planes, solved by
    Cramer's rule in long double (64-bit mantissa), and the conditioning
    kappa = |n_a| |n_b| |n_c| / |det| of the three plane normals.  With
    ``relative_ld`` the vertices are returned in long double, relative to
    their owner's generator.

    Plane ids: q >= 0 is the bisector of the owner and point q (normal
    P[q] - P[i], offset |P[q] - P[i]|^2 / 2 relative to P[i]); -1..-6 are
    the box walls x-, x+, y-, y+, z-, z+."""
    L = np.longdouble
    P = np.asarray(P, dtype=np.float64)
    vplanes = np.asarray(vplanes)
    pi = P[owner].astype(L)
    nv = len(owner)
    n = np.zeros((nv, 3, 3), L)
    r = np.zeros((nv, 3), L)
    lo_, hi_ = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    for c in range(3):
        q = vplanes[:, c]
        nb = q >= 0
        d = P[np.where(nb, q, 0)].astype(L) - pi
        n[nb, c] = d[nb]
        r[nb, c] = (d[nb] ** 2).sum(1) / 2
        w = np.nonzero(~nb)[0]
        ax = (-q[w] - 1) // 2
        wall = np.where((-q[w] - 1) % 2 == 1, hi_[ax], lo_[ax]).astype(L)
        n[w, c, ax] = 1
        r[w, c] = wall - pi[w, ax]

    def det(m):
        a, b, cc = m[:, 0], m[:, 1], m[:, 2]
        return (a[:, 0] * (b[:, 1] * cc[:, 2] - b[:, 2] * cc[:, 1]) - a[:, 1] * (b[:, 0] * cc[:, 2] - b[:, 2] * cc[:, 0])
                + a[:, 2] * (b[:, 0] * cc[:, 1] - b[:, 1] * cc[:, 0]))

    D = det(n)
    y = np.zeros((nv, 3), L)
    with np.errstate(divide="ignore", invalid="ignore"):  # singular triples give inf/nan
        for k in range(3):
            m = n.copy()
            m[:, :, k] = r
            y[:, k] = det(m) / D
        kappa = np.sqrt((n.astype(np.float64) ** 2).sum(2)).prod(1) / np.abs(D.astype(np.float64))
    if relative_ld:
        return y, kappa
    return (y + pi).astype(np.float64), kappa


# Per-face outputs.  Both precisions compute them in double from double
# vertices.  A face area is a sum of corner terms n.(v x (e' - e)) / 2 with
# |v|, |e|, |e'| <= R (R = the cell's farthest vertex from its generator), so
# each term carries an absolute error of order kappa u R^2 (u = 2^-53, kappa
# the conditioning of the vertex); the centroid is a first moment (terms of
# order R^4) over a volume.  The oracle clips from the box, so its vertices
# carry an absolute error of order u times the box size L, and its face areas
# u L R (this dominates for cells far smaller than the box, as in cluster
# cores).  Bars: area within 1e-10 relative, or 1e-12 R^2 + 2e-15 R L;
# centroid within 1e-10 R or 1e-12 R^4 / V.
AREA_RTOL, AREA_FLOOR, AREA_BOX = 1e-10, 1e-12, 2e-15
CEN_RTOL, CEN_FLOOR = 1e-10, 1e-12


def radius_of_cells(P, orc):
    """R^2 of every cell: the largest squared distance from its generator to
    one of its vertices, from the oracle (vertices=True)."""
    n = len(orc["vrow_ptr"]) - 1
    owner = np.repeat(np.arange(n), np.diff(orc["vrow_ptr"]))
    d2 = ((orc["vxyz"] - np.asarray(P, dtype=np.float64)[owner]) ** 2).sum(1)
    r2 = np.zeros(n)
    np.maximum.at(r2, owner, d2)
    return r2


def face_errors(gpu_area, gpu_cen, orc, r2, rows=None, gpu_row_ptr=None, box_size=1.0):
    """(area violations, centroid violations, max area ratio, max centroid
    ratio): ratios are error / bar, for rows (default all) whose neighbour
    lists already match the oracle's (the GPU's row_ptr is needed when the
    oracle computed only ``rows``)."""
    rp = orc["row_ptr"]
    n = len(rp) - 1
    rows = np.arange(n) if rows is None else np.asarray(rows)
    own = np.repeat(np.arange(n), np.diff(rp))
    sel = np.isin(own, rows)
    a_o = orc["area"][sel]
    if gpu_row_ptr is None:
        a_g = np.asarray(gpu_area)[sel]
    else:
        grp = np.asarray(gpu_row_ptr)
        idx = np.concatenate([np.arange(grp[i], grp[i + 1]) for i in rows]) if len(rows) else np.zeros(0, int)
        a_g = np.asarray(gpu_area)[idx]
    bar_a = AREA_RTOL * np.abs(a_o) + AREA_FLOOR * r2[own[sel]] + AREA_BOX * np.sqrt(r2[own[sel]]) * box_size
    ra = np.abs(a_g - a_o) / bar_a
    c_o = orc["centroid"][rows]
    c_g = np.asarray(gpu_cen)[rows]
    R = np.sqrt(r2[rows])
    V = orc["volume"][rows]
    bar_c = CEN_RTOL * R + CEN_FLOOR * r2[rows] ** 2 / V
    rc = np.abs(c_g - c_o).max(axis=1) / bar_c
    return int((ra > 1).sum()), int((rc > 1).sum()), float(ra.max(initial=0)), float(rc.max(initial=0))


def knn_ref_f32(S32, queries, k):
    """k nearest by (d^2, sorted index), d^2 = (dx dx + dy dy) + dz dz in
    float32 with every product and sum rounded on its own (numpy float32
    ufuncs do not fuse)."""
    out = np.full((len(queries), k), -1, np.int64)
    for a in range(0, len(queries), 256):
        q = queries[a:a + 256]
        D = S32[None, :, :] - S32[q, None, :]
        d2 = (D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1]) + D[..., 2] * D[..., 2]
        d2[np.arange(len(q)), q] = np.inf
        idx = np.argsort(d2, axis=1, kind="stable")[:, :k]
        out[a:a + 256] = idx
    return out
