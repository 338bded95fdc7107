"""Shared helpers of the GPU parity tests (comparison against the oracle)."""
from __future__ import annotations

import sys

import numpy as np

# Parity bars.  FP64 path: neighbour sets bit-exact, volumes 1e-12 relative
# with a floor of 1e-14 of the mean cell volume (cells orders of magnitude
# smaller than the mean carry rounding from the box-scale start of clipping).
# FP32 path: neighbour sets bit-exact, volumes 1e-5 relative.
VOL_RTOL = {"f64": 1e-12, "f32": 1e-5}
VOL_FLOOR = {"f64": 1e-14, "f32": 0.0}


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


def volume_errors(gpu_vol, orc_vol, prec: str, box_vol: float = 1.0, rows=None):
    g = np.asarray(gpu_vol, dtype=np.float64)
    o = np.asarray(orc_vol, dtype=np.float64)
    if rows is not None:
        g, o = g[rows], o[rows]
    n = len(np.asarray(orc_vol))
    tol = VOL_RTOL[prec] * np.abs(o) + VOL_FLOOR[prec] * box_vol / max(n, 1)
    err = np.abs(g - o)
    rel = err / np.maximum(np.abs(o), 1e-300)
    return err > tol, rel


def vertex_map(vrow_ptr, vxyz, vplanes, i):
    a, b = int(vrow_ptr[i]), int(vrow_ptr[i + 1])
    return {tuple(sorted(int(x) for x in vplanes[k])): np.asarray(vxyz[k]) for k in range(a, b)}


def triple_vertices(P, owner, vplanes, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Each vertex as the meeting point of its three planes, solved by
    Cramer's rule in long double (64-bit mantissa), and the conditioning
    kappa = |n_a| |n_b| |n_c| / |det| of the three plane normals.

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
