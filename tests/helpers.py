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
