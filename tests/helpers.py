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
