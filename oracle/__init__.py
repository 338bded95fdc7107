"""CPU oracle for the cell-by-cell Voronoi method and its learned-k network.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It shares no
code with the HIP path.

* :func:`tessellate` -- exact FP64 cells (volumes, centroids, neighbour
  lists, face areas, vertices) from the C++ file ``voronoi_oracle.cpp``;
* :func:`kneeded`    -- the least neighbour-list size k at which the method
  certifies each cell, and the method's work at a given k;
* :func:`labels`     -- the list-size bucket a cell's k_needed maps to;
* ``oracle.mlp``     -- FP64 forward/backward of the k-bucket network;
* ``oracle.features``-- the network's 12 input features from their definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "voronoi_oracle.cpp")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {1: "bad box", 2: "point outside the box", 3: "duplicate point",
          4: "periodic boxes keep no vertices and clip with the certificate", 5: "image shift out of range"}


def build(force: bool = True) -> str:
    """Compile the oracle (g++, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.orc_tessellate.argtypes = [P, i64, P, P, P, i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(P)]
        lib.orc_tessellate.restype = ctypes.c_int
        lib.orc_nnz.argtypes = [P]
        lib.orc_nnz.restype = i64
        lib.orc_nvert.argtypes = [P]
        lib.orc_nvert.restype = i64
        lib.orc_fetch.argtypes = [P] * 11
        lib.orc_fetch.restype = None
        lib.orc_fetch_vol_ld.argtypes = [P, P]
        lib.orc_fetch_vol_ld.restype = None
        lib.orc_fetch_centroid.argtypes = [P, P]
        lib.orc_fetch_centroid.restype = None
        lib.orc_free.argtypes = [P]
        lib.orc_free.restype = None
        lib.orc_kneeded.argtypes = [P, i64, P, P, P, i64, i64, i64, ctypes.c_int, P, P, P, P, P]
        lib.orc_kneeded.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def _box(lo, hi):
    return np.ascontiguousarray(lo, dtype=np.float64), np.ascontiguousarray(hi, dtype=np.float64)


class OracleError(ValueError):
    pass


def tessellate(points, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), all_planes=False, vertices=False,
               threads=0, cells=None, volume_ld=False, periodic=False) -> dict:
    """Exact cells of every point (rows in input order, neighbours ascending).

    With ``cells`` (indices), only those rows are computed; the other rows are
    empty with volume 0.

    ``all_planes`` clips by every other point (no early stop) -- the check of
    the stopping lemma.  Returns a dict with ``row_ptr, col, area, volume,
    centroid [n,3], work [n,4] (tested, cuts, evals, created), euler`` and,
    with ``vertices``,
    ``vrow_ptr, vxyz [nv,3], vplanes [nv,3], vdeg``.  With ``volume_ld`` also
    ``volume_ld``: each cell's volume in long double from its vertices re-solved
    from their planes (free of the box-scale rounding the primal clip leaves
    in small cells).  With ``periodic`` the box is a 3-torus: every cell is the
    region nearer its generator than any image of any point, neighbours are
    the indices of the points whose images share a face with it (an index
    once per such image; a cell may neighbour images of its own generator
    when there are few points), centroids are not wrapped into the box, and
    points must lie in [lo, hi).
    """
    lib = _load()
    P = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    n = P.shape[0]
    lo_, hi_ = _box(lo, hi)
    h = ctypes.c_void_p()
    flags = (1 if all_planes else 0) | (2 if vertices else 0) | (4 if volume_ld else 0) | (8 if periodic else 0)
    c = None if cells is None else np.ascontiguousarray(cells, dtype=np.int64)
    rc = lib.orc_tessellate(_ptr(P), n, _ptr(lo_), _ptr(hi_), _ptr(c), 0 if c is None else c.shape[0], flags,
                            threads, ctypes.byref(h))
    if rc:
        raise OracleError(ERRORS.get(rc, str(rc)))
    try:
        nnz = lib.orc_nnz(h)
        nv = lib.orc_nvert(h)
        out = dict(row_ptr=np.zeros(n + 1, np.int64), col=np.zeros(nnz, np.int32),
                   area=np.zeros(nnz, np.float64), volume=np.zeros(n, np.float64),
                   work=np.zeros((n, 4), np.int64), euler=np.zeros(n, np.int32),
                   centroid=np.zeros((n, 3), np.float64))
        if vertices:
            out.update(vrow_ptr=np.zeros(n + 1, np.int64), vxyz=np.zeros((nv, 3), np.float64),
                       vplanes=np.zeros((nv, 3), np.int32), vdeg=np.zeros(nv, np.int32))
        g = out.get
        lib.orc_fetch(h, _ptr(out["row_ptr"]), _ptr(out["col"]), _ptr(out["area"]), _ptr(out["volume"]),
                      _ptr(out["work"]), _ptr(out["euler"]), _ptr(g("vrow_ptr")), _ptr(g("vxyz")),
                      _ptr(g("vplanes")), _ptr(g("vdeg")))
        lib.orc_fetch_centroid(h, _ptr(out["centroid"]))
        if volume_ld:
            out["volume_ld"] = np.zeros(n, np.float64)
            lib.orc_fetch_vol_ld(h, _ptr(out["volume_ld"]))
    finally:
        lib.orc_free(h)
    return out


def kneeded(points, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), cells=None, kcap=64, kwork=0, threads=0) -> dict:
    """Least certifying list size per cell (``kcap+1`` = more than kcap).

    With ``kwork > 0`` also returns the method's work at list size ``kwork``:
    planes tested, vertex evaluations, vertices created and vertex norms
    evaluated to update R^2 after cuts (``r2upd``), per cell.
    """
    lib = _load()
    P = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    n = P.shape[0]
    lo_, hi_ = _box(lo, hi)
    c = None if cells is None else np.ascontiguousarray(cells, dtype=np.int64)
    nc = n if c is None else c.shape[0]
    kn = np.zeros(nc, np.int32)
    tested = np.zeros(nc, np.int64)
    evals = np.zeros(nc, np.int64)
    created = np.zeros(nc, np.int64)
    r2upd = np.zeros(nc, np.int64)
    rc = lib.orc_kneeded(_ptr(P), n, _ptr(lo_), _ptr(hi_), _ptr(c), nc, kcap, kwork, threads, _ptr(kn),
                         _ptr(tested), _ptr(evals), _ptr(created), _ptr(r2upd))
    if rc:
        raise OracleError(ERRORS.get(rc, str(rc)))
    return dict(kneeded=kn, tested=tested, evals=evals, created=created, r2upd=r2upd)


BUCKETS = (8, 12, 16, 24, 32, 48, 64)


def labels(kneeded) -> np.ndarray:
    """Training label of each cell (the least list-size bucket that
    certifies it): the first b with BUCKETS[b] >= k_needed, or the largest
    bucket when the cell needs more than the largest bucket."""
    out = []
    for kn in np.asarray(kneeded).tolist():
        b = len(BUCKETS) - 1
        for i, k in enumerate(BUCKETS):
            if k >= kn:
                b = i
                break
        out.append(b)
    return np.array(out, dtype=np.uint8)


def rows(res: dict):
    """Neighbour lists as a list of numpy arrays."""
    rp, col = res["row_ptr"], res["col"]
    return [col[rp[i]:rp[i + 1]] for i in range(len(rp) - 1)]
