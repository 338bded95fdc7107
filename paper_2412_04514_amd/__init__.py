"""Cell-by-cell 3D Voronoi tessellation on MI355X (gfx950).

Thin Python binding over the C ABI of ``libvotess.so`` (include/votess.h).
Every step of the method runs in the library's HIP kernels (and its host
fallback for uncertified cells); this module only marshals arguments.  PyTorch
provides device memory (the library allocates through torch's caching
allocator) and the current HIP stream.

    import torch, paper_2412_04514_amd as vt
    pts = torch.rand(1 << 20, 3, device="cuda")
    res = vt.tessellate(pts, k0=32)          # CSR neighbours + volumes
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import CLIP_F32_RECHECK, CLIP_F64, F32, F64, VotessError, check

__all__ = ["Context", "Result", "tessellate", "grid_plan", "grid_sort", "knn", "clip_cells", "VotessError",
           "BUCKETS", "CELL_CERTIFIED", "CELL_RADIUS", "CELL_CAPACITY", "CELL_UNRESOLVED"]

BUCKETS = (8, 12, 16, 24, 32, 48, 64)
CELL_CERTIFIED, CELL_RADIUS, CELL_CAPACITY, CELL_UNRESOLVED = 0, 1, 2, 3
_PREC = {"f64": CLIP_F64, "f32": CLIP_F32_RECHECK, "f32_recheck": CLIP_F32_RECHECK}


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"points must be float32 or float64, got {t.dtype}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _box(box) -> _lib.Box:
    lo, hi = box
    b = _lib.Box()
    for a in range(3):
        b.lo[a] = float(lo[a])
        b.hi[a] = float(hi[a])
    return b


class Context:
    """A library context on one device whose device memory comes from torch."""

    _default = {}

    def __init__(self, device: int | None = None):
        self.lib = _lib.load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._live: dict[int, torch.Tensor] = {}
        h = self.lib.votess_create(self.device)
        if not h:
            raise VotessError(5, self.lib.votess_last_error().decode())
        self.handle = C.c_void_p(h)

        def _alloc(nbytes, _user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{self.device}")
            p = t.data_ptr()
            self._live[p] = t
            return p

        def _release(p, _user):
            self._live.pop(int(p or 0), None)

        self._alloc_cb = _lib.ALLOC_FN(_alloc)
        self._release_cb = _lib.RELEASE_FN(_release)
        self.lib.votess_set_allocator(self.handle, self._alloc_cb, self._release_cb, None)

    @classmethod
    def get(cls, device: int | None = None) -> "Context":
        d = torch.cuda.current_device() if device is None else int(device)
        if d not in cls._default:
            cls._default[d] = Context(d)
        return cls._default[d]

    def take(self, ptr: int, dtype: torch.dtype, shape) -> torch.Tensor:
        """Adopts a buffer the library allocated through this context."""
        raw = self._live.pop(int(ptr))
        n = 1
        for s in shape:
            n *= s
        return raw[: n * torch.empty((), dtype=dtype).element_size()].view(dtype).view(*shape)

    def errors(self) -> int:
        e = C.c_uint32(0)
        check(self.lib.votess_ctx_errors(self.handle, _stream(), C.byref(e)))
        return e.value

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.lib.votess_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


# --------------------------------------------------------------- low level

def grid_plan(n: int, box=((0, 0, 0), (1, 1, 1)), pts_per_cell: float = 2.0) -> _lib.Grid:
    g = _lib.Grid()
    b = _box(box)
    check(_lib.load().votess_grid_plan(int(n), C.byref(b), float(pts_per_cell), C.byref(g)))
    return g


class GridIndex:
    """The grid of a sort (``.c``: the C struct) and its dense-cell sub-grids."""

    def __init__(self, c: _lib.Grid, subinfo=None, sub_start=None):
        self.c = c
        self.subinfo = subinfo
        self.sub_start = sub_start

    g = property(lambda self: self.c.g)
    lo = property(lambda self: self.c.lo)
    hi = property(lambda self: self.c.hi)
    inv_h = property(lambda self: self.c.inv_h)
    ncells = property(lambda self: self.c.ncells)


def _grid_c(grid):
    return grid.c if isinstance(grid, GridIndex) else grid


def _sub(grid):
    if isinstance(grid, GridIndex) and grid.subinfo is not None:
        return _ptr(grid.subinfo), _ptr(grid.sub_start)
    return None, None


def grid_sort(points: torch.Tensor, box=((0, 0, 0), (1, 1, 1)), grid: _lib.Grid | None = None,
              pts_per_cell: float = 2.0, subgrids: bool = True, ctx: Context | None = None):
    """Counting sort into the grid: returns (cell_start, perm, sorted[n,4], GridIndex)."""
    ctx = ctx or Context.get()
    pts = points.contiguous()
    n = pts.shape[0]
    grid = grid or grid_plan(n, box, pts_per_cell)
    dev = pts.device
    cell_start = torch.empty(grid.ncells + 1, dtype=torch.int32, device=dev)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    sorted_ = torch.empty(max(n, 1), 4, dtype=pts.dtype, device=dev)
    subinfo = sub_start = None
    if subgrids:
        subinfo = torch.empty(2 * grid.ncells, dtype=torch.int32, device=dev)
        sub_start = torch.empty(ctx.lib.votess_sub_capacity(n), dtype=torch.int32, device=dev)
    b = _box(box)
    check(ctx.lib.votess_grid_sort(ctx.handle, _ptr(pts), _dtype_code(pts), n, C.byref(b), C.byref(grid),
                                   _ptr(cell_start), _ptr(perm), _ptr(sorted_), _ptr(subinfo), _ptr(sub_start),
                                   _stream()))
    return cell_start, perm[:n], sorted_[:n], GridIndex(grid, subinfo, sub_start)


def knn(sorted_: torch.Tensor, grid: _lib.Grid, cell_start: torch.Tensor, k: int, queries=None,
        dist: str = "f64", ctx: Context | None = None) -> torch.Tensor:
    """k nearest other points (sorted indices, ascending distance, -1 padded)."""
    ctx = ctx or Context.get()
    n = sorted_.shape[0]
    nq = n if queries is None else queries.shape[0]
    out = torch.empty(max(nq, 1), k, dtype=torch.int32, device=sorted_.device)
    si, ss = _sub(grid)
    check(ctx.lib.votess_knn(ctx.handle, _ptr(sorted_), _dtype_code(sorted_), n, C.byref(_grid_c(grid)),
                             _ptr(cell_start), si, ss, _ptr(queries), nq, int(k), F32 if dist == "f32" else F64,
                             _ptr(out), _stream()))
    return out[:nq]


def clip_cells(sorted_: torch.Tensor, knn_: torch.Tensor, k: int, box=((0, 0, 0), (1, 1, 1)), cells=None,
               precision: str = "f64", eps: float = 1e-6, knn_dist: str | None = None, max_nbr: int = 64,
               max_vert: int = 0, capacity: int = 0, kneeded: bool = True, stream: bool = False, grid=None,
               cell_start=None, faces: bool = False, ctx: Context | None = None) -> dict:
    """Clips each cell by its k-list; per-cell status, neighbours, volume.

    With ``stream`` (needs ``grid`` and ``cell_start``), a cell its list does
    not certify keeps clipping by grid rings until certified.  With ``faces``,
    also ``area`` [rows, max_nbr] (next to ``nbr``) and ``centroid`` [rows, 3]."""
    ctx = ctx or Context.get()
    n = sorted_.shape[0]
    nc = n if cells is None else cells.shape[0]
    dev = sorted_.device
    rows = max(nc, 1)
    out = dict(status=torch.empty(rows, dtype=torch.uint8, device=dev),
               nbr_count=torch.empty(rows, dtype=torch.int32, device=dev),
               nbr=torch.empty(rows, max_nbr, dtype=torch.int32, device=dev),
               volume=torch.empty(rows, dtype=torch.float64, device=dev))
    if kneeded:
        out["kneeded"] = torch.empty(rows, dtype=torch.int32, device=dev)
    if max_vert > 0:
        out["vcount"] = torch.empty(rows, dtype=torch.int32, device=dev)
        out["verts"] = torch.empty(rows, max_vert, 3, dtype=torch.float64, device=dev)
        out["vplanes"] = torch.empty(rows, max_vert, 3, dtype=torch.int32, device=dev)
    if faces:
        out["area"] = torch.empty(rows, max_nbr, dtype=torch.float64, device=dev)
        out["centroid"] = torch.empty(rows, 3, dtype=torch.float64, device=dev)
    o = _lib.ClipOpts()
    o.precision = _PREC[precision]
    o.eps = eps
    o.knn_dist = (F32 if precision != "f64" else F64) if knn_dist is None else (F32 if knn_dist == "f32" else F64)
    o.max_nbr = max_nbr
    o.max_vert = max_vert
    o.capacity = capacity
    o.out_by_id = 0
    o.stream = int(bool(stream))
    if stream:
        gc = _grid_c(grid)
        o.grid = C.cast(C.pointer(gc), C.c_void_p)
        o.cell_start = cell_start.data_ptr()
        si, ss = _sub(grid)
        o.subinfo = si.value if si is not None else None
        o.sub_start = ss.value if ss is not None else None
    b = _box(box)
    check(ctx.lib.votess_clip_cells(ctx.handle, _ptr(sorted_), _dtype_code(sorted_), n, C.byref(b), _ptr(cells), nc,
                                    _ptr(knn_), int(k), C.byref(o), _ptr(out["status"]), _ptr(out["nbr_count"]),
                                    _ptr(out["nbr"]), _ptr(out["volume"]), _ptr(out.get("kneeded")),
                                    _ptr(out.get("vcount")), _ptr(out.get("verts")), _ptr(out.get("vplanes")),
                                    _ptr(out.get("area")), _ptr(out.get("centroid")), _stream()))
    return {key: v[:nc] for key, v in out.items()}


# -------------------------------------------------------------- one call

@dataclass
class Result:
    row_ptr: torch.Tensor          # [n+1] int64
    col: torch.Tensor              # [nnz] int32, each row ascending
    volume: torch.Tensor           # [n] float64
    vrow_ptr: torch.Tensor | None = None
    vxyz: torch.Tensor | None = None
    vplanes: torch.Tensor | None = None
    area: torch.Tensor | None = None      # [nnz] float64: face shared with col[e] (faces=True)
    centroid: torch.Tensor | None = None  # [n,3] float64 (faces=True)
    stats: dict = field(default_factory=dict)

    def neighbours(self, i: int) -> torch.Tensor:
        return self.col[self.row_ptr[i]:self.row_ptr[i + 1]]


def tessellate(points: torch.Tensor, box=((0, 0, 0), (1, 1, 1)), k0: int = 32, max_gpu_retries: int = 1,
               precision: str = "f64", eps: float = 1e-6, pts_per_cell: float = 2.0, kmodel=None, tau: float = 0.9,
               vertices: bool = False, index_space: str = "original", host_fallback: bool = True,
               host_threads: int = 0, force_fail_every: int = 0, gpu_stream: bool = True, faces: bool = False,
               periodic: bool = False, ctx: Context | None = None) -> Result:
    """Voronoi cells of ``points`` [n,3] (cuda, float32/float64) clipped to ``box``.

    With ``faces``, also the area of every neighbour's face (``area``, next to
    ``col``) and the cell centroids (``centroid``).  With ``periodic`` the box
    is a 3-torus (points in [lo, hi)): rows list the index of every point whose
    image shares a face with the cell, once per image."""
    ctx = ctx or Context.get(points.device.index)
    pts = points.contiguous()
    p = _lib.Params()
    ctx.lib.votess_params_default(C.byref(p))
    p.k0 = k0
    p.max_gpu_retries = max_gpu_retries
    p.pts_per_cell = pts_per_cell
    p.precision = _PREC[precision]
    p.eps = eps
    p.kmodel = None if kmodel is None else kmodel.handle
    p.tau = tau
    p.want_vertices = int(bool(vertices))
    p.index_space = 1 if index_space == "sorted" else 0
    p.host_fallback = int(bool(host_fallback))
    p.host_threads = host_threads
    p.force_fail_every = force_fail_every
    p.gpu_stream = int(bool(gpu_stream))
    p.want_faces = int(bool(faces))
    p.periodic = int(bool(periodic))
    r = _lib.Result()
    b = _box(box)
    n = pts.shape[0]
    check(ctx.lib.votess_tessellate(ctx.handle, _ptr(pts), _dtype_code(pts), n, C.byref(b), C.byref(p), C.byref(r),
                                    _stream()))
    out = Result(row_ptr=ctx.take(r.row_ptr, torch.int64, (n + 1,)),
                 col=ctx.take(r.col, torch.int32, (max(r.nnz, 1),))[: r.nnz],
                 volume=ctx.take(r.volume, torch.float64, (max(n, 1),))[:n],
                 stats=r.stats.as_dict())
    if vertices:
        out.vrow_ptr = ctx.take(r.vrow_ptr, torch.int64, (n + 1,))
        out.vxyz = ctx.take(r.vxyz, torch.float64, (max(r.nvert, 1), 3))[: r.nvert]
        out.vplanes = ctx.take(r.vplanes, torch.int32, (max(r.nvert, 1), 3))[: r.nvert]
    if faces:
        out.area = ctx.take(r.area, torch.float64, (max(r.nnz, 1),))[: r.nnz]
        out.centroid = ctx.take(r.centroid, torch.float64, (max(n, 1), 3))[:n]
    return out
