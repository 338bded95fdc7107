"""ctypes declarations of the C ABI in include/votess.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvotess.so")

VOTESS_OK = 0
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "EOUTOFBOX", 3: "EDUPLICATE", 4: "ENOMEM", 5: "EHIP", 6: "EUNRESOLVED",
                7: "ECAPACITY"}
F32, F64 = 0, 1
CLIP_F64, CLIP_F32_RECHECK = 0, 1
MAX_PASSES = 8
NPARAM = 5447
NFEAT = 12
NBUCKET = 7


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class Grid(C.Structure):
    _fields_ = [("g", C.c_int32 * 3), ("ncells", C.c_int64), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("inv_h", C.c_double * 3)]


class ClipOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("eps", C.c_double), ("knn_dist", C.c_int), ("max_nbr", C.c_int32),
                ("max_vert", C.c_int32), ("capacity", C.c_int32), ("out_by_id", C.c_int32),
                ("stream", C.c_int32), ("grid", C.c_void_p), ("cell_start", C.c_void_p),
                ("subinfo", C.c_void_p), ("sub_start", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("k0", C.c_int32), ("max_gpu_retries", C.c_int32), ("pts_per_cell", C.c_double),
                ("precision", C.c_int), ("eps", C.c_double), ("kmodel", C.c_void_p), ("tau", C.c_double),
                ("want_vertices", C.c_int32), ("index_space", C.c_int32), ("host_fallback", C.c_int32),
                ("host_threads", C.c_int32), ("force_fail_every", C.c_int32), ("gpu_stream", C.c_int32),
                ("want_faces", C.c_int32), ("periodic", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("npasses", C.c_int32), ("pass_k", C.c_int32 * MAX_PASSES), ("pass_cells", C.c_int64 * MAX_PASSES),
                ("pass_failed", C.c_int64 * MAX_PASSES), ("capacity_cells", C.c_int64),
                ("fallback_cells", C.c_int64), ("unresolved_cells", C.c_int64), ("rechecks", C.c_int64),
                ("refined_cells", C.c_int64), ("streamed_cells", C.c_int64), ("bucket_cells", C.c_int64 * 8),
                ("ms_sort", C.c_double), ("ms_knn", C.c_double), ("ms_clip", C.c_double),
                ("ms_features", C.c_double), ("ms_mlp", C.c_double), ("ms_assemble", C.c_double),
                ("ms_fallback", C.c_double), ("ms_total", C.c_double),
                ("pass_streamed", C.c_int64 * MAX_PASSES)]

    def as_dict(self) -> dict:
        n = self.npasses
        return dict(passes=[dict(k=self.pass_k[i], cells=self.pass_cells[i], failed=self.pass_failed[i],
                                 streamed=self.pass_streamed[i]) for i in range(n)],
                    capacity_cells=self.capacity_cells, fallback_cells=self.fallback_cells,
                    unresolved_cells=self.unresolved_cells, rechecks=self.rechecks,
                    refined_cells=self.refined_cells, streamed_cells=self.streamed_cells, bucket_cells=list(self.bucket_cells)[:NBUCKET],
                    ms_sort=self.ms_sort, ms_knn=self.ms_knn, ms_clip=self.ms_clip, ms_features=self.ms_features,
                    ms_mlp=self.ms_mlp, ms_assemble=self.ms_assemble, ms_fallback=self.ms_fallback,
                    ms_total=self.ms_total)


class Result(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("volume", C.c_void_p), ("nvert", C.c_int64), ("vrow_ptr", C.c_void_p), ("vxyz", C.c_void_p),
                ("vplanes", C.c_void_p), ("area", C.c_void_p), ("centroid", C.c_void_p), ("stats", Stats)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

P = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64

# name -> (restype, argtypes): every entry point declared in include/votess.h
SIGNATURES = {
    "votess_create": (P, [C.c_int]),
    "votess_destroy": (None, [P]),
    "votess_last_error": (C.c_char_p, []),
    "votess_version": (C.c_char_p, []),
    "votess_set_allocator": (None, [P, ALLOC_FN, RELEASE_FN, P]),
    "votess_ctx_errors": (C.c_int, [P, P, C.POINTER(C.c_uint32)]),
    "votess_grid_plan": (C.c_int, [i64, C.POINTER(Box), C.c_double, C.POINTER(Grid)]),
    "votess_grid_sort": (C.c_int, [P, P, C.c_int, i64, C.POINTER(Box), C.POINTER(Grid), P, P, P, P, P, P]),
    "votess_sub_capacity": (i64, [i64]),
    "votess_knn": (C.c_int, [P, P, C.c_int, i64, C.POINTER(Grid), P, P, P, P, i64, i32, C.c_int, P, P]),
    "votess_clip_cells": (C.c_int, [P, P, C.c_int, i64, C.POINTER(Box), P, i64, P, i32, C.POINTER(ClipOpts),
                                    P, P, P, P, P, P, P, P, P, P, P]),
    "votess_params_default": (None, [C.POINTER(Params)]),
    "votess_tessellate": (C.c_int, [P, P, C.c_int, i64, C.POINTER(Box), C.POINTER(Params), C.POINTER(Result), P]),
    "votess_result_free": (None, [P, C.POINTER(Result)]),
    "votess_kmodel_create": (P, [P, C.c_uint64]),
    "votess_kmodel_destroy": (None, [P]),
    "votess_kmodel_set_params": (C.c_int, [P, P, P, P]),
    "votess_kmodel_get_params": (C.c_int, [P, P, P, P]),
    "votess_features": (C.c_int, [P, P, i64, C.POINTER(Grid), P, P, P, P, i64, P, P]),
    "votess_kmodel_forward": (C.c_int, [P, P, i64, P, P]),
    "votess_kmodel_grad": (C.c_int, [P, P, P, i64, P, P, P]),
    "votess_kmodel_train_step": (C.c_int, [P, P, P, i64, C.c_float, P, P]),
    "votess_kmodel_choose": (C.c_int, [P, P, i64, C.c_float, P, P]),
    "votess_features_noalloc_max": (i64, []),
    "votess_features_noalloc": (C.c_int, [P, P, i64, C.POINTER(Grid), P, P, P, P, i64, P, P]),
    "votess_kmodel_labels": (C.c_int, [P, P, P, i64, P, P]),
    "votess_kmodel_fit_norm": (C.c_int, [P, P, i64, P]),
    "votess_kmodel_blob_size": (C.c_size_t, []),
    "votess_kmodel_save": (C.c_int, [P, C.c_double, P, C.c_size_t, C.POINTER(C.c_size_t)]),
    "votess_kmodel_load": (C.c_int, [P, P, C.c_size_t, C.POINTER(P), C.POINTER(C.c_double)]),
}
DATA_SYMBOLS = ["votess_buckets"]

_lib = None


def load():
    """Loads libvotess.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_04514_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class VotessError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int):
    if status != VOTESS_OK:
        raise VotessError(status, load().votess_last_error().decode())
