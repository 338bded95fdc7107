"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates arguments on the host."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2412_04514_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "votess.h")


def _declared():
    text = open(HEADER).read()
    funcs = re.findall(r"VOTESS_API\s+[\w\s\*]+?\b(votess_\w+)\s*\(", text)
    data = re.findall(r"extern VOTESS_API const \w+ (votess_\w+)\[", text)
    return sorted(set(funcs)), sorted(set(data))


def test_header_and_binding_agree():
    funcs, data = _declared()
    assert len(funcs) >= 20
    assert sorted(_lib.SIGNATURES) == funcs
    assert _lib.DATA_SYMBOLS == data


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    funcs, data = _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in funcs + data:
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_no_oracle_linkage():
    """The product library neither links nor names the oracle."""
    blob = open(_lib.LIB_PATH, "rb").read()
    assert b"liboracle" not in blob and b"orc_tessellate" not in blob


def test_version_and_buckets():
    lib = _lib.load()
    assert lib.votess_version().decode().count(".") == 2
    b = (C.c_int32 * 7).in_dll(lib, "votess_buckets")
    assert list(b) == [8, 12, 16, 24, 32, 48, 64]


def test_grid_plan_sizes():
    lib = _lib.load()
    box = _lib.Box((0, 0, 0), (1, 1, 1))
    for n, g in [(10_000, 17), (1 << 20, 81), (1 << 22, 128), (1 << 24, 203), (1 << 26, 323)]:
        grid = _lib.Grid()
        assert lib.votess_grid_plan(n, C.byref(box), 2.0, C.byref(grid)) == 0
        assert list(grid.g) == [g, g, g]
        assert grid.ncells == g ** 3
    aniso = _lib.Box((0, 0, 0), (4, 1, 1))
    grid = _lib.Grid()
    assert lib.votess_grid_plan(4000, C.byref(aniso), 2.0, C.byref(grid)) == 0
    assert grid.g[0] == 4 * grid.g[1]


def test_host_side_validation():
    lib = _lib.load()
    bad = _lib.Box((0, 0, 0), (1, 0, 1))
    grid = _lib.Grid()
    assert lib.votess_grid_plan(10, C.byref(bad), 2.0, C.byref(grid)) == 1
    assert b"box" in lib.votess_last_error()
    ok = _lib.Box((0, 0, 0), (1, 1, 1))
    assert lib.votess_grid_plan(-1, C.byref(ok), 2.0, C.byref(grid)) == 1
    assert lib.votess_grid_sort(None, None, 0, 10, C.byref(ok), C.byref(grid), None, None, None, None, None, None) == 1
    assert lib.votess_knn(None, None, 0, 10, C.byref(grid), None, None, None, None, 10, 32, 0, None, None) == 1
    opts = _lib.ClipOpts()
    assert lib.votess_clip_cells(None, None, 0, 10, C.byref(ok), None, 10, None, 32, C.byref(opts),
                                 *([None] * 11)) == 1
    r = _lib.Result()
    assert lib.votess_tessellate(None, None, 0, 10, C.byref(ok), None, C.byref(r), None) == 1


def test_params_default():
    lib = _lib.load()
    p = _lib.Params()
    lib.votess_params_default(C.byref(p))
    assert p.k0 == 32 and p.max_gpu_retries == 1 and p.pts_per_cell == 2.0 and p.host_fallback == 1
    assert p.want_faces == 0 and p.gpu_stream == 1
    assert abs(p.eps - 1e-6) < 1e-18


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_create_without_gpu_fails_cleanly():
    lib = _lib.load()
    assert not lib.votess_create(0)
    assert lib.votess_last_error()
