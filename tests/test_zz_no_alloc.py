"""The allocation-free feature pass (static device scratch) against the
allocating one: the same 12 features bit for bit, on two calls in a row (the
second with fewer queries), no device allocation during the call, and a clear
error above the scratch's size."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2412_04514_amd import gen

pytestmark = pytest.mark.gpu

vt = pytest.importorskip("paper_2412_04514_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _features_noalloc(srt, grid, cs, q, out):
    ctx = vt.Context.get()
    si, ss = vt._sub(grid)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctx.lib.votess_features_noalloc(ctx.handle, C.c_void_p(srt.data_ptr()), srt.shape[0],
                                           C.byref(vt._grid_c(grid)), C.c_void_p(cs.data_ptr()), si, ss,
                                           C.c_void_p(q.data_ptr()), q.shape[0], C.c_void_p(out.data_ptr()), st)


def test_noalloc_features_match_allocating_pass():
    from paper_2412_04514_amd import _lib, kmodel
    P = gen.cluster(300_000, seed=41, dtype=np.float32)
    cs, perm, srt, grid = vt.grid_sort(torch.from_numpy(P).cuda())
    lib = vt.Context.get().lib
    mx = lib.votess_features_noalloc_max()
    assert mx == 65536
    calls = [torch.arange(0, len(P), 4, dtype=torch.int32, device="cuda")[:mx],      # the full scratch
             torch.arange(7, len(P), 301, dtype=torch.int32, device="cuda")]         # then a smaller call
    assert calls[0].shape[0] == mx and calls[1].shape[0] < mx
    for q in calls:
        ref = kmodel.features(srt, grid, cs, q)
        out = torch.empty(q.shape[0], 12, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        _lib.check(_features_noalloc(srt, grid, cs, q, out))
        torch.cuda.synchronize()
        after = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        assert after == before  # nothing allocated through the context's allocator
        assert torch.equal(out, ref)
    too_many = torch.zeros(mx + 1, dtype=torch.int32, device="cuda")
    out = torch.empty(mx + 1, 12, dtype=torch.float32, device="cuda")
    rc = _features_noalloc(srt, grid, cs, too_many, out)
    assert rc == 1  # VOTESS_EINVAL
    assert "exceed the static scratch" in lib.votess_last_error().decode()
