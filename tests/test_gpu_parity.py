"""GPU parity: HIP path (through the C ABI) against the FP64 oracle.

Bars: neighbour sets bit-exact on generic input; volumes within 1e-12
relative (FP64 path; floor 1e-14 of the mean cell volume) or 1e-5 relative
(FP32 path); grid sort bit-exact against a stable argsort; k-NN lists exact
in FP64; certified-cell counts at fixed k equal to the oracle's k_needed
prediction.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import compare_rows, note, vertex_map, volume_errors
from paper_2412_04514_amd import gen

pytestmark = pytest.mark.gpu

vt = pytest.importorskip("paper_2412_04514_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cells_np(P, grid):
    """Grid cell ids from the documented formula (float64 floor, clamped)."""
    P = np.asarray(P, dtype=np.float64)
    g = np.array(list(grid.g))
    lo = np.array(list(grid.lo))
    ih = np.array(list(grid.inv_h))
    c = np.clip(np.floor((P - lo) * ih), 0, g - 1).astype(np.int64)
    return c[:, 0] + g[0] * (c[:, 1] + g[1] * c[:, 2])


# ------------------------------------------------------------------ grid sort

@pytest.mark.parametrize("kind,n,dt", [("uniform", 1 << 20, np.float32), ("cluster", 1 << 20, np.float32),
                                       ("uniform", 10_000, np.float64), ("cluster", 3000, np.float64)])
def test_grid_sort_bit_exact(kind, n, dt):
    note(f"grid_sort {kind} n={n} {dt.__name__}")
    P = getattr(gen, kind)(n, seed=0, dtype=dt)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    cid = _cells_np(P, grid)
    ref_perm = np.argsort(cid, kind="stable")
    ref_cs = np.searchsorted(cid[ref_perm], np.arange(grid.ncells + 1), side="left")
    assert np.array_equal(perm.cpu().numpy(), ref_perm)
    assert np.array_equal(cs.cpu().numpy(), ref_cs)
    s = srt.cpu().numpy()
    assert np.array_equal(s[:, :3], P[ref_perm])
    ib = s[:, 3].view(np.int32 if dt == np.float32 else np.int64)
    assert np.array_equal(ib, ref_perm)


def test_grid_sort_deterministic():
    P = gen.cluster(1 << 19, seed=3, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    a = vt.grid_sort(pts)
    b = vt.grid_sort(pts)
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)


def test_out_of_box_and_nan():
    P = gen.uniform(1000, seed=1, dtype=np.float32)
    P[17] = [0.5, 1.5, 0.5]
    with pytest.raises(vt.VotessError, match="EOUTOFBOX"):
        vt.tessellate(torch.from_numpy(P).cuda())
    P[17] = [0.5, np.nan, 0.5]
    with pytest.raises(vt.VotessError, match="EOUTOFBOX"):
        vt.tessellate(torch.from_numpy(P).cuda())


def test_duplicate_point():
    P = gen.uniform(1000, seed=2, dtype=np.float64)
    P[5] = P[700]
    with pytest.raises(vt.VotessError, match="EDUPLICATE"):
        vt.tessellate(torch.from_numpy(P).cuda())


# ------------------------------------------------------------------------ kNN

def _knn_ref(S, queries, k, dist):
    """Exact k nearest by (d^2, sorted index) with d^2 in float64."""
    out = np.full((len(queries), k), -1, np.int64)
    X = S.astype(np.float64)
    for a in range(0, len(queries), 256):
        q = queries[a:a + 256]
        d2 = ((X[None, :, :] - X[q, None, :]) ** 2).sum(-1)
        d2[np.arange(len(q)), q] = np.inf
        idx = np.argsort(d2, axis=1, kind="stable")[:, :k]  # stable: ties by sorted index
        m = np.take_along_axis(d2, idx, 1)
        idx[~np.isfinite(m)] = -1
        out[a:a + 256] = idx
    return out


@pytest.mark.parametrize("kind,dt", [("uniform", np.float64), ("cluster", np.float32), ("filament", np.float32)])
@pytest.mark.parametrize("k", [8, 24, 64])
def test_knn_f64_exact(kind, dt, k):
    note(f"knn f64 {kind} k={k}")
    P = getattr(gen, kind)(20_000, seed=4, dtype=dt)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    S = srt[:, :3].cpu().numpy()
    rng = np.random.default_rng(0)
    q = np.sort(rng.choice(len(P), 1500, replace=False)).astype(np.int32)
    got = vt.knn(srt, grid, cs, k, queries=torch.from_numpy(q).cuda(), dist="f64").cpu().numpy()
    ref = _knn_ref(S, q, k, "f64")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("kind", ["uniform", "cluster"])
def test_knn_f32_lists(kind):
    """Float distances: the list is the k nearest up to float rounding of d^2."""
    P = getattr(gen, kind)(20_000, seed=5, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    S = srt[:, :3].cpu().numpy().astype(np.float64)
    k = 32
    got = vt.knn(srt, grid, cs, k, dist="f32").cpu().numpy()
    q = np.arange(0, len(P), 13)
    ref = _knn_ref(S, q, k, "f64")
    for r, i in enumerate(q):
        g = got[i]
        d_ref = ((S[ref[r]] - S[i]) ** 2).sum(1)
        d_got = ((S[g] - S[i]) ** 2).sum(1)
        kth = d_ref[-1]
        assert np.all(g >= 0)
        # every returned point is within float rounding of the true k-th distance,
        # every true neighbour clearly inside it is returned, order is ascending
        assert np.all(d_got <= kth * (1 + 4e-7))
        must = set(ref[r][d_ref < kth * (1 - 4e-7)].tolist())
        assert must <= set(g.tolist())
        assert np.all(np.diff(d_got) >= -4e-7 * kth)


def test_knn_padding_and_small_n():
    P = gen.uniform(5, seed=6, dtype=np.float64)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    got = vt.knn(srt, grid, cs, 8).cpu().numpy()
    assert np.all(got[:, 4:] == -1) and np.all(got[:, :4] >= 0)
    for i in range(5):
        assert sorted(got[i, :4].tolist()) == [j for j in range(5) if j != i]


# ------------------------------------------------------------- tessellation

CASES = [
    # name, generator, n, dtype, kwargs
    ("uniform-10k-f64-k16-retry32", "uniform", 10_000, np.float64, dict(k0=16, max_gpu_retries=1)),
    ("uniform-200k-f32-f64clip", "uniform", 200_000, np.float32, dict(k0=32, max_gpu_retries=1)),
    ("uniform-200k-f32-f32clip", "uniform", 200_000, np.float32, dict(k0=32, max_gpu_retries=1, precision="f32")),
    ("cluster-200k-f64clip", "cluster", 200_000, np.float32, dict(k0=32, max_gpu_retries=1)),
    ("cluster-200k-f32clip", "cluster", 200_000, np.float32, dict(k0=32, max_gpu_retries=1, precision="f32")),
    ("filament-200k-f32clip", "filament", 200_000, np.float32, dict(k0=64, max_gpu_retries=0, precision="f32")),
    ("cluster-50k-f64-k64", "cluster", 50_000, np.float64, dict(k0=64, max_gpu_retries=0)),
    ("cluster-200k-f64-nostream", "cluster", 200_000, np.float32, dict(k0=32, max_gpu_retries=1, gpu_stream=False)),
    ("uniform-10k-f64-k8-stream", "uniform", 10_000, np.float64, dict(k0=8, max_gpu_retries=0)),
    ("filament-200k-f32-k16-stream", "filament", 200_000, np.float32, dict(k0=16, max_gpu_retries=0,
                                                                          precision="f32")),
]


@pytest.mark.parametrize("name,kind,n,dt,kw", CASES, ids=[c[0] for c in CASES])
def test_tessellate_parity(name, kind, n, dt, kw):
    note(f"tessellate {name}")
    P = getattr(gen, kind)(n, seed=0, dtype=dt)
    res = vt.tessellate(torch.from_numpy(P).cuda(), **kw)
    torch.cuda.synchronize()
    orc = oracle.tessellate(P.astype(np.float64))
    prec = kw.get("precision", "f64")
    bad = compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    assert not bad, f"{len(bad)} rows differ, e.g. {bad[:5]}"
    viol, rel = volume_errors(res.volume.cpu().numpy(), orc["volume"], prec)
    note(f"  {name}: max rel vol err {rel.max():.3e}  stats {res.stats}")
    assert not viol.any(), f"{viol.sum()} volumes out of tolerance, max rel {rel.max():.3e}"
    assert abs(res.volume.sum().item() - 1.0) < (1e-12 if prec == "f64" else 1e-6)


def test_anisotropic_box_and_boundary_points():
    lo, hi = (-0.5, 0.0, 2.0), (1.5, 0.25, 3.0)
    rng = np.random.default_rng(7)
    P = np.array(lo) + rng.random((5000, 3)) * (np.array(hi) - np.array(lo))
    P[:4] = [lo, hi, (lo[0], hi[1], lo[2]), (0.1, 0.1, 2.5)]
    P[4] = (hi[0], 0.125, 2.5)  # on a face
    res = vt.tessellate(torch.from_numpy(P).cuda(), box=(lo, hi), k0=32)
    orc = oracle.tessellate(P, lo, hi)
    assert not compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    viol, _ = volume_errors(res.volume.cpu().numpy(), orc["volume"], "f64", box_vol=2 * 0.25 * 1.0)
    assert not viol.any()


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7])
def test_tiny_inputs(n):
    P = gen.uniform(n, seed=8, dtype=np.float64) if n else np.zeros((0, 3))
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=8)
    assert res.row_ptr.shape[0] == n + 1
    if n == 0:
        return
    orc = oracle.tessellate(P)
    assert not compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    np.testing.assert_allclose(res.volume.cpu().numpy(), orc["volume"], rtol=1e-12)
    assert res.stats["fallback_cells"] == 0  # lists shorter than k hold every other point


def test_octant_centres_closed_form():
    P = np.array([[0.25 + 0.5 * ((i >> a) & 1) for a in range(3)] for i in range(8)])
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=8)
    np.testing.assert_allclose(res.volume.cpu().numpy(), 0.125, rtol=1e-14)


def test_bcc_lattice_volumes():
    """Degenerate input (many co-spherical points): volumes still exact."""
    m = 8
    g = (np.arange(m) + 0.5) / m
    sc = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    h = np.arange(1, m) / m
    bc = np.stack(np.meshgrid(h, h, h, indexing="ij"), -1).reshape(-1, 3)
    P = np.concatenate([sc, bc])
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=32)
    orc = oracle.tessellate(P)
    np.testing.assert_allclose(res.volume.cpu().numpy(), orc["volume"], rtol=1e-12, atol=1e-17)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["uniform", "cluster"])
def test_status_counts_match_kneeded(kind, prec):
    """Certified counts at fixed k = #{k_needed <= k} of the oracle (the method's own labels)."""
    P = getattr(gen, kind)(50_000, seed=9, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    pn = perm.cpu().numpy()
    kn_ref = oracle.kneeded(P.astype(np.float64), kcap=64)["kneeded"][pn]
    for k in (16, 32, 64):
        lists = vt.knn(srt, grid, cs, k, dist=prec)
        r = vt.clip_cells(srt, lists, k, precision=prec)
        st = r["status"].cpu().numpy()
        cap = np.nonzero(st == 2)[0]
        if len(cap):  # overflow of the fast kernel: same lists in the large-capacity kernel
            rc = vt.clip_cells(srt, lists[torch.from_numpy(cap).cuda()].contiguous(), k, precision=prec,
                               cells=torch.from_numpy(cap.astype(np.int32)).cuda(), capacity=1)
            st[cap] = rc["status"].cpu().numpy()
            kn_all = r["kneeded"].clone()
            kn_all[torch.from_numpy(cap).cuda()] = rc["kneeded"]
            r["kneeded"] = kn_all
        cert = st == 0
        pred = kn_ref <= k
        note(f"  {kind} {prec} k={k}: certified {cert.sum()} predicted {pred.sum()} other statuses "
             f"{np.bincount(st, minlength=4).tolist()}")
        if prec == "f64":
            assert np.array_equal(cert, pred)
            assert np.array_equal(r["kneeded"].cpu().numpy()[cert], kn_ref[cert])
        else:
            # float lists certify with a slack of 8 ulp on d^2: only near-ties may differ
            assert np.sum(cert != pred) <= max(3, 1e-4 * len(P))
            assert not np.any(cert & ~pred & (st == 0) & (kn_ref > k + 1))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_vertices_parity(prec):
    P = gen.cluster(20_000, seed=10, dtype=np.float32, n_clusters=64)
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=64, precision=prec, vertices=True)
    orc = oracle.tessellate(P.astype(np.float64), vertices=True)
    vrp = res.vrow_ptr.cpu().numpy()
    vx = res.vxyz.cpu().numpy()
    vp = res.vplanes.cpu().numpy()
    errs = []
    for i in range(0, len(P), 7):
        g = vertex_map(vrp, vx, vp, i)
        o = vertex_map(orc["vrow_ptr"], orc["vxyz"], orc["vplanes"], i)
        assert set(g) == set(o), i
        R = max(np.abs(x - P[i]).max() for x in o.values())
        # absolute coordinates round at ulp(1) ~ 1e-16 whatever the cell size
        floor = 1e-15 if prec == "f64" else 1e-7
        errs += [np.abs(x - o[key]).max() / (R + floor / 1e-12) for key, x in g.items()]
    errs = np.array(errs)
    p50, p99, worst = np.percentile(errs, 50), np.percentile(errs, 99), errs.max()
    note(f"  vertices {prec}: error / R  p50 {p50:.2e}  p99 {p99:.2e}  max {worst:.2e}")
    # The oracle interpolates along edges, the kernel solves each vertex from its
    # three planes: they agree to rounding amplified by the vertex's conditioning.
    if prec == "f64":
        assert p99 <= 1e-13 and worst <= 1e-10
    else:
        assert p99 <= 1e-6 and worst <= 1e-5


def test_host_fallback_forced():
    P = gen.uniform(20_000, seed=11, dtype=np.float32)
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=32, force_fail_every=3)
    assert res.stats["fallback_cells"] >= len(P) // 3
    orc = oracle.tessellate(P.astype(np.float64))
    assert not compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    viol, _ = volume_errors(res.volume.cpu().numpy(), orc["volume"], "f64")
    assert not viol.any()


def test_no_fallback_raises():
    P = gen.uniform(5000, seed=12, dtype=np.float32)
    with pytest.raises(vt.VotessError, match="EUNRESOLVED"):
        vt.tessellate(torch.from_numpy(P).cuda(), k0=8, max_gpu_retries=0, host_fallback=False, gpu_stream=False)


def test_sorted_index_space():
    P = gen.uniform(30_000, seed=13, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    a = vt.tessellate(pts, k0=64, max_gpu_retries=0)
    b = vt.tessellate(pts, k0=64, max_gpu_retries=0, index_space="sorted")
    _, perm, _, _ = vt.grid_sort(pts)
    pn = perm.cpu().numpy()
    inv = np.empty_like(pn)
    inv[pn] = np.arange(len(pn))
    ra, ca = a.row_ptr.cpu().numpy(), a.col.cpu().numpy()
    rb, cb = b.row_ptr.cpu().numpy(), b.col.cpu().numpy()
    for s in range(0, len(P), 17):
        i = pn[s]
        assert np.array_equal(np.sort(inv[ca[ra[i]:ra[i + 1]]]), cb[rb[s]:rb[s + 1]])
    assert np.array_equal(a.volume.cpu().numpy()[pn], b.volume.cpu().numpy())


def test_tessellate_deterministic():
    P = gen.cluster(100_000, seed=14, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    a = vt.tessellate(pts, k0=32, precision="f32")
    b = vt.tessellate(pts, k0=32, precision="f32")
    assert torch.equal(a.row_ptr, b.row_ptr) and torch.equal(a.col, b.col)
    assert torch.equal(a.volume, b.volume)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_clip_stream_phase(prec):
    """Lists of 8 certify almost nothing; the stream phase finishes every cell on the GPU."""
    P = gen.cluster(100_000, seed=15, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    lists = vt.knn(srt, grid, cs, 8, dist=prec)
    r = vt.clip_cells(srt, lists, 8, precision=prec, stream=True, grid=grid, cell_start=cs)
    st = r["status"].cpu().numpy()
    note(f"  stream {prec}: statuses {np.bincount(st, minlength=4).tolist()}")
    assert (st == 0).mean() > 0.999
    pn = perm.cpu().numpy()
    orc = oracle.tessellate(P.astype(np.float64))
    ok = np.nonzero(st == 0)[0]
    vol = r["volume"].cpu().numpy()
    viol, rel = volume_errors(vol[ok], orc["volume"][pn[ok]], prec)
    assert not viol.any(), rel.max()
    cnt = r["nbr_count"].cpu().numpy()
    nbr = r["nbr"].cpu().numpy()
    for s in ok[::5]:
        i = pn[s]
        got = np.sort(pn[nbr[s, :cnt[s]]])
        assert np.array_equal(got, orc["col"][orc["row_ptr"][i]:orc["row_ptr"][i + 1]])
