"""GPU parity: HIP path (through the C ABI) against the FP64 oracle.

Bars: neighbour sets bit-exact on generic input; volumes within 1e-12
relative (FP64 path; a cell beyond it is arbitrated by its volume recomputed
in long double from the oracle's vertex plane triples, and the GPU must be
within 1e-12 of that) or 1e-5 relative (FP32 path); FP32 vertices within
1e-5 R; grid sort bit-exact against a stable argsort; k-NN lists exact
in FP64; certified-cell counts at fixed k equal to the oracle's k_needed
prediction.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import triple_vertices, compare_rows, note, vertex_map, volume_errors, knn_ref_f32
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


def _sub_records(P, grid, cid, sub_start, subinfo):
    """Sub-cell id of every point from its cell's sub-grid record (m0, m1,
    m2, lo[3], ih[3]), after checking the record against the documented
    rule: m_a >= 1, m0 m1 m2 <= count / 2, and the box [lo, lo + m / ih]
    holds the central 90% of the cell's points per axis (up to one of the
    1024 histogram bins over their bounding box)."""
    P = np.asarray(P, dtype=np.float64)
    info = subinfo.reshape(-1, 2)
    cnt = np.bincount(cid, minlength=len(info))
    dense = np.nonzero(cnt > 16)[0]
    assert np.array_equal(np.nonzero(info[:, 0] >= 0)[0], dense)
    sid = np.zeros(len(P), np.int64)
    order = np.argsort(cid, kind="stable")
    starts = np.searchsorted(cid[order], np.arange(len(info) + 1))
    recs = {}
    for c in dense:
        off = info[c, 0]
        assert off % 4 == 0
        rec = sub_start[off:off + 16]
        m = rec[:3].astype(np.int64)
        lo = rec[4:10].copy().view(np.float64)
        ih = rec[10:16].copy().view(np.float64)
        assert info[c, 1] == m.prod() and np.all(m >= 1) and m.prod() <= cnt[c] // 2
        pts = P[order[starts[c]:starts[c + 1]]]
        bw = (pts.max(0) - pts.min(0)) / 1024 * (1 + 1e-9) + 1e-300
        inside = (pts >= lo - bw) & (pts <= lo + m / ih + bw)
        assert np.all(inside.sum(0) >= len(pts) - 2 * (len(pts) // 20)), (c, inside.sum(0), len(pts))
        s = np.clip(np.floor((pts - lo) * ih), 0, m - 1).astype(np.int64)
        sid[order[starts[c]:starts[c + 1]]] = s[:, 0] + m[0] * (s[:, 1] + m[1] * s[:, 2])
        recs[c] = (off, int(m.prod()))
    return sid, recs


# ------------------------------------------------------------------ grid sort

def _one_giant_cell(n, crowded, seed=0):
    """n/3 uniform points plus 2n/3 in a Gaussian (sigma 1e-4) inside one grid
    cell, so that the cell holds far more than 8192 points (its
    sub-cell counts no longer fit in LDS); ``crowded`` puts n/8 of those in a
    far tighter core (sigma 3e-7), so that single sub-cells hold hundreds of
    points.  Exact duplicates are dropped."""
    rng = np.random.default_rng(seed)
    c = 0.3  # well inside one grid cell for the grid sizes n gives (32 to 34 per axis)
    parts = [rng.random((n // 3, 3)), c + 1e-4 * rng.standard_normal((2 * n // 3 - (n // 8 if crowded else 0), 3))]
    if crowded:
        parts.append(c + 3e-7 * rng.standard_normal((n // 8, 3)))
    P = np.concatenate(parts).astype(np.float32)
    P = np.unique(P[np.all((P >= 0) & (P < 1), axis=1)], axis=0)
    return P[rng.permutation(len(P))]


@pytest.mark.parametrize("kind,n,dt", [("uniform", 1 << 20, np.float32), ("cluster", 1 << 20, np.float32),
                                       ("uniform", 10_000, np.float64), ("cluster", 3000, np.float64),
                                       ("giant", 70_000, np.float32), ("crowded", 70_000, np.float32)])
def test_grid_sort_bit_exact(kind, n, dt):
    note(f"grid_sort {kind} n={n} {dt.__name__}")
    if kind in ("giant", "crowded"):
        P = _one_giant_cell(n, kind == "crowded")
    else:
        P = getattr(gen, kind)(n, seed=0, dtype=dt)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    cid = _cells_np(P, grid)
    sst = grid.sub_start.cpu().numpy()
    sid, recs = _sub_records(P, grid, cid, sst, grid.subinfo.cpu().numpy())
    ref_perm = np.lexsort((np.arange(len(P)), sid, cid))
    ref_cs = np.searchsorted(cid[ref_perm], np.arange(grid.ncells + 1), side="left")
    assert np.array_equal(perm.cpu().numpy(), ref_perm)
    assert np.array_equal(cs.cpu().numpy(), ref_cs)
    s = srt.cpu().numpy()
    assert np.array_equal(s[:, :3], P[ref_perm])
    ib = s[:, 3].view(np.int32 if dt == np.float32 else np.int64)
    assert np.array_equal(ib, ref_perm)
    # sub-cell starts of (a sample of) the dense cells
    dense = sorted(recs)
    note(f"  {len(dense)} dense cells, sub-cells per dense cell up to {max([r[1] for r in recs.values()] or [0])}, "
         f"points per cell up to {np.diff(ref_cs).max()}")
    for c in dense[:: max(1, len(dense) // 200)]:
        off, ns = recs[c]
        a, b = ref_cs[c], ref_cs[c + 1]
        ids = sid[ref_perm[a:b]]
        want = np.searchsorted(ids, np.arange(ns + 1), side="left")
        assert np.array_equal(sst[off + 16:off + 16 + ns + 1], want), c


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


@pytest.mark.parametrize("kind,dt", [("uniform", np.float64), ("cluster", np.float32), ("filament", np.float32),
                                     ("cluster64", np.float32)])
@pytest.mark.parametrize("k", [8, 24, 64, 256])
def test_knn_f64_exact(kind, dt, k):
    """cluster64: 64 clusters, 89% of the points in cells with sub-grids (m up to 5)."""
    note(f"knn f64 {kind} k={k}")
    if kind == "cluster64":
        P = gen.cluster(20_000, seed=4, dtype=dt, n_clusters=64)
    else:
        P = getattr(gen, kind)(20_000, seed=4, dtype=dt)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    S = srt[:, :3].cpu().numpy()
    rng = np.random.default_rng(0)
    q = np.sort(rng.choice(len(P), 1500, replace=False)).astype(np.int32)
    got = vt.knn(srt, grid, cs, k, queries=torch.from_numpy(q).cuda(), dist="f64").cpu().numpy()
    ref = _knn_ref(S, q, k, "f64")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("kind", ["uniform", "cluster", "cluster64"])
def test_knn_f32_lists(kind):
    """Float distances: the list is the k nearest up to float rounding of d^2."""
    if kind == "cluster64":
        P = gen.cluster(20_000, seed=5, dtype=np.float32, n_clusters=64)
    else:
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


@pytest.mark.parametrize("kind", ["uniform", "cluster", "filament"])
@pytest.mark.parametrize("k", [32, 64])
def test_knn_f32_keys_exact(kind, k):
    """Float lists are exactly the k smallest (float d^2, sorted index) keys,
    d^2 rounded term by term: the clip compares its own d^2 with the list's
    last one bit for bit, so the k-NN must not round it any other way (a
    fused multiply-add would)."""
    P = getattr(gen, kind)(20_000, seed=6, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    S32 = srt[:, :3].cpu().numpy()
    q = np.sort(np.random.default_rng(1).choice(len(P), 1500, replace=False)).astype(np.int32)
    got = vt.knn(srt, grid, cs, k, queries=torch.from_numpy(q).cuda(), dist="f32").cpu().numpy()
    assert np.array_equal(got, knn_ref_f32(S32, q, k))


def _tied_boundary_points(dtype, k=8, n_base=20_000, n_seeds=1500, seed=0):
    """Uniform points on a dyadic grid; for each chosen seed s, its k-th
    nearest point q gets a mirror image s + (dy, dx, dz) of q - s = (dx, dy,
    dz).  The grid makes every coordinate difference exact, so q and its image
    are at the same distance from s, also when d^2 is rounded term by term
    (the two sums take the same terms), while a fused multiply-add would
    round them differently.  Returns the points and the seeds whose k-th and
    (k+1)-th nearest points are still such a tie."""
    rng = np.random.default_rng(seed)
    step = 2.0 ** (-23 if dtype == np.float32 else -50)
    P = np.round(rng.uniform(0.15, 0.85, (n_base, 3)) / step) * step
    seeds = rng.choice(n_base, n_seeds, replace=False)
    add = []
    for s in seeds:
        d = ((P - P[s]) ** 2).sum(1)
        o = np.argpartition(d, k + 1)[:k + 2]
        o = o[np.argsort(d[o], kind="stable")]
        off = P[o[k]] - P[s]
        if abs(off[0] - off[1]) > 1e-3 * np.sqrt(d[o[k]]):  # a distinct point
            add.append(P[s] + off[[1, 0, 2]])
    P = np.vstack([P, np.array(add)]).astype(dtype)
    assert len(np.unique(P, axis=0)) == len(P)
    X = P.astype(np.float64)
    tied = []
    for s in seeds:
        d = ((X - X[s]) ** 2).sum(1)
        o = np.argpartition(d, k + 1)[:k + 2]
        ds = np.sort(d[o])
        if ds[k] == ds[k + 1]:
            tied.append(s)
    return P, np.array(tied)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_ties_at_the_list_boundary(prec):
    """Lists of 8 whose 8th and 9th points tie exactly: the list keeps the
    lower sorted index and the stream phase must take the other one (it is a
    face in most of these cells).  Every cell must match the oracle."""
    dt = np.float32 if prec == "f32" else np.float64
    P, tied = _tied_boundary_points(dt)
    assert len(tied) > 500
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=8, max_gpu_retries=0, precision=prec)
    orc = oracle.tessellate(P.astype(np.float64), volume_ld=True)
    note(f"  ties {prec}: {len(tied)} seeds with a tie at ranks 8/9; stats {res.stats['passes']}")
    assert res.stats["fallback_cells"] == 0
    rp, col = res.row_ptr.cpu().numpy(), res.col.cpu().numpy()
    for s in tied:
        assert np.array_equal(col[rp[s]:rp[s + 1]], orc["col"][orc["row_ptr"][s]:orc["row_ptr"][s + 1]]), s
    assert np.array_equal(rp, orc["row_ptr"]) and np.array_equal(col, orc["col"])
    viol, rel = volume_errors(res.volume.cpu().numpy(), orc, prec)
    assert not viol.any(), rel.max()


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
    orc = oracle.tessellate(P.astype(np.float64), volume_ld=True)
    prec = kw.get("precision", "f64")
    bad = compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    assert not bad, f"{len(bad)} rows differ, e.g. {bad[:5]}"
    ve = volume_errors(res.volume.cpu().numpy(), orc, prec)
    viol, rel = ve
    note(f"  {name}: max rel vol err {rel.max():.3e} (oracle's double volume off on {ve.oracle_off}) "
         f"stats {res.stats}")
    assert not viol.any(), f"{viol.sum()} volumes out of tolerance, max rel {rel.max():.3e}"
    assert abs(res.volume.sum().item() - 1.0) < (1e-12 if prec == "f64" else 1e-6)


def test_anisotropic_box_and_boundary_points():
    lo, hi = (-0.5, 0.0, 2.0), (1.5, 0.25, 3.0)
    rng = np.random.default_rng(7)
    P = np.array(lo) + rng.random((5000, 3)) * (np.array(hi) - np.array(lo))
    P[:4] = [lo, hi, (lo[0], hi[1], lo[2]), (0.1, 0.1, 2.5)]
    P[4] = (hi[0], 0.125, 2.5)  # on a face
    res = vt.tessellate(torch.from_numpy(P).cuda(), box=(lo, hi), k0=32)
    orc = oracle.tessellate(P, lo, hi, volume_ld=True)
    assert not compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    viol, _ = volume_errors(res.volume.cpu().numpy(), orc, "f64")
    assert not viol.any()


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7])
def test_tiny_inputs(n):
    P = gen.uniform(n, seed=8, dtype=np.float64) if n else np.zeros((0, 3))
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=8)
    assert res.row_ptr.shape[0] == n + 1
    if n == 0:
        return
    orc = oracle.tessellate(P, volume_ld=True)
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
    orc = oracle.tessellate(P, volume_ld=True)
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
    orc = oracle.tessellate(P.astype(np.float64), vertices=True, volume_ld=True)
    vrp = res.vrow_ptr.cpu().numpy()
    vx = res.vxyz.cpu().numpy()
    vp = res.vplanes.cpu().numpy()
    P64 = P.astype(np.float64)
    rows, keys, got = [], [], []
    for i in range(0, len(P), 7):
        g = vertex_map(vrp, vx, vp, i)
        o = vertex_map(orc["vrow_ptr"], orc["vxyz"], orc["vplanes"], i)
        assert set(g) == set(o), i  # the combinatorics are exact
        for key, x in g.items():
            rows.append(i)
            keys.append(key)
            got.append(x)
    rows, keys, got = np.array(rows), np.array(keys), np.array(got)
    # reference: each vertex as the meeting point of its three planes (long double)
    ref, kappa = triple_vertices(P64, rows, keys)
    R = np.zeros(len(P))
    np.maximum.at(R, rows, np.abs(ref - P64[rows]).max(1))
    err = np.abs(got - ref).max(1)
    u = 2.0 ** -53 if prec == "f64" else 2.0 ** -24
    ratio = np.maximum(err - 2 * 2.0 ** -53, 0) / (u * kappa * R[rows])
    note(f"  vertices {prec}: error / R  p50 {np.median(err / R[rows]):.2e}  p99 "
         f"{np.percentile(err / R[rows], 99):.2e}  max {(err / R[rows]).max():.2e}; "
         f"error / (u kappa R) p99 {np.percentile(ratio, 99):.2f} max {ratio.max():.2f}")
    if prec == "f64":
        # Cramer's rule in double relative to the seed: a few roundings per
        # determinant term, amplified by the conditioning of the three planes;
        # adding the seed rounds once more in absolute terms.
        assert ratio.max() <= 64
    else:
        # a float vertex whose forward error bound exceeds 16 eps |v|_inf
        # (eps = 1e-6, the FP32 form's tolerance) is re-solved in double; the
        # bar is the FP32 form's 1e-5 R
        rel = err / R[rows]
        assert np.percentile(rel, 99) <= 1e-6 and rel.max() <= 1e-5


def test_host_fallback_forced():
    P = gen.uniform(20_000, seed=11, dtype=np.float32)
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=32, force_fail_every=3)
    assert res.stats["fallback_cells"] >= len(P) // 3
    orc = oracle.tessellate(P.astype(np.float64), volume_ld=True)
    assert not compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    viol, _ = volume_errors(res.volume.cpu().numpy(), orc, "f64")
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
    """Lists of 8 certify almost nothing; the stream phase finishes every cell
    on the GPU: the fast kernel certifies each cell that fits its 32 plane
    slots, the large-capacity kernel (same lists, same stream) the rest."""
    P = gen.cluster(100_000, seed=15, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    lists = vt.knn(srt, grid, cs, 8, dist=prec)
    r = vt.clip_cells(srt, lists, 8, precision=prec, stream=True, grid=grid, cell_start=cs)
    st = r["status"].cpu().numpy()
    pn = perm.cpu().numpy()
    orc = oracle.tessellate(P.astype(np.float64), volume_ld=True)
    deg = np.diff(orc["row_ptr"])[pn]  # faces of each cell, by sorted index
    cap = np.nonzero(st == 2)[0]
    note(f"  stream {prec}: statuses {np.bincount(st, minlength=4).tolist()}; faces of overflowing cells "
         f"min {deg[cap].min() if len(cap) else 0} median {np.median(deg[cap]) if len(cap) else 0}; "
         f"cells with > 32 faces {(deg > 32).sum()}")
    assert not np.any(st == 1)  # no cell is left waiting for a longer list
    assert np.all(st[deg > 34] == 2)  # cannot fit: 2F - 4 triangles > 64
    assert np.mean(st[deg <= 24] == 0) > 0.999  # small cells fit
    if len(cap):
        idx = torch.from_numpy(cap.astype(np.int32)).cuda()
        rc = vt.clip_cells(srt, lists[idx.long()].contiguous(), 8, cells=idx, precision=prec, stream=True,
                           grid=grid, cell_start=cs, capacity=1)
        assert np.all(rc["status"].cpu().numpy() == 0)
        for key in ("status", "volume", "nbr_count", "nbr"):
            r[key][idx.long()] = rc[key]
        st = r["status"].cpu().numpy()
    assert np.all(st == 0)
    ok = np.nonzero(st == 0)[0]
    vol = r["volume"].cpu().numpy()
    vol_orig = np.zeros(len(pn))
    vol_orig[pn[ok]] = vol[ok]
    viol, rel = volume_errors(vol_orig, orc, prec, rows=pn[ok])
    assert not viol.any(), rel.max()
    cnt = r["nbr_count"].cpu().numpy()
    nbr = r["nbr"].cpu().numpy()
    for s in np.concatenate([ok[::5], cap]):
        i = pn[s]
        got = np.sort(pn[nbr[s, :cnt[s]]])
        assert np.array_equal(got, orc["col"][orc["row_ptr"][i]:orc["row_ptr"][i + 1]])


# ------------------------------------------------------------ dataset reports

_ORC_CACHE = {}


def _oracle_full(name):
    if name not in _ORC_CACHE:
        P = gen.make(name, seed=0)
        _ORC_CACHE[name] = (P, oracle.tessellate(P.astype(np.float64), volume_ld=True))
    return _ORC_CACHE[name]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_uniform_1m_every_cell(prec):
    """2^20 uniform points (FP32 positions), k 32 -> 64 then the stream phase:
    every neighbour set and every volume against the oracle."""
    P, orc = _oracle_full("uniform-1m-f32")
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=32, max_gpu_retries=1, precision=prec)
    bad = compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    assert not bad, bad[:5]
    ve = volume_errors(res.volume.cpu().numpy(), orc, prec)
    viol, rel = ve
    note(f"  uniform 1M {prec}: passes {res.stats['passes']} streamed {res.stats['streamed_cells']} "
         f"max rel vol err {rel.max():.2e} (oracle's double volume off on {ve.oracle_off})")
    assert not viol.any()
    # pairwise summation (numpy) of the volumes: the cells tile the box
    assert abs(np.sum(res.volume.cpu().numpy()) - 1.0) <= (1e-12 if prec == "f64" else 1e-6)


def test_cluster_4m_fp32_report():
    """2^22 clustered points, FP32 clipping with FP64 rechecks (eps 1e-6), k 32
    -> 64 then the stream phase: per-pass failures, recheck count, and the FP32
    error against the oracle on 3000 seeded cells (volumes; vertices solved
    from each vertex's three planes in long double)."""
    P = gen.make("cluster-4m-f32", seed=0)
    pts = torch.from_numpy(P).cuda()
    res = vt.tessellate(pts, k0=32, max_gpu_retries=1, precision="f32")
    st = res.stats
    note(f"  cluster 4M f32: passes {st['passes']} streamed {st['streamed_cells']} capacity "
         f"{st['capacity_cells']} host {st['fallback_cells']} rechecks {st['rechecks']} refined "
         f"{st['refined_cells']} unresolved {st['unresolved_cells']}")
    assert st["unresolved_cells"] == 0
    rng = np.random.default_rng(7)
    cells = np.sort(rng.choice(len(P), 3000, replace=False))
    P64 = P.astype(np.float64)
    orc = oracle.tessellate(P64, cells=cells, volume_ld=True)
    viol, rel = volume_errors(res.volume.cpu().numpy(), orc, "f32", rows=cells)
    note(f"  volume rel err p50 {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e} max {rel.max():.2e}")
    assert not viol.any()
    # vertices of the same cells from the clip call (sorted indices), FP32 path
    cs, perm, srt, grid = vt.grid_sort(pts)
    pn = perm.cpu().numpy()
    inv = np.empty_like(pn)
    inv[pn] = np.arange(len(pn))
    q = torch.from_numpy(inv[cells].astype(np.int32)).cuda()
    lists = vt.knn(srt, grid, cs, 64, queries=q, dist="f32")
    r = vt.clip_cells(srt, lists, 64, cells=q, precision="f32", stream=True, grid=grid, cell_start=cs,
                      max_vert=256, max_nbr=256)
    stc = r["status"].cpu().numpy()
    ok = np.nonzero(stc == 0)[0]
    vc, vv, vp = r["vcount"].cpu().numpy(), r["verts"].cpu().numpy(), r["vplanes"].cpu().numpy()
    rows, keys, got = [], [], []
    for t in ok:
        i = cells[t]
        for m in range(vc[t]):
            pl = vp[t, m]
            rows.append(i)
            keys.append([pn[x] if x >= 0 else x for x in pl])
            got.append(vv[t, m])
    rows, keys, got = np.array(rows), np.array(keys), np.array(got)
    ref, kappa = triple_vertices(P64, rows, keys)
    R = np.zeros(len(P))
    np.maximum.at(R, rows, np.abs(ref - P64[rows]).max(1))
    err = np.abs(got - ref).max(1) / R[rows]
    note(f"  vertex err / R p50 {np.median(err):.2e} p99 {np.percentile(err, 99):.2e} max {err.max():.2e} "
         f"({len(err)} vertices of {len(ok)} cells)")
    assert len(ok) >= 0.99 * len(cells)
    assert np.percentile(err, 99) <= 1e-6 and err.max() <= 1e-5


@pytest.mark.parametrize("kind,n,prec", [("uniform", 20_000, "f64"), ("cluster", 100_000, "f32"),
                                         ("cluster", 100_000, "f64"), ("uniform", 3, "f64"), ("uniform", 1, "f32")])
def test_fused_no_list_every_cell(kind, n, prec):
    """The fused form (k0 = 0): no k-NN pass, every cell clipped straight
    from the grid rings around its generator; every neighbour set and volume
    against the oracle."""
    dt = np.float64 if (prec == "f64" and kind == "uniform") else np.float32
    P = getattr(gen, kind)(n, seed=17, dtype=dt)
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=0, precision=prec)
    st = res.stats
    assert st["ms_knn"] == 0.0 and st["passes"][0]["k"] == 0
    orc = oracle.tessellate(P.astype(np.float64), volume_ld=True)
    bad = compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc)
    assert not bad, bad[:5]
    ve = volume_errors(res.volume.cpu().numpy(), orc, prec)
    note(f"  fused {kind} {n} {prec}: max rel vol err {ve.rel.max(initial=0):.2e}; stats {st['passes']} "
         f"streamed {st['streamed_cells']} capacity {st['capacity_cells']} host {st['fallback_cells']}")
    assert not ve.viol.any()


@pytest.mark.parametrize("m,vertices", [(100, False), (160, True)])
def test_cell_with_more_neighbours_than_the_kernels_hold(m, vertices):
    """A generator inside a shell of m others (Fibonacci sphere, radius 0.1,
    jittered) has m faces: more planes than any GPU clip kernel holds, so the
    host fallback builds the cell, and the result carries its whole row (and,
    for m = 160, its 316 vertices, more than the per-cell vertex staging).
    Every row, volume, face area and vertex against the oracle."""
    rng = np.random.default_rng(m)
    k = np.arange(m) + 0.5
    phi = np.arccos(1 - 2 * k / m)
    theta = np.pi * (1 + 5 ** 0.5) * k
    shell = 0.5 + 0.1 * np.stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)], 1)
    shell += 1e-4 * rng.standard_normal(shell.shape)
    bg = rng.random((4000, 3))
    bg = bg[np.linalg.norm(bg - 0.5, axis=1) > 0.25]
    P = np.concatenate([[[0.5, 0.5, 0.5]], shell, bg])
    P = P[rng.permutation(len(P))]
    centre = int(np.nonzero(np.all(P == 0.5, axis=1))[0][0])
    res = vt.tessellate(torch.from_numpy(P).cuda(), k0=32, vertices=vertices, faces=True)
    orc = oracle.tessellate(P, vertices=vertices, volume_ld=True)
    st = res.stats
    note(f"  shell of {m}: host cells {st['fallback_cells']}, capacity cells {st['capacity_cells']}")
    assert st["fallback_cells"] >= 1
    rp, col = res.row_ptr.cpu().numpy(), res.col.cpu().numpy()
    assert rp[centre + 1] - rp[centre] == m
    assert not compare_rows(rp, col, orc)
    assert not volume_errors(res.volume.cpu().numpy(), orc, "f64").viol.any()
    a_g, a_o = res.area.cpu().numpy(), orc["area"]
    assert np.all(np.abs(a_g - a_o) <= 1e-10 * np.abs(a_o) + 1e-15)
    if vertices:
        vrp, vx, vp = res.vrow_ptr.cpu().numpy(), res.vxyz.cpu().numpy(), res.vplanes.cpu().numpy()
        assert vrp[centre + 1] - vrp[centre] == 2 * m - 4
        for i in [centre] + list(range(0, len(P), 97)):
            g = vertex_map(vrp, vx, vp, i)
            o = vertex_map(orc["vrow_ptr"], orc["vxyz"], orc["vplanes"], i)
            assert set(g) == set(o), i
            for key in g:
                assert np.max(np.abs(g[key] - o[key])) <= 1e-9, (i, key)


@pytest.mark.parametrize("kind,n,dt,box", [
    ("uniform", 20_000, np.float64, ((0, 0, 0), (1, 1, 1))),
    ("cluster", 200_000, np.float32, ((0, 0, 0), (1, 1, 1))),
    ("uniform", 5000, np.float64, ((-0.5, 0.0, 0.25), (0.5, 2.0, 0.85))),
    ("uniform", 7, np.float64, ((0, 0, 0), (1, 1, 1))),
    ("uniform", 1, np.float32, ((0, 0, 0), (1, 1, 1))),
])
def test_periodic_every_cell(kind, n, dt, box):
    """Periodic boxes (the box a 3-torus): every cell's neighbour multiset and
    volume against the periodic oracle, face areas too; the volumes tile the
    box."""
    lo, hi = np.array(box[0], float), np.array(box[1], float)
    P = getattr(gen, kind)(n, seed=19, dtype=dt)
    P = (lo + P.astype(np.float64) * (hi - lo)).astype(dt)
    P = np.minimum(P, np.nextafter(hi, lo).astype(dt))  # [lo, hi)
    res = vt.tessellate(torch.from_numpy(P).cuda(), box=box, periodic=True, faces=True)
    orc = oracle.tessellate(P.astype(np.float64), box[0], box[1], periodic=True, volume_ld=True)
    rp, col = res.row_ptr.cpu().numpy(), res.col.cpu().numpy()
    bad = compare_rows(rp, col, orc)
    assert not bad, (bad[:5], [list(col[rp[i]:rp[i + 1]]) for i in bad[:2]],
                     [list(orc["col"][orc["row_ptr"][i]:orc["row_ptr"][i + 1]]) for i in bad[:2]])
    ve = volume_errors(res.volume.cpu().numpy(), orc, "f64")
    st = res.stats
    note(f"  periodic {kind} {n}: max rel vol err {ve.rel.max():.2e}; passes {st['passes']} "
         f"host {st['fallback_cells']} capacity {st['capacity_cells']}")
    assert not ve.viol.any()
    assert abs(np.sum(res.volume.cpu().numpy()) / np.prod(hi - lo) - 1.0) <= 1e-12
    # a row may name one point once per image: compare the areas of equal ids as sets
    own = np.repeat(np.arange(len(P)), np.diff(rp))
    a_g = res.area.cpu().numpy()[np.lexsort((res.area.cpu().numpy(), col, own))]
    a_o = orc["area"][np.lexsort((orc["area"], orc["col"], own))]
    assert np.all(np.abs(a_g - a_o) <= 1e-9 * np.abs(a_o) + 1e-14 * np.prod(hi - lo) ** (2 / 3))
