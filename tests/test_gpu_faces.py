"""GPU parity of the per-face outputs (the area of each neighbour's face and
the cell centroids) against the FP64 oracle, through every path a cell can
take: the fast and large-capacity clip kernels, the GPU stream phase, the
host fallback, the learned first pass, and both index spaces.

Bars (see ``helpers``): area within 1e-10 relative or 1e-12 R^2 + 2e-15 R L
(L the box size: the oracle's own error on cells far smaller than the box),
centroid within 1e-10 R or 1e-12 R^4 / V; the other outputs are bit-identical
to a run without face outputs.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from helpers import compare_rows, face_errors, note, radius_of_cells
from paper_2412_04514_amd import gen

pytestmark = pytest.mark.gpu

vt = pytest.importorskip("paper_2412_04514_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(res, P, orc, name, rows=None):
    bad = compare_rows(res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), orc, rows=rows)
    assert not bad, f"{name}: {len(bad)} rows differ, e.g. {bad[:5]}"
    r2 = radius_of_cells(P, orc)
    na, nc, ra, rc = face_errors(res.area.cpu().numpy(), res.centroid.cpu().numpy(), orc, r2, rows=rows,
                                 gpu_row_ptr=res.row_ptr.cpu().numpy())
    note(f"  {name}: area err/bar max {ra:.3f}, centroid err/bar max {rc:.3f}  stats {res.stats}")
    assert na == 0 and nc == 0, (na, nc, ra, rc)


CASES = [
    # name, generator, n, dtype, kwargs
    ("uniform-50k-f64", "uniform", 50_000, np.float64, dict(k0=32, max_gpu_retries=1)),
    ("uniform-100k-f32clip", "uniform", 100_000, np.float32, dict(k0=32, max_gpu_retries=1, precision="f32")),
    ("cluster-100k-f64clip", "cluster", 100_000, np.float32, dict(k0=32, max_gpu_retries=1)),
    ("cluster-100k-f32clip", "cluster", 100_000, np.float32, dict(k0=32, max_gpu_retries=1, precision="f32")),
    ("filament-100k-f32-k16-stream", "filament", 100_000, np.float32, dict(k0=16, max_gpu_retries=0,
                                                                          precision="f32")),
    ("cluster-50k-f64-k8-stream", "cluster", 50_000, np.float64, dict(k0=8, max_gpu_retries=0)),
    ("uniform-20k-f32-fallback", "uniform", 20_000, np.float32, dict(k0=32, force_fail_every=3)),
    ("cluster-30k-f64-nostream", "cluster", 30_000, np.float32, dict(k0=16, max_gpu_retries=0, gpu_stream=False)),
]


@pytest.mark.parametrize("name,kind,n,dt,kw", CASES, ids=[c[0] for c in CASES])
def test_faces_parity(name, kind, n, dt, kw):
    note(f"faces {name}")
    P = getattr(gen, kind)(n, seed=0, dtype=dt)
    pts = torch.from_numpy(P).cuda()
    res = vt.tessellate(pts, faces=True, **kw)
    plain = vt.tessellate(pts, **kw)
    # the face outputs change nothing else
    assert torch.equal(res.row_ptr, plain.row_ptr) and torch.equal(res.col, plain.col)
    assert torch.equal(res.volume, plain.volume)
    orc = oracle.tessellate(P.astype(np.float64), vertices=True)
    _check(res, P.astype(np.float64), orc, name)
    if kw.get("force_fail_every"):
        assert res.stats["fallback_cells"] >= n // 3
    if "stream" in name and kw.get("gpu_stream", True):
        assert res.stats["streamed_cells"] > 0
    if name.startswith("cluster-100k"):
        assert res.stats["capacity_cells"] > 0


def test_faces_closed_forms():
    """The golden closed forms: centroids and face areas of boxes, slabs,
    octant cubes and the hexagonal mid-section of the cube."""
    with open(os.path.join(GOLDEN, "closed_forms.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        P = np.array(case["points"], dtype=np.float64)
        lo, hi = case.get("lo", [0, 0, 0]), case.get("hi", [1, 1, 1])
        res = vt.tessellate(torch.from_numpy(P).cuda(), box=(lo, hi), k0=8, faces=True)
        np.testing.assert_allclose(res.centroid.cpu().numpy(), case["centroid"], rtol=1e-13, atol=1e-15,
                                   err_msg=case["name"])
        want = np.array([a for row in case["area"] for a in row], dtype=np.float64)
        np.testing.assert_allclose(res.area.cpu().numpy(), want, rtol=1e-13, atol=1e-15, err_msg=case["name"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_faces_bcc_lattice(prec):
    """Degenerate input (a binary-exact BCC lattice, four or more planes per
    vertex): interior cells are truncated octahedra centred on their
    generators, 8 hexagons of area 3 sqrt(3) a^2 / 16 and 6 squares of a^2 / 8."""
    m = 8
    a = 1.0 / m
    g = (np.arange(m) + 0.5) / m
    sc = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    h = np.arange(1, m) / m
    bc = np.stack(np.meshgrid(h, h, h, indexing="ij"), -1).reshape(-1, 3)
    P = np.concatenate([sc, bc])
    dt = np.float32 if prec == "f32" else np.float64
    res = vt.tessellate(torch.from_numpy(P.astype(dt)).cuda(), k0=32, precision=prec, faces=True)
    orc = oracle.tessellate(P, vertices=True)
    _check(res, P, orc, f"bcc {prec}")
    rp, col = res.row_ptr.cpu().numpy(), res.col.cpu().numpy()
    area, cen = res.area.cpu().numpy(), res.centroid.cpu().numpy()
    interior = np.concatenate([np.all((sc > 1.4 * a) & (sc < 1 - 1.4 * a), axis=1),
                               np.all((bc > 1.9 * a) & (bc < 1 - 1.9 * a), axis=1)])
    np.testing.assert_allclose(cen[interior], P[interior], rtol=0, atol=1e-14)
    for i in np.nonzero(interior)[0]:
        d = np.linalg.norm(P[col[rp[i]:rp[i + 1]]] - P[i], axis=1)
        want = np.where(d < 0.9 * a, 3 * np.sqrt(3) * a * a / 16, a * a / 8)
        np.testing.assert_allclose(area[rp[i]:rp[i + 1]], want, rtol=1e-12)


def test_faces_sorted_index_space():
    P = gen.cluster(40_000, seed=13, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    a = vt.tessellate(pts, k0=32, faces=True)
    b = vt.tessellate(pts, k0=32, faces=True, index_space="sorted")
    _, perm, _, _ = vt.grid_sort(pts)
    pn = perm.cpu().numpy()
    inv = np.empty_like(pn)
    inv[pn] = np.arange(len(pn))
    ra, ca, aa = a.row_ptr.cpu().numpy(), a.col.cpu().numpy(), a.area.cpu().numpy()
    rb, cb, ab = b.row_ptr.cpu().numpy(), b.col.cpu().numpy(), b.area.cpu().numpy()
    for s in range(0, len(P), 13):
        i = pn[s]
        o = np.argsort(inv[ca[ra[i]:ra[i + 1]]])
        assert np.array_equal(inv[ca[ra[i]:ra[i + 1]]][o], cb[rb[s]:rb[s + 1]])
        assert np.array_equal(aa[ra[i]:ra[i + 1]][o], ab[rb[s]:rb[s + 1]])
    assert np.array_equal(a.centroid.cpu().numpy()[pn], b.centroid.cpu().numpy())


def test_faces_deterministic():
    P = gen.cluster(100_000, seed=14, dtype=np.float32)
    pts = torch.from_numpy(P).cuda()
    a = vt.tessellate(pts, k0=32, precision="f32", faces=True)
    b = vt.tessellate(pts, k0=32, precision="f32", faces=True)
    assert torch.equal(a.area, b.area) and torch.equal(a.centroid, b.centroid)


def test_clip_cells_faces_next_to_nbr():
    """The per-cell clip call: each area sits at its neighbour's position."""
    P = gen.uniform(30_000, seed=16, dtype=np.float64)
    pts = torch.from_numpy(P).cuda()
    cs, perm, srt, grid = vt.grid_sort(pts)
    lists = vt.knn(srt, grid, cs, 64, dist="f64")
    r = vt.clip_cells(srt, lists, 64, precision="f64", stream=True, grid=grid, cell_start=cs, faces=True)
    st = r["status"].cpu().numpy()
    pn = perm.cpu().numpy()
    orc = oracle.tessellate(P, vertices=True)
    r2 = radius_of_cells(P, orc)
    cnt, nbr, area = r["nbr_count"].cpu().numpy(), r["nbr"].cpu().numpy(), r["area"].cpu().numpy()
    cen = r["centroid"].cpu().numpy()
    ok = np.nonzero(st == 0)[0]
    assert len(ok) > 0.99 * len(P)
    for s in ok[::7]:
        i = pn[s]
        ids = pn[nbr[s, :cnt[s]]]
        o = np.argsort(ids)
        a0, a1 = orc["row_ptr"][i], orc["row_ptr"][i + 1]
        assert np.array_equal(ids[o], orc["col"][a0:a1])
        bar = 1e-10 * orc["area"][a0:a1] + 1e-12 * r2[i] + 2e-15 * np.sqrt(r2[i])
        assert np.all(np.abs(area[s, :cnt[s]][o] - orc["area"][a0:a1]) <= bar), i
        bar_c = 1e-10 * np.sqrt(r2[i]) + 1e-12 * r2[i] ** 2 / orc["volume"][i]
        assert np.all(np.abs(cen[s] - orc["centroid"][i]) <= bar_c), i


def test_faces_cluster_4m_properties():
    """2^22 clustered points, FP32 clipping: what holds at any size (the first
    moments of the cells add up to the box's; each face has one area seen from
    both sides) and 2000 seeded cells against the oracle."""
    P = gen.make("cluster-4m-f32", seed=0)
    pts = torch.from_numpy(P).cuda()
    res = vt.tessellate(pts, k0=32, max_gpu_retries=1, precision="f32", faces=True)
    n = len(P)
    vol, cen = res.volume, res.centroid
    mom = (vol[:, None] * (cen - 0.5)).sum(0).cpu().numpy()
    note(f"  cluster 4M faces: first moment about the box centre {mom} stats {res.stats}")
    # zero for exact volumes; the FP32 path's volumes carry up to 1e-5
    # relative error each (the centroids are computed in double)
    assert np.all(np.abs(mom) <= 1e-6)
    src = torch.repeat_interleave(torch.arange(n, device="cuda"), (res.row_ptr[1:] - res.row_ptr[:-1]).long())
    c = res.col.long()
    kf, of = torch.sort(src * n + c)
    kb, ob = torch.sort(c * n + src)
    assert torch.equal(kf, kb)
    af, ab = res.area[of], res.area[ob]
    rel = ((af - ab).abs() / torch.maximum(af.abs(), ab.abs())).cpu().numpy()
    note(f"  mutual areas: rel diff p50 {np.median(rel):.2e} p99.99 {np.percentile(rel, 99.99):.2e} "
         f"max {rel.max():.2e}")
    # both sides are within their bars of the same exact area
    big = (torch.maximum(af.abs(), ab.abs()) > 1e-4 * (1.0 / n) ** (2 / 3)).cpu().numpy()
    assert np.percentile(rel[big], 99.99) <= 1e-8
    del src, c, kf, kb, of, ob, af, ab
    rng = np.random.default_rng(17)
    cells = np.sort(rng.choice(n, 2000, replace=False))
    P64 = P.astype(np.float64)
    orc = oracle.tessellate(P64, cells=cells, vertices=True)
    _check(res, P64, orc, "cluster 4M sampled", rows=cells)
