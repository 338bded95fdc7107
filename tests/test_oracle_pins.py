"""Pins of the FP64 oracle against what geometry fixes (no GPU).

The paper prints no worked example or number for the method, so the oracle is
pinned by: brute force on tiny inputs (every plane triple, no clipping); the
stopping lemma (the certified cell equals the cell clipped by all N-1
bisectors); an independent half-space intersection (scipy's Qhull) on medium
inputs; closed forms (one point, a slab split, BCC and simple-cubic lattices,
the 8 octant centres, with their centroids and face areas); invariants
(volumes tile the box, first moments add up to the box's, pyramids over the
faces of interior cells fill the cell, symmetric neighbour relation, Euler's
formula, equidistant vertices, empty spheres, equal face areas seen from both
sides); the Poisson-Voronoi mean face count; and the work counters of the
k_needed pass (planes tested, vertex evaluations, vertices created, R^2
updates) by closed forms and by a Qhull replay of the nearest-first clipping.
"""
import json
import os

import numpy as np
import pytest

import brute
import oracle
from paper_2412_04514_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(r):
    return [list(x) for x in oracle.rows(r)]


@pytest.mark.parametrize("seed", range(60))
def test_oracle_matches_brute_force(seed):
    """Neighbour sets equal, volumes to 1e-13 (abs, unit box), vertices to 1e-12."""
    rng = np.random.default_rng(1000 + seed)
    n = [2, 3, 5, 8, 13, 21, 34, 40][seed % 8]
    if seed % 3 == 0:  # a tight clump plus a few far points
        P = np.concatenate([0.5 + 0.02 * rng.standard_normal((n, 3)), rng.random((3, 3))])
        P = np.clip(P, 0, 1)
    else:
        P = rng.random((n, 3))
    lo, hi = ((0, 0, 0), (1, 1, 1)) if seed % 4 else ((-0.1, 0.0, -0.3), (1.2, 1.0, 1.05))
    r = oracle.tessellate(P, lo, hi, vertices=True, volume_ld=True)
    vol, nbrs, verts, areas, cents = brute.brute_cells(P, lo, hi, geometry=True)
    np.testing.assert_allclose(r["volume"], vol, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r["volume_ld"], vol, rtol=0, atol=1e-13)
    assert _rows(r) == nbrs
    want_area = np.array([areas[i][j] for i in range(len(P)) for j in nbrs[i]])
    np.testing.assert_allclose(r["area"], want_area, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["centroid"], cents, rtol=0, atol=1e-11)
    for i in range(len(P)):
        a, b = r["vrow_ptr"][i], r["vrow_ptr"][i + 1]
        got = {tuple(int(x) for x in r["vplanes"][k]): r["vxyz"][k] for k in range(a, b)}
        assert set(got) == set(verts[i])
        for t, x in got.items():
            np.testing.assert_allclose(x, verts[i][t], rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind,n,seed", [("uniform", 1500, 0), ("cluster", 1500, 1), ("uniform", 400, 2)])
def test_stopping_lemma(kind, n, seed):
    """Certified early stop gives exactly the cell clipped by every bisector."""
    # FP32-rounded inputs (as in the clustered workloads): q - p is then exact in
    # FP64, so two clipping orders agree to rounding of the cell's own size.
    if kind == "cluster":
        P = gen.cluster(n, seed=seed, dtype=np.float32, n_clusters=8).astype(np.float64)
    else:
        P = getattr(gen, kind)(n, seed=seed, dtype=np.float64)
    a = oracle.tessellate(P)
    b = oracle.tessellate(P, all_planes=True)
    assert np.array_equal(a["row_ptr"], b["row_ptr"]) and np.array_equal(a["col"], b["col"])
    # 1e-12 relative, floored at 1e-14 of the mean cell volume: cells far below
    # the mean size (cluster cores) carry rounding from the box-scale start.
    np.testing.assert_allclose(a["volume"], b["volume"], rtol=1e-12, atol=1e-14 / n)


def _inner(ns, cs, p):
    """A strictly interior point: a quarter of the half nearest-neighbour distance
    from the seed, toward the box centre (the seed itself may lie on a wall)."""
    bis = np.abs(ns).sum(axis=1) > 0
    dist = cs[6:] / np.linalg.norm(ns[6:], axis=1)
    u = 0.5 - p
    u = u / np.linalg.norm(u)
    return 0.25 * dist.min() * u


def test_against_halfspace_intersection():
    """Volumes and neighbour sets against scipy's Qhull half-space intersection."""
    from scipy.spatial import ConvexHull, HalfspaceIntersection
    P = gen.cluster(300, seed=5, dtype=np.float64, n_clusters=6)
    r = oracle.tessellate(P)
    rows = _rows(r)
    for i in range(len(P)):
        ns, cs, ids = brute.halfspaces(P, i, (0, 0, 0), (1, 1, 1))
        hs = np.hstack([ns, -cs[:, None]])
        H = HalfspaceIntersection(hs, _inner(ns, cs, P[i]))
        hull = ConvexHull(H.intersections)
        assert abs(hull.volume - r["volume"][i]) <= 1e-10 * max(hull.volume, 1e-12)
        act = np.abs(H.intersections @ ns.T - cs) <= 1e-9 * np.linalg.norm(ns, axis=1)
        faces = sorted(int(ids[f]) for f in range(len(cs)) if ids[f] >= 0 and act[:, f].sum() >= 3)
        # a plane touching >=3 vertices has positive area on generic input
        assert faces == rows[i]


def test_closed_forms():
    with open(os.path.join(GOLDEN, "closed_forms.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        P = np.array(case["points"], dtype=np.float64)
        lo, hi = case.get("lo", [0, 0, 0]), case.get("hi", [1, 1, 1])
        r = oracle.tessellate(P, lo, hi)
        np.testing.assert_allclose(r["volume"], case["volume"], rtol=1e-13, atol=1e-15, err_msg=case["name"])
        assert _rows(r) == case["neighbours"], case["name"]
        np.testing.assert_allclose(r["centroid"], case["centroid"], rtol=1e-13, atol=1e-15, err_msg=case["name"])
        want = np.array([a for row in case["area"] for a in row], dtype=np.float64)
        np.testing.assert_allclose(r["area"], want, rtol=1e-13, atol=1e-15, err_msg=case["name"])


def _lattice_bcc(m):
    """Simple-cubic part at (i+1/2)/m and body centres at (i+1)/m (binary exact for m=8)."""
    g = (np.arange(m) + 0.5) / m
    sc = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    h = np.arange(1, m) / m
    bc = np.stack(np.meshgrid(h, h, h, indexing="ij"), -1).reshape(-1, 3)
    return sc, bc


def test_bcc_truncated_octahedra():
    """Interior cells of a BCC lattice are truncated octahedra: volume a^3/2, 14 neighbours."""
    m = 8
    a = 1.0 / m
    sc, bc = _lattice_bcc(m)
    P = np.concatenate([sc, bc])
    r = oracle.tessellate(P, vertices=True)
    deg = np.diff(r["row_ptr"])
    i_sc = np.all((sc > 1.4 * a) & (sc < 1 - 1.4 * a), axis=1)
    i_bc = np.all((bc > 1.9 * a) & (bc < 1 - 1.9 * a), axis=1)
    interior = np.concatenate([i_sc, i_bc])
    assert interior.sum() > 100
    np.testing.assert_allclose(r["volume"][interior], a ** 3 / 2, rtol=1e-12)
    assert np.all(deg[interior] == 14)
    # 24 vertices, each on exactly three faces
    vr = np.diff(r["vrow_ptr"])
    assert np.all(vr[interior] == 24)
    assert abs(r["volume"].sum() - 1.0) < 1e-12
    # centrally symmetric cells: centroid = generator; 8 regular hexagons of
    # edge a sqrt(2)/4 towards the body-diagonal neighbours (3 sqrt(3) a^2/16)
    # and 6 squares of that edge towards the axis neighbours (a^2/8)
    np.testing.assert_allclose(r["centroid"][interior], P[interior], rtol=0, atol=1e-14)
    for i in np.nonzero(interior)[0]:
        a0, a1 = r["row_ptr"][i], r["row_ptr"][i + 1]
        d = np.linalg.norm(P[r["col"][a0:a1]] - P[i], axis=1)
        want = np.where(d < 0.9 * a, 3 * np.sqrt(3) * a * a / 16, a * a / 8)
        np.testing.assert_allclose(r["area"][a0:a1], want, rtol=1e-12)


def test_simple_cubic_lattice():
    m = 8  # binary-exact lattice: degenerate planes pass exactly through vertices
    g = (np.arange(m) + 0.5) / m
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    r = oracle.tessellate(P)
    np.testing.assert_allclose(r["volume"], 1.0 / m ** 3, rtol=1e-12)
    idx = np.rint(P * m - 0.5).astype(int)
    expect = 6 - np.sum((idx == 0) | (idx == m - 1), axis=1)
    assert np.array_equal(np.diff(r["row_ptr"]), expect)
    # every cell is the cube around its generator: centroid = generator, faces 1/m^2
    np.testing.assert_allclose(r["centroid"], P, rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["area"], 1.0 / m ** 2, rtol=1e-13)


def _invariants(P, r, tol_rel=1e-12):
    n = len(P)
    rows = oracle.rows(r)
    # volumes tile the box
    assert abs(np.sum(np.sort(r["volume"])) - 1.0) < 1e-12
    assert np.all(r["volume"] > 0)
    # neighbour relation symmetric, face areas agree from both sides
    area = {}
    for i in range(n):
        for k, j in enumerate(rows[i]):
            area[(i, int(j))] = r["area"][r["row_ptr"][i] + k]
    for (i, j), a in area.items():
        assert (j, i) in area, (i, j)
        # relative, floored at 1e-12 of the mean face scale (tiny cluster faces)
        assert abs(area[(j, i)] - a) <= 1e-10 * a + 1e-12 * (1.0 / n) ** (2 / 3)
    # centroids: the first moments of the cells add up to the box's (centre 1/2)
    mom = (r["volume"][:, None] * r["centroid"]).sum(0)
    np.testing.assert_allclose(mom, 0.5, rtol=0, atol=1e-12)
    # areas: a cell with no box-wall face is the union of the pyramids from its
    # generator over its faces, of height |p_j - p_i| / 2
    walls = np.zeros(n, bool)
    owner = np.repeat(np.arange(n), np.diff(r["vrow_ptr"]))
    np.logical_or.at(walls, owner, np.any(r["vplanes"] < 0, axis=1))
    own = np.repeat(np.arange(n), np.diff(r["row_ptr"]))
    h = np.linalg.norm(P[r["col"]] - P[own], axis=1) / 2
    pyr = np.bincount(own, weights=r["area"] * h / 3, minlength=n)
    inner = ~walls
    assert inner.sum() > n // 2
    np.testing.assert_allclose(pyr[inner], r["volume"][inner], rtol=1e-11)
    # closed convex polyhedra
    assert np.all(r["euler"] == 2)
    # generic vertices: three faces; equidistant from the generators of their faces
    assert np.all(r["vdeg"] == 3)
    from scipy.spatial import cKDTree
    tree = cKDTree(P)
    for i in range(n):
        a, b = r["vrow_ptr"][i], r["vrow_ptr"][i + 1]
        X = r["vxyz"][a:b]
        d0 = np.linalg.norm(X - P[i], axis=1)
        for k in range(a, b):
            for j in r["vplanes"][k]:
                if j >= 0:
                    dj = np.linalg.norm(r["vxyz"][k] - P[j])
                    assert abs(dj - d0[k - a]) <= tol_rel * d0[k - a] + 1e-15
        # empty sphere: nothing strictly closer to a vertex than its own generator
        dn, _ = tree.query(X, k=1)
        assert np.all(dn >= d0 * (1 - 1e-12) - 1e-15)


@pytest.mark.parametrize("kind,seed", [("uniform", 0), ("cluster", 1), ("filament", 2)])
def test_invariants(kind, seed):
    P = getattr(gen, kind)(3000, seed=seed, dtype=np.float64)
    r = oracle.tessellate(P, vertices=True)
    _invariants(P, r)


def test_fp32_inputs_are_exact_in_fp64():
    P = gen.uniform(2000, seed=7, dtype=np.float32)
    r = oracle.tessellate(P.astype(np.float64), vertices=True)
    _invariants(P.astype(np.float64), r)


def test_poisson_voronoi_mean_faces():
    """Typical Poisson-Voronoi cell: E[faces] = 2 + 48 pi^2 / 35 (Meijering 1953)."""
    P = gen.uniform(200_000, seed=11, dtype=np.float64)
    r = oracle.tessellate(P)
    inner = np.all((P > 0.12) & (P < 0.88), axis=1)  # seeds chosen by position only
    faces = np.diff(r["row_ptr"])[inner]
    expect = 2 + 48 * np.pi ** 2 / 35
    se = faces.std() / np.sqrt(len(faces))
    assert abs(faces.mean() - expect) < 5 * se + 0.02, (faces.mean(), expect, se)
    # and the mean cell volume is exactly the box volume over N
    assert abs(r["volume"].mean() - 1 / len(P)) < 1e-18


def test_validation_errors():
    with pytest.raises(oracle.OracleError):
        oracle.tessellate(np.array([[0.5, 0.5, 1.5]]))
    with pytest.raises(oracle.OracleError):
        oracle.tessellate(np.array([[0.5, 0.5, 0.5], [0.1, 0.2, 0.3], [0.5, 0.5, 0.5]]))
    r = oracle.tessellate(np.zeros((0, 3)))
    assert r["row_ptr"].tolist() == [0]


def _kneeded_by_halfspaces(P, i, kmax):
    """Least k with d_k^2 > 4 R_k^2, R_k from a Qhull intersection of the box and
    the k nearest bisectors (exact (d^2, index) order)."""
    from scipy.spatial import HalfspaceIntersection
    d2 = np.sum((P - P[i]) ** 2, axis=1)
    order = [j for j in np.lexsort((np.arange(len(P)), d2)) if j != i]
    for k in range(1, min(kmax, len(P) - 1) + 1):
        ns, cs, _ = brute.halfspaces(P, i, (0, 0, 0), (1, 1, 1), subset=order[:k])
        H = HalfspaceIntersection(np.hstack([ns, -cs[:, None]]), _inner(ns, cs, P[i]))
        R2 = np.max(np.sum(H.intersections ** 2, axis=1))
        if d2[order[k - 1]] > 4 * R2:
            return k
    return len(P) - 1 if kmax >= len(P) - 1 else kmax + 1


def test_kneeded_against_halfspaces():
    P = gen.uniform(400, seed=3, dtype=np.float64)
    cells = np.arange(0, 400, 20)
    kn = oracle.kneeded(P, cells=cells, kcap=128)["kneeded"]
    ref = [_kneeded_by_halfspaces(P, int(i), 128) for i in cells]
    assert kn.tolist() == ref


def test_kneeded_monotone_and_work():
    P = gen.uniform(5000, seed=4, dtype=np.float64)
    k = oracle.kneeded(P, kcap=4096, kwork=32)
    kn = k["kneeded"]
    assert kn.min() >= 1
    # at list size 32, certified cells never test more planes than they have
    cert = kn <= 32
    assert np.all(k["tested"][cert] <= kn[cert])
    assert np.all(k["tested"] <= 32)
    # the exhaustive cell count: N=1 needs nothing, N=2 needs its one neighbour
    assert oracle.kneeded(np.array([[0.3, 0.4, 0.5]]))["kneeded"].tolist() == [0]
    two = oracle.kneeded(np.array([[0.3, 0.5, 0.5], [0.7, 0.5, 0.5]]))["kneeded"]
    assert two.tolist() == [1, 1]


def test_oracle_vertices_meet_their_three_planes():
    """Each oracle vertex lies where the three planes it names meet (solved
    in long double): the edge interpolation keeps the geometry it reports."""
    from helpers import triple_vertices
    P = gen.cluster(4000, seed=21, dtype=np.float32, n_clusters=16).astype(np.float64)
    o = oracle.tessellate(P, vertices=True)
    owner = np.repeat(np.arange(len(P)), np.diff(o["vrow_ptr"]))
    ref, kappa = triple_vertices(P, owner, o["vplanes"])
    R = np.zeros(len(P))
    np.maximum.at(R, owner, np.abs(ref - P[owner]).max(1))
    rel = np.abs(o["vxyz"] - ref).max(1) / R[owner]
    assert np.median(rel) <= 1e-15 and rel.max() <= 1e-9
    # the order in which the three planes are named does not matter ...
    swapped = o["vplanes"][:, [1, 0, 2]]
    ref2, _ = triple_vertices(P, owner, swapped)
    assert np.allclose(ref2, ref, rtol=0, atol=1e-12)
    # ... but a wrong plane does: each vertex moves off when one id is replaced
    wrong = o["vplanes"].copy()
    wrong[:, 0] = (owner + len(P) // 2) % len(P)
    ref3, _ = triple_vertices(P, owner, wrong)
    moved = np.abs(ref3 - o["vxyz"]).max(1) / R[owner]
    assert np.median(np.nan_to_num(moved, nan=np.inf)) > 1e-3  # singular triples count as moved


def _work_by_halfspaces(P, i, kwork):
    """Work of nearest-first clipping of cell i with a list of ``kwork``,
    replayed with Qhull: C_0 is the box; before bisector m the cell stops if
    d_m^2 > 4 R_{m-1}^2; else plane m is tested against every vertex of
    C_{m-1} (|V(C_{m-1})| evaluations), and if it cuts, C_m is the Qhull
    intersection of the box with the first m bisectors, the vertices created
    are those of C_m that were not inside vertices of C_{m-1}, and R^2 is
    updated over every vertex of C_m."""
    from scipy.spatial import HalfspaceIntersection
    d2 = np.sum((P - P[i]) ** 2, axis=1)
    order = [j for j in np.lexsort((np.arange(len(P)), d2)) if j != i]
    ns0, cs0, _ = brute.halfspaces(P, i, (0, 0, 0), (1, 1, 1), subset=[])
    corners = np.array([[(cs0[1] if b & 1 else -cs0[0]), (cs0[3] if b & 2 else -cs0[2]),
                         (cs0[5] if b & 4 else -cs0[4])] for b in range(8)])
    V = corners
    tested = evals = created = r2 = 0
    for m in range(1, min(kwork, len(P) - 1) + 1):
        q = order[m - 1]
        if d2[q] > 4 * np.max(np.sum(V ** 2, axis=1)):
            break
        tested += 1
        evals += len(V)
        n = P[q] - P[i]
        s = V @ n - 0.5 * (n @ n)
        if not np.any(s > 0):
            continue
        ns, cs, _ = brute.halfspaces(P, i, (0, 0, 0), (1, 1, 1), subset=order[:m])
        H = HalfspaceIntersection(np.hstack([ns, -cs[:, None]]), _inner(ns, cs, P[i]))
        Vm = H.intersections
        created += len(Vm) - int(np.sum(~(s > 0)))
        r2 += len(Vm)
        V = Vm
    return tested, evals, created, r2


def test_work_counters_closed_forms():
    """Two points split by a plane parallel to two walls: one plane tested
    against the 8 box corners, 4 edges cut, R^2 over the 8 vertices of the
    slab.  A third point whose bisector misses the slab adds 8 evaluations
    and nothing else."""
    two = oracle.kneeded(np.array([[0.1, 0.5, 0.5], [0.3, 0.5, 0.5]]), kcap=8, kwork=8)
    assert [int(two[k][0]) for k in ("tested", "evals", "created", "r2upd")] == [1, 8, 4, 8]
    three = oracle.kneeded(np.array([[0.1, 0.5, 0.5], [0.3, 0.5, 0.5], [0.6, 0.5, 0.5]]), kcap=8, kwork=8)
    assert [int(three[k][0]) for k in ("tested", "evals", "created", "r2upd")] == [2, 16, 4, 8]
    # a list of one stops the count after the first plane
    one = oracle.kneeded(np.array([[0.1, 0.5, 0.5], [0.3, 0.5, 0.5], [0.6, 0.5, 0.5]]), kcap=8, kwork=1)
    assert [int(one[k][0]) for k in ("tested", "evals", "created", "r2upd")] == [1, 8, 4, 8]
    # the plane x + y + z = 3/2 through the cube's centre: 4 corners beyond it,
    # its hexagonal section adds 6 vertices, 10 remain
    c = oracle.kneeded(np.array([[0.05, 0.05, 0.05], [0.95, 0.95, 0.95]]), kcap=8, kwork=8)
    assert [int(c[k][0]) for k in ("tested", "evals", "created", "r2upd")] == [1, 8, 6, 10]


@pytest.mark.parametrize("kind,seed", [("uniform", 7), ("cluster", 8)])
def test_work_counters_against_halfspaces(kind, seed):
    """Every counter of the oracle's k_needed pass equals a Qhull replay."""
    P = getattr(gen, kind)(300, seed=seed, dtype=np.float64)
    cells = np.arange(0, 300, 15)
    for kwork in (8, 32):
        k = oracle.kneeded(P, cells=cells, kcap=kwork, kwork=kwork)
        got = list(zip(k["tested"].tolist(), k["evals"].tolist(), k["created"].tolist(), k["r2upd"].tolist()))
        ref = [_work_by_halfspaces(P, int(i), kwork) for i in cells]
        assert got == ref


def test_volume_ld_against_independent_long_double():
    """The oracle's long-double volume (vertices re-solved from their planes)
    equals an independent numpy long-double evaluation of the same cells
    (faces ordered by angle, fanned from their mean), tiles the box, and
    agrees with the double volume wherever the cell is not far smaller than
    the box; on cluster cores the double volume is the one that drifts."""
    from helpers import ld_volumes
    P = gen.cluster(6000, seed=31, dtype=np.float32, n_clusters=6).astype(np.float64)
    r = oracle.tessellate(P, volume_ld=True)
    v, vl = r["volume"], r["volume_ld"]
    assert abs(np.sum(vl) - 1.0) <= 1e-13
    drift = np.abs(v - vl) / vl
    off = np.nonzero(drift > 1e-12)[0]
    pick = np.unique(np.concatenate([off[:40], np.arange(0, len(P), 150)]))
    ref = ld_volumes(P, pick)
    assert np.max(np.abs(vl[pick] - ref) / ref) <= 1e-14
    # where the double volume drifts the cells are tiny next to the box
    big = vl > 1e-3 / len(P)
    assert np.all(drift[big] <= 1e-12)


# ------------------------------------------------------------ periodic boxes

def _periodic_rows(r):
    return [sorted(int(x) for x in row) for row in oracle.rows(r)]


def test_periodic_closed_forms():
    """One point: its cell is the box, with its six own images as neighbours
    (also in an anisotropic box); two points split along x: two slabs of
    half the volume, each with its two images of the other point and its own
    four y/z images; simple-cubic and BCC lattices: cubes of 1/m^3 with 6
    neighbours and truncated octahedra of a^3 / 2 with 14, for EVERY cell."""
    r = oracle.tessellate(np.array([[0.3, 0.4, 0.5]]), periodic=True)
    assert r["volume"].tolist() == [1.0] and _periodic_rows(r) == [[0] * 6]
    r = oracle.tessellate(np.array([[0.3, 0.4, 0.5]]), lo=(0, 0, 0), hi=(1, 2, 0.6), periodic=True)
    np.testing.assert_allclose(r["volume"], [1.2], rtol=1e-15)
    assert _periodic_rows(r) == [[0] * 6]
    r = oracle.tessellate(np.array([[0.1, 0.5, 0.5], [0.6, 0.5, 0.5]]), periodic=True)
    np.testing.assert_allclose(r["volume"], [0.5, 0.5], rtol=1e-15)
    assert _periodic_rows(r) == [[0, 0, 0, 0, 1, 1], [0, 0, 1, 1, 1, 1]]
    m = 4
    g = (np.arange(m) + 0.25) / m
    P = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T
    r = oracle.tessellate(P, periodic=True, volume_ld=True)
    np.testing.assert_allclose(r["volume_ld"], 1 / m ** 3, rtol=1e-14)
    assert set(np.diff(r["row_ptr"]).tolist()) == {6}
    a = 0.25
    base = np.array(np.meshgrid(*[np.arange(4)] * 3, indexing="ij")).reshape(3, -1).T * a + 0.0625
    P = np.concatenate([base, base + a / 2])
    r = oracle.tessellate(P, periodic=True)
    np.testing.assert_allclose(r["volume"], a ** 3 / 2, rtol=1e-13)
    assert set(np.diff(r["row_ptr"]).tolist()) == {14}


@pytest.mark.parametrize("kind,seed", [("uniform", 41), ("cluster", 42)])
def test_periodic_invariants(kind, seed):
    """Volumes tile the torus; the neighbour relation is symmetric with
    multiplicity; translating every point by t (mod L) changes no neighbour
    set and moves volumes by rounding only.  (FP32-rounded points and a
    dyadic t, so that the translated set is exact in double.)"""
    P = getattr(gen, kind)(6000, seed=seed, dtype=np.float32).astype(np.float64)
    r = oracle.tessellate(P, periodic=True, volume_ld=True)
    assert abs(np.sum(r["volume_ld"]) - 1.0) <= 1e-13
    assert abs(np.sum(r["volume"]) - 1.0) <= 1e-12
    src = np.repeat(np.arange(len(P)), np.diff(r["row_ptr"]))
    fwd = np.sort(src * len(P) + r["col"])
    bwd = np.sort(r["col"].astype(np.int64) * len(P) + src)
    assert np.array_equal(fwd, bwd)
    t = np.array([0.375, 0.125, 0.6875])
    r2 = oracle.tessellate((P + t) % 1.0, periodic=True, volume_ld=True)
    assert _periodic_rows(r2) == _periodic_rows(r)
    np.testing.assert_allclose(r2["volume_ld"], r["volume_ld"], rtol=1e-11)


def _periodic_cell_qhull(P, i, span=2):
    """The periodic cell of point i from Qhull: the intersection of the
    bisectors of p_i with every image p_j + m (m in {-span..span}^3, unit
    box) -- enough for the point counts used here -- with its neighbour
    multiset (the point index of each plane holding at least three vertices)."""
    from scipy.spatial import ConvexHull, HalfspaceIntersection
    rng = range(-span, span + 1)
    shifts = np.array([(a, b, c) for a in rng for b in rng for c in rng], dtype=np.float64)
    Q = (P[None, :, :] + shifts[:, None, :]).reshape(-1, 3)
    owner = np.tile(np.arange(len(P)), len(shifts))
    keep = np.any(Q != P[i], axis=1)
    Q, owner = Q[keep], owner[keep]
    ns = Q - P[i]
    cs = 0.5 * np.sum(ns ** 2, axis=1)
    H = HalfspaceIntersection(np.hstack([ns, -cs[:, None]]), np.zeros(3))
    vol = ConvexHull(H.intersections).volume
    act = np.abs(H.intersections @ ns.T - cs) <= 1e-9 * np.linalg.norm(ns, axis=1)
    faces = sorted(int(owner[f]) for f in np.nonzero(act.sum(0) >= 3)[0])
    return vol, faces


@pytest.mark.parametrize("seed", range(12))
def test_periodic_against_all_images(seed):
    """Every cell of a small periodic set against Qhull over all images within
    two periods: volumes and neighbour multisets."""
    rng = np.random.default_rng(500 + seed)
    n = [3, 5, 8, 13, 21, 34][seed % 6]
    P = rng.random((n, 3))
    r = oracle.tessellate(P, periodic=True)
    rows = _periodic_rows(r)
    for i in range(n):
        vol, faces = _periodic_cell_qhull(P, i)
        assert abs(vol - r["volume"][i]) <= 1e-10 * vol
        assert faces == rows[i], (seed, i)


def test_periodic_poisson_voronoi_mean_faces():
    """With no boundary every cell counts: the mean face count of a Poisson-
    Voronoi tessellation, 2 + 48 pi^2 / 35 = 15.535 (Meijering)."""
    P = gen.uniform(40_000, seed=43, dtype=np.float64)
    r = oracle.tessellate(P, periodic=True)
    mean = np.diff(r["row_ptr"]).mean()
    assert abs(mean - (2 + 48 * np.pi ** 2 / 35)) <= 0.06, mean
