"""Seeded synthetic point sets for the cell-by-cell Voronoi path.

This module only draws random numbers and rounds them; it holds none of the
tessellation arithmetic.  Both the GPU path and the CPU oracle take their
inputs from here, so the two sides always see the same arrays.

The paper measures on no public dataset; its only workload statement is that
the method targets "large datasets" (Performance section).  The sets below
are the synthetic stand-ins used throughout this project:

* ``uniform``   i.i.d. uniform points in the unit cube;
* ``cluster``   a mixture of isotropic Gaussians (centres uniform, sigma
                log-uniform) plus a uniform background;
* ``filament``  points scattered around random line segments plus a uniform
                background.

Every generator draws in float64 with numpy's PCG64 ``default_rng(seed)``,
rounds once to the requested dtype, rejects and redraws points that fall
outside ``[0, 1)^3`` after rounding, redraws exact duplicate rows, and finally
shuffles the rows so that the input is spatially unordered.
"""
from __future__ import annotations

import numpy as np

__all__ = ["uniform", "cluster", "filament", "make", "WORKLOADS"]


def _inside(p: np.ndarray) -> np.ndarray:
    return np.all((p >= 0.0) & (p < 1.0), axis=1)


def _dup_mask(p: np.ndarray) -> np.ndarray:
    """True for every row that repeats an earlier row (exact bit equality)."""
    n = p.shape[0]
    dup = np.zeros(n, dtype=bool)
    if n < 2:
        return dup
    if p.dtype == np.float32:
        b = np.ascontiguousarray(p).view(np.uint32).reshape(-1, 3)
        key = (b[:, 0].astype(np.uint64) << np.uint64(32)) | b[:, 1].astype(np.uint64)
        order = np.argsort(key, kind="stable")
        ks = key[order]
        same = ks[1:] == ks[:-1]
        if not same.any():
            return dup
        # rows sharing (x, y): settle on z among them only
        idx = np.unique(np.concatenate([order[1:][same], order[:-1][same]]))
        sub = _dup_mask_lex(b[idx])
        dup[idx[sub]] = True
        return dup
    return _dup_mask_lex(np.ascontiguousarray(p).view(np.uint64).reshape(-1, 3))


def _dup_mask_lex(b: np.ndarray) -> np.ndarray:
    order = np.lexsort((b[:, 2], b[:, 1], b[:, 0]))
    s = b[order]
    same = np.all(s[1:] == s[:-1], axis=1)
    dup = np.zeros(b.shape[0], dtype=bool)
    dup[order[1:][same]] = True
    return dup


def _finish(rng, draw, n: int, dtype) -> np.ndarray:
    """Round to dtype, redraw rejects (outside the cube) and duplicates, shuffle."""
    out = draw(n).astype(dtype)

    def redraw_outside(rows):
        for _ in range(1000):
            bad = rows[~_inside(out[rows])]
            if bad.size == 0:
                return
            out[bad] = draw(bad.size).astype(dtype)
            rows = bad
        raise RuntimeError("could not draw in-box points")  # pragma: no cover

    redraw_outside(np.arange(n))
    for _ in range(100):
        dup = np.nonzero(_dup_mask(out))[0]
        if dup.size == 0:
            break
        out[dup] = draw(dup.size).astype(dtype)
        redraw_outside(dup)
    else:  # pragma: no cover - would need an absurd generator
        raise RuntimeError("could not draw a duplicate-free set")
    return out[rng.permutation(n)]


def uniform(n: int, seed: int = 0, dtype=np.float32) -> np.ndarray:
    """``n`` i.i.d. uniform points in the unit cube."""
    rng = np.random.default_rng(seed)
    return _finish(rng, lambda m: rng.random((m, 3)), n, dtype)


def cluster(n: int, seed: int = 0, dtype=np.float32, n_clusters: int = 4096,
            log10_sigma=(-4.0, -2.0), background: float = 0.1) -> np.ndarray:
    """Gaussian-mixture points plus a uniform background.

    Centres are uniform in the unit cube, each cluster's sigma is
    ``10**U(log10_sigma)``, cluster labels are uniform over the clusters, and
    ``round(background * n)`` points are uniform.  A point that lands outside
    the cube is redrawn (same procedure, fresh label).
    """
    rng = np.random.default_rng(seed)
    centres = rng.random((n_clusters, 3))
    sigma = 10.0 ** rng.uniform(log10_sigma[0], log10_sigma[1], n_clusters)
    n_bg = int(round(background * n))

    def draw_cl(m):
        lab = rng.integers(0, n_clusters, m)
        return centres[lab] + sigma[lab, None] * rng.standard_normal((m, 3))

    def draw(m):
        # during redraws keep the background / cluster split proportional
        m_bg = int(round(background * m)) if m != n else n_bg
        return np.concatenate([rng.random((m_bg, 3)), draw_cl(m - m_bg)])

    return _finish(rng, draw, n, dtype)


def filament(n: int, seed: int = 0, dtype=np.float32, n_segments: int = 20000,
             frac: float = 0.6, sigma: float = 2e-4) -> np.ndarray:
    """Points scattered around random segments plus a uniform background.

    Segment endpoints are uniform in the cube; a filament point picks a segment
    uniformly, a parameter ``t ~ U[0, 1]`` along it, and adds a 2-D Gaussian
    offset (std ``sigma``) perpendicular to the segment.
    """
    rng = np.random.default_rng(seed)
    a = rng.random((n_segments, 3))
    b = rng.random((n_segments, 3))
    d = b - a
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # two unit vectors perpendicular to each segment
    helper = np.where(np.abs(d[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    u = np.cross(d, helper)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(d, u)
    n_fil = int(round(frac * n))

    def draw_fil(m):
        s = rng.integers(0, n_segments, m)
        t = rng.random(m)[:, None]
        g = sigma * rng.standard_normal((m, 2))
        return a[s] + t * (b[s] - a[s]) + g[:, :1] * u[s] + g[:, 1:] * v[s]

    def draw(m):
        m_fil = int(round(frac * m)) if m != n else n_fil
        return np.concatenate([draw_fil(m_fil), rng.random((m - m_fil, 3))])

    return _finish(rng, draw, n, dtype)


# Named workloads: (generator, n, dtype).  The sizes follow the paper's
# framing of large point sets; the small one is sized for the CPU oracle.
WORKLOADS = {
    "uniform-10k-f64": (uniform, 10_000, np.float64),
    "uniform-1m-f32": (uniform, 1 << 20, np.float32),
    "cluster-4m-f32": (cluster, 1 << 22, np.float32),
    "cluster-16m-f32": (cluster, 1 << 24, np.float32),
    "uniform-16m-f32": (uniform, 1 << 24, np.float32),
    "filament-64m-f32": (filament, 1 << 26, np.float32),
}


def make(name: str, seed: int = 0) -> np.ndarray:
    fn, n, dt = WORKLOADS[name]
    return fn(n, seed=seed, dtype=dt)
