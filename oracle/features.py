"""The learned-k network's 12 input features, computed from their definitions
(test infrastructure only; numpy + scipy's k-d tree for the 16 nearest).

For a point p with nearest neighbours q_1..q_16 (distances d_1 <= ... <= d_16),
l = (box volume / N)^(1/3) and the uniform grid of about 2 points per cell
(g_a = max(1, round(ext_a (N / (2 vol))^(1/3))), cell = clamp(floor((x - lo)
g / ext), 0, g - 1)):

  f1..f3  log2(1 + n_s / (nbar * c_s)), s = 0, 1, 2: n_s points in the
          (2s+1)^3 block of grid cells around p's cell (clipped to the grid,
          c_s cells), nbar = N / G
  f4..f6  log2(d_4 / l), log2(d_8 / l), log2(d_16 / l)
  f7      |mean of the offsets q_i - p| / d_16
  f8      log2(d_1 / l)
  f9..f11 eigenvalues of the offsets' covariance (mean removed, 1/16
          normalisation), largest first, divided by their sum
  f12     min(distance from p to the nearest box wall / d_16, 4)
"""
from __future__ import annotations

import numpy as np

NFEAT = 12


def grid_dims(n, lo, hi, pts_per_cell=2.0):
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    ext = hi - lo
    scale = np.cbrt(max(n, 1) / (pts_per_cell * np.prod(ext)))
    return np.maximum(1, np.rint(ext * scale)).astype(np.int64)


def features(points, lo=(0, 0, 0), hi=(1, 1, 1), rows=None, nbr=None) -> np.ndarray:
    """Features of points[rows] (all points by default).  The 16 nearest come
    from a k-d tree in double, or, with ``nbr`` ([len(rows), 16] point indices
    in ascending order of distance), from that list: the features of a given
    neighbour list, for lists whose order at equal float distances is fixed
    by another rule."""
    from scipy.spatial import cKDTree

    P = np.asarray(points, dtype=np.float64)
    n = len(P)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    ext = hi - lo
    g = grid_dims(n, lo, hi)
    G = int(np.prod(g))
    c = np.clip(np.floor((P - lo) * (g / ext)), 0, g - 1).astype(np.int64)
    counts = np.zeros(tuple(g[::-1]), dtype=np.int64)  # [z, y, x]
    np.add.at(counts, (c[:, 2], c[:, 1], c[:, 0]), 1)
    cum = np.zeros(tuple(g[::-1] + 1), dtype=np.int64)  # 3-D prefix sums for block counts
    cum[1:, 1:, 1:] = counts.cumsum(0).cumsum(1).cumsum(2)
    nbar = n / G
    ell = np.cbrt(np.prod(ext) / n)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    if nbr is None:
        tree = cKDTree(P)
        kq = min(17, n)
        dist, idx = tree.query(P[rows], k=kq)
        dist, idx = dist.reshape(len(rows), kq)[:, 1:], idx.reshape(len(rows), kq)[:, 1:]
    else:
        idx = np.asarray(nbr, dtype=np.int64)
        dist = np.sqrt(((P[idx] - P[rows][:, None, :]) ** 2).sum(-1))
    F = np.zeros((len(rows), NFEAT))
    cr = c[rows]
    for s in range(3):
        a = np.maximum(cr - s, 0)
        b = np.minimum(cr + s, g - 1) + 1
        tot = (cum[b[:, 2], b[:, 1], b[:, 0]] - cum[a[:, 2], b[:, 1], b[:, 0]] - cum[b[:, 2], a[:, 1], b[:, 0]]
               - cum[b[:, 2], b[:, 1], a[:, 0]] + cum[a[:, 2], a[:, 1], b[:, 0]] + cum[a[:, 2], b[:, 1], a[:, 0]]
               + cum[b[:, 2], a[:, 1], a[:, 0]] - cum[a[:, 2], a[:, 1], a[:, 0]])
        ncell = np.prod(b - a, axis=1)
        F[:, s] = np.log2(1.0 + tot / (nbar * ncell))
    m = dist.shape[1]
    d = lambda i: dist[:, min(i, m) - 1]  # noqa: E731
    F[:, 3] = np.log2(d(4) / ell)
    F[:, 4] = np.log2(d(8) / ell)
    F[:, 5] = np.log2(d(16) / ell)
    off = P[idx] - P[rows][:, None, :]
    mu = off.mean(axis=1)
    F[:, 6] = np.linalg.norm(mu, axis=1) / d(16)
    F[:, 7] = np.log2(d(1) / ell)
    cen = off - mu[:, None, :]
    cov = np.einsum("nki,nkj->nij", cen, cen) / m
    ev = np.linalg.eigvalsh(cov)[:, ::-1]
    tr = ev.sum(axis=1, keepdims=True)
    F[:, 8:11] = np.where(tr > 0, ev / np.where(tr > 0, tr, 1.0), 1.0 / 3.0)
    wall = np.minimum(P[rows] - lo, hi - P[rows]).min(axis=1)
    F[:, 11] = np.minimum(wall / d(16), 4.0)
    return F
