"""Pins of the learned-k oracle (network + features); CPU only."""
import numpy as np
import pytest
import torch

from oracle import features as ofeat
from oracle import mlp


def _batch(seed, B=64):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(B, 12)) * 2 + 1
    y = rng.integers(0, 7, size=B)
    mean, std = x.mean(0), x.std(0) + 0.1
    return x, y, mean, std


def test_nparam():
    assert mlp.NPARAM == 5447


def test_fp64_gradient_matches_finite_differences():
    x, y, mean, std = _batch(0)
    theta = mlp.init_params(1) + np.random.default_rng(2).normal(scale=0.05, size=mlp.NPARAM)
    _, g = mlp.loss_and_grad(theta, x, y, mean, std, bf16_points=False)
    rng = np.random.default_rng(3)
    idx = rng.choice(mlp.NPARAM, 200, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = mlp.loss_and_grad(tp, x, y, mean, std, bf16_points=False)
        lm, _ = mlp.loss_and_grad(tm, x, y, mean, std, bf16_points=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, 10000), [0.0, -0.0, 1.0, 65504.0]])
    ours = mlp.bf16(x)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_bf16_forward_close_to_fp64():
    x, y, mean, std = _batch(5, B=256)
    theta = mlp.init_params(6)
    a, _ = mlp.forward(theta, x, mean, std, bf16_points=True)
    b, _ = mlp.forward(theta, x, mean, std, bf16_points=False)
    assert np.max(np.abs(a - b)) < 0.05 * np.max(np.abs(b)) + 1e-3


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    th = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=50)
        th, m, v = mlp.adam_step(th, g, m, v, t)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_choose_threshold_rule():
    theta = np.zeros(mlp.NPARAM)
    # zero weights: uniform softmax, P(label <= b) = (b + 1) / 7
    b3 = np.zeros(7)
    parts = mlp.unpack(theta)
    parts["b3"] = b3
    th = mlp.pack(parts)
    x = np.zeros((3, 12))
    for tau, want in [(0.1, 0), (0.5, 3), (0.99, 6), (1.0, 6)]:
        assert mlp.choose(th, x, np.zeros(12), np.ones(12), tau).tolist() == [want] * 3


def _brute_features(P, i, lo, hi):
    n = len(P)
    d = np.sqrt(((P - P[i]) ** 2).sum(1))
    d[i] = np.inf
    order = np.argsort(d, kind="stable")[:16]
    ds = d[order]
    g = ofeat.grid_dims(n, lo, hi)
    ext = np.asarray(hi, float) - np.asarray(lo, float)
    cell = np.clip(np.floor((P - lo) * g / ext), 0, g - 1).astype(int)
    f = np.zeros(12)
    nbar = n / np.prod(g)
    for s in range(3):
        inblk = np.all(np.abs(cell - cell[i]) <= s, axis=1)
        ncell = 1
        for a in range(3):
            ncell *= min(cell[i, a] + s, g[a] - 1) - max(cell[i, a] - s, 0) + 1
        f[s] = np.log2(1 + inblk.sum() / (nbar * ncell))
    ell = (np.prod(ext) / n) ** (1 / 3)
    f[3], f[4], f[5], f[7] = [np.log2(ds[k - 1] / ell) for k in (4, 8, 16, 1)]
    off = P[order] - P[i]
    mu = off.mean(0)
    f[6] = np.linalg.norm(mu) / ds[15]
    C = np.zeros((3, 3))
    for o in off:
        C += np.outer(o - mu, o - mu)
    C /= 16
    ev = np.sort(np.linalg.eigvalsh(C))[::-1]
    f[8:11] = ev / ev.sum()
    f[11] = min(min((P[i] - lo).min(), (hi - P[i]).min()) / ds[15], 4.0)
    return f


def test_features_against_brute_force():
    rng = np.random.default_rng(8)
    P = np.concatenate([rng.random((300, 3)), 0.3 + 0.01 * rng.normal(size=(100, 3))])
    P = np.clip(P, 0, 1)
    rows = np.arange(0, 400, 7)
    F = ofeat.features(P, rows=rows)
    for k, i in enumerate(rows):
        np.testing.assert_allclose(F[k], _brute_features(P, i, np.zeros(3), np.ones(3)), rtol=1e-10, atol=1e-12)


def test_features_of_a_given_list():
    """With the k-d tree's own 16-nearest list passed in, the list path gives
    the same features; a list in another order of equal distances moves only
    the order-free features' rounding."""
    rng = np.random.default_rng(9)
    P = np.concatenate([rng.random((300, 3)), 0.6 + 0.02 * rng.normal(size=(100, 3))])
    P = np.clip(P, 0, 1)
    rows = np.arange(0, 400, 5)
    d2 = ((P[rows][:, None, :] - P[None, :, :]) ** 2).sum(-1)
    d2[np.arange(len(rows)), rows] = np.inf
    nbr = np.argsort(d2, axis=1, kind="stable")[:, :16]
    np.testing.assert_allclose(ofeat.features(P, rows=rows, nbr=nbr), ofeat.features(P, rows=rows),
                               rtol=1e-12, atol=1e-14)
    # the first 15 reversed: d_4, d_8 and d_1 read other entries, the rest is order-free
    rev = np.concatenate([nbr[:, :15][:, ::-1], nbr[:, 15:]], axis=1)
    a, b = ofeat.features(P, rows=rows, nbr=rev), ofeat.features(P, rows=rows)
    keep = [0, 1, 2, 5, 6, 8, 9, 10, 11]
    np.testing.assert_allclose(a[:, keep], b[:, keep], rtol=1e-10, atol=1e-12)
    assert not np.allclose(a[:, 3], b[:, 3])


def test_features_closed_forms():
    # two points in every grid cell of a 6^3 grid: block occupancy ratio 1 -> log2(2)
    g = 6
    c = (np.arange(g) + 0.25) / g
    A = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    P = np.concatenate([A, A + 0.5 / g])
    F = ofeat.features(P)
    np.testing.assert_allclose(F[:, :3], 1.0, atol=1e-12)
    # points on a line: covariance of rank one
    t = np.linspace(0.1, 0.9, 41)
    L = np.stack([t, 0.5 + 0 * t, 0.5 + 0 * t], 1)
    F = ofeat.features(L, rows=[20])
    np.testing.assert_allclose(F[0, 8:11], [1.0, 0.0, 0.0], atol=1e-12)
    assert abs(F[0, 6]) < 1e-12  # symmetric neighbourhood: zero mean offset
    # nearest wall at 0.5 over d_16 = 8 * 0.02
    assert abs(F[0, 11] - 0.5 / 0.16) < 1e-9
    F = ofeat.features(L, rows=[2])  # near the x- wall: 0.14 / d_16
    assert F[0, 11] < 4.0
