"""The margin behind the stream phase's vertex pruning, checked in the
arithmetic the float clip uses.  A float vertex v with per-axis error bound e
stands for a true vertex c with |c_a - v_a| <= e; the ball through the seed
centred at c has radius |c| and reaches |q| <= 2 |c| from the seed.  The
kernel widens the radius to rad = |v| (1 + 1e-5) + 4 e (in float) and leaves
the vertex out when rad < rlim = float(sqrt(d_k^2 (1 - 1e-6)) / 2 (1 - 1e-6)).
Such a ball must hold list members only: 2 |c| < sqrt(d_k^2 (1 - 1e-6)), the
radius of the ball whose points are list members after the rounding of d^2."""
import numpy as np

f32 = np.float32


def rad_f32(v, e):
    x, y, z = (f32(t) for t in v)
    n = np.sqrt(f32(x * x + y * y) + f32(z * z), dtype=f32)
    return f32(f32(n * f32(1.0 + 1e-5)) + f32(f32(4.0) * f32(e)))


def rlim_f32(dk2):
    dk2in = float(dk2) * (1.0 - 1e-6)
    return f32(0.5 * np.sqrt(dk2in) * (1.0 - 1e-6))


def worst_c_norm(v, e):
    # the largest |c| over the box |c_a - v_a| <= e: each axis pushed away
    # from the seed
    c = np.abs(np.asarray(v, dtype=np.longdouble)) + np.longdouble(float(e))
    return np.sqrt(np.sum(c * c))


def test_pruned_balls_stay_inside_the_list_ball():
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(20000):
        v = (rng.standard_normal(3) * 10.0 ** rng.uniform(-4, 0)).astype(f32)
        e = f32(abs(v).max() * 10.0 ** rng.uniform(-8, -4.8))  # up to 16 eps |v|
        rad = rad_f32(v, e)
        # list distances from one to three radii, and just above the pruning
        # threshold, where the margin is thinnest: 2 rad (1 + s)
        ts = list(rng.uniform(1.0, 3.0, 3)) + [2.0 * (1.0 + s) for s in (1e-9, 1e-7, 1e-6, 3e-6, 1e-5)]
        for t in ts:
            dk2 = f32((float(rad) * t) ** 2)
            if not rad < rlim_f32(dk2):
                continue
            checked += 1
            assert 2 * worst_c_norm(v, e) < np.sqrt(np.longdouble(float(dk2)) * np.longdouble(1 - 1e-6))
    assert checked > 10000


def test_vertices_reaching_the_list_ball_are_kept():
    # a vertex whose true ball reaches past the list's ball is never left out
    rng = np.random.default_rng(8)
    for _ in range(20000):
        v = (rng.standard_normal(3) * 10.0 ** rng.uniform(-4, 0)).astype(f32)
        e = f32(abs(v).max() * 10.0 ** rng.uniform(-8, -4.8))
        two_c = 2 * float(np.sqrt(np.sum(np.asarray(v, np.float64) ** 2)))
        dk2 = f32((two_c * (1.0 - 1e-7)) ** 2)  # the ball of c = v reaches past it
        assert not rad_f32(v, e) < rlim_f32(dk2)


def d2_f32(q, p):
    # the clip's float d^2: each coordinate difference rounded to float, each
    # square rounded, (x^2 + y^2) + z^2 with no fused multiply-add
    dx, dy, dz = (f32(f32(a) - f32(b)) for a, b in zip(q, p))
    return f32(f32(f32(dx * dx) + f32(dy * dy)) + f32(dz * dz))


def test_float_d2_within_the_list_ball_margin():
    # a box skipped as inside the list's ball, d^2 < d_k^2 (1 - 1e-6) in exact
    # arithmetic, holds only points whose float d^2 is below the list's float
    # d_k^2: the float d^2 is within 1e-6 relative of the exact one
    rng = np.random.default_rng(9)
    p = rng.uniform(0, 1, (50000, 3)).astype(f32)
    q = (p.astype(np.float64) + rng.standard_normal((50000, 3)) * 10.0 ** rng.uniform(-5, -1, (50000, 1)))
    q = np.clip(q, 0, 1).astype(f32)
    exact = np.sum((q.astype(np.float64) - p.astype(np.float64)) ** 2, axis=1)
    got = np.array([d2_f32(a, b) for a, b in zip(q, p)], dtype=np.float64)
    keep = exact > 0
    rel = np.abs(got[keep] - exact[keep]) / exact[keep]
    assert rel.max() < 1e-6 / 2
