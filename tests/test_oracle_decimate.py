"""Pins of the oracle's Visvalingam-Whyatt polyline decimation (Sec. 3.1: straight runs of
densely sampled road polylines are thinned by removing the points of least effective
area): a brute force that recomputes every area from scratch on tiny polylines, straight
lines, the stopping invariant, the triangle area against the shoelace formula, and the
directions of the kept points."""
import math

import numpy as np
import pytest


def _area32(x, y, a, b, c):
    f = np.float32
    ux, uy = f(x[b] - x[a]), f(y[b] - y[a])
    vx, vy = f(x[c] - x[a]), f(y[c] - y[a])
    return f(0.5) * abs(f(f(ux * vy) - f(uy * vx)))


def _brute(x, y, min_area):
    """Visvalingam-Whyatt by definition: recompute the area of every interior point of the
    current polyline, drop the smallest (first on ties) while it is below min_area."""
    alive = list(range(len(x)))
    while len(alive) > 2:
        areas = [_area32(x, y, alive[j - 1], alive[j], alive[j + 1]) for j in range(1, len(alive) - 1)]
        j = int(np.argmin(areas))
        if not areas[j] < np.float32(min_area):
            break
        del alive[j + 1]
    keep = np.zeros(len(x), np.uint8)
    keep[alive] = 1
    return keep


def test_matches_brute_force_on_tiny_polylines(oracle_mod):
    rng = np.random.default_rng(0)
    polys, xs, ys, off = [], [], [], [0]
    for _ in range(400):
        n = int(rng.integers(1, 13))
        x = rng.normal(0, 3, n).cumsum()
        y = rng.normal(0, 1, n).cumsum()
        if rng.random() < 0.3:  # some exactly collinear runs and repeated points
            y[: n // 2] = 0.0
            x[: n // 2] = np.arange(n // 2)
        if rng.random() < 0.2 and n > 3:
            x[2], y[2] = x[1], y[1]
        xs.append(x.astype(np.float32)); ys.append(y.astype(np.float32))
        off.append(off[-1] + n)
    x, y = np.concatenate(xs), np.concatenate(ys)
    for min_area in (0.0, 0.05, 0.7, 4.0):
        keep, _ = oracle_mod.decimate(off, x, y, min_area)
        want = np.concatenate([_brute(xs[i], ys[i], min_area) for i in range(len(xs))])
        np.testing.assert_array_equal(keep, want)
        assert keep[np.array(off[:-1])].all() and keep[np.array(off[1:]) - 1].all()  # end points


def test_straight_lines_keep_only_their_ends(oracle_mod):
    n = 500
    t = np.arange(n, dtype=np.float64) * 0.1
    off = [0, n, 2 * n]
    x = np.concatenate([t, np.full(n, 3.0)]).astype(np.float32)
    y = np.concatenate([np.zeros(n), t]).astype(np.float32)
    keep, dr = oracle_mod.decimate(off, x, y, 1e-6)
    assert keep.sum() == 4 and keep[[0, n - 1, n, 2 * n - 1]].all()
    np.testing.assert_allclose(dr[[0, n - 1]], 0.0, atol=1e-12)
    np.testing.assert_allclose(dr[[n, 2 * n - 1]], math.pi / 2, atol=1e-12)
    keep0, _ = oracle_mod.decimate(off, x, y, 0.0)
    assert keep0.all()  # nothing has an area below 0


def test_stop_rule_and_directions(oracle_mod):
    """After decimation every kept interior point spans at least min_area with its kept
    neighbours, and each kept point's direction points at the next kept point."""
    rng = np.random.default_rng(1)
    n = 3000
    s = np.linspace(0, 300, n)
    x = (s + rng.normal(0, 0.01, n)).astype(np.float32)
    y = (20 * np.sin(s / 40) + rng.normal(0, 0.01, n)).astype(np.float32)
    for min_area in (0.01, 0.5):
        keep, dr = oracle_mod.decimate([0, n], x, y, min_area)
        k = np.flatnonzero(keep)
        assert 2 < len(k) < n
        areas = [_area32(x, y, k[j - 1], k[j], k[j + 1]) for j in range(1, len(k) - 1)]
        assert min(areas) >= np.float32(min_area)
        want = np.arctan2(np.diff(y[k].astype(np.float64)), np.diff(x[k].astype(np.float64)))
        np.testing.assert_allclose(dr[k[:-1]], want, atol=1e-12)
        np.testing.assert_allclose(dr[k[-1]], want[-1], atol=1e-12)
        print("min_area %.2f: %d of %d points kept" % (min_area, len(k), n))


@pytest.mark.parametrize("seed", range(5))
def test_area_is_the_triangle_area(oracle_mod, seed):
    """The binary32 area agrees with the FP64 shoelace area: a three-point polyline loses
    its middle point exactly when min_area exceeds the area (away from rounding)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-50, 50, (3, 2))
    area = 0.5 * abs((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[1, 1] - p[0, 1]) * (p[2, 0] - p[0, 0]))
    x, y = p[:, 0].astype(np.float32), p[:, 1].astype(np.float32)
    a64 = 0.5 * abs((float(x[1]) - x[0]) * (float(y[2]) - y[0]) - (float(y[1]) - y[0]) * (float(x[2]) - x[0]))
    assert abs(a64 - area) < 1e-3 * max(area, 1.0)
    lo, _ = oracle_mod.decimate([0, 3], x, y, a64 * (1 - 1e-5))
    hi, _ = oracle_mod.decimate([0, 3], x, y, a64 * (1 + 1e-5))
    assert lo.tolist() == [1, 1, 1] and hi.tolist() == [1, 0, 1]
