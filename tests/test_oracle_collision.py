"""Pins of the oracle's oriented-box collision (Sec. 3.1: convex objects, candidate
pairs; Sec. 3.2 "Termination": vehicles collide with road edges).

The separating-axis value is checked against an independent brute force (two convex
polygons intersect iff some pair of edges properly crosses or a vertex of one lies
strictly inside the other), against closed forms for axis-aligned boxes, and against
hand-derived cases in tests/golden/collision_cases.json.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "collision_cases.json")


def corners(b):
    cx, cy, yaw, L, W = b
    c = complex(cx, cy)
    r = complex(math.cos(yaw), math.sin(yaw))
    return [c + r * complex(sx * L / 2, sy * W / 2) for sx, sy in ((1, 1), (-1, 1), (-1, -1), (1, -1))]


def orient(a, b, c):
    return ((b - a).conjugate() * (c - a)).imag


def seg_cross(p1, p2, q1, q2):
    d1, d2 = orient(q1, q2, p1), orient(q1, q2, p2)
    d3, d4 = orient(p1, p2, q1), orient(p1, p2, q2)
    return d1 * d2 < 0 and d3 * d4 < 0


def inside(poly, p):
    s = [orient(poly[k], poly[(k + 1) % len(poly)], p) for k in range(len(poly))]
    return all(v > 0 for v in s) or all(v < 0 for v in s)


def brute_boxes(a, b):
    pa, pb = corners(a), corners(b)
    for i in range(4):
        for j in range(4):
            if seg_cross(pa[i], pa[(i + 1) % 4], pb[j], pb[(j + 1) % 4]):
                return True
    return any(inside(pa, p) for p in pb) or any(inside(pb, p) for p in pa)


def brute_box_seg(a, s0, s1):
    pa = corners(a)
    if any(seg_cross(pa[i], pa[(i + 1) % 4], s0, s1) for i in range(4)):
        return True
    return inside(pa, s0) or inside(pa, s1)


def test_box_box_sat_vs_bruteforce(oracle_mod):
    rng = np.random.default_rng(1)
    n_hit = n_miss = 0
    for _ in range(4000):
        a = [rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-4, 4), rng.uniform(1, 6), rng.uniform(0.5, 3)]
        b = [rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-4, 4), rng.uniform(1, 6), rng.uniform(0.5, 3)]
        sep = oracle_mod.box_box_sep(a, b)
        sep2 = oracle_mod.box_box_sep(b, a)
        assert abs(sep - sep2) < 1e-12  # symmetric
        if abs(sep) < 1e-6:
            continue
        want = brute_boxes(a, b)
        assert (sep < 0) == want, (a, b, sep)
        n_hit += want
        n_miss += not want
    assert n_hit > 500 and n_miss > 500


def test_box_seg_sat_vs_bruteforce(oracle_mod):
    rng = np.random.default_rng(2)
    n_hit = n_miss = 0
    for _ in range(4000):
        a = [rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(-4, 4), rng.uniform(1, 6), rng.uniform(0.5, 3)]
        s0 = complex(rng.uniform(-5, 5), rng.uniform(-5, 5))
        s1 = s0 + complex(rng.uniform(-4, 4), rng.uniform(-4, 4))
        sep = oracle_mod.box_seg_sep(a, s0.real, s0.imag, s1.real, s1.imag)
        sep_rev = oracle_mod.box_seg_sep(a, s1.real, s1.imag, s0.real, s0.imag)
        assert abs(sep - sep_rev) < 1e-12
        if abs(sep) < 1e-6:
            continue
        want = brute_box_seg(a, s0, s1)
        assert (sep < 0) == want, (a, s0, s1, sep)
        n_hit += want
        n_miss += not want
    assert n_hit > 500 and n_miss > 500


def test_axis_aligned_closed_forms(oracle_mod):
    """Axis-aligned boxes: overlap -> sep = -min(overlap_x, overlap_y) (penetration
    depth); separated along x only -> sep = gap."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        L1, W1, L2, W2 = rng.uniform(1, 5, 4)
        dx, dy = rng.uniform(-6, 6, 2)
        a, b = [0, 0, 0, L1, W1], [dx, dy, 0, L2, W2]
        gx = abs(dx) - (L1 + L2) / 2
        gy = abs(dy) - (W1 + W2) / 2
        np.testing.assert_allclose(oracle_mod.box_box_sep(a, b), max(gx, gy), atol=1e-12)
        # a quarter turn of both boxes swaps the roles of L and W, nothing else
        a90, b90 = [0, 0, math.pi / 2, W1, L1], [dx, dy, math.pi / 2, W2, L2]
        np.testing.assert_allclose(oracle_mod.box_box_sep(a90, b90), max(gx, gy), atol=1e-12)


def test_golden_cases(oracle_mod):
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        if c["kind"] == "box_box":
            got = oracle_mod.box_box_sep(c["a"], c["b"])
        else:
            got = oracle_mod.box_seg_sep(c["a"], *c["seg"])
        assert abs(got - c["sep"]) < 1e-9, (c["name"], got, c["sep"])
        assert (got < 0) == c["collide"], c["name"]


def _tiny_world(agents, segs, lanes=()):
    from tests._util import tiny_world
    return tiny_world(agents, edges=segs, lanes=lanes)


def test_world_flags_pairs_and_edges(oracle_mod):
    """All-pairs definition over alive agents; edge segments only between consecutive
    edge points of one polyline; lane polylines never collide."""
    agents = [(0, 0, 0, 4.5, 2), (3.0, 0.5, 0.3, 4.5, 2), (20, 0, 0, 4.5, 2), (40, 0, 0, 4.5, 2),
              (60, 0, 0, 4.5, 2)]
    edges = [[(20, 0.5), (20, 5)],            # pokes into agent 2 from above
             [(38, 5), (39, 5), (41, 5)],      # passes 4 m beside agent 3
             [(35, -5)], ]                     # single-point polyline: no segment
    lanes = [[(58, 0), (62, 0)]]               # lane through agent 4: not a collision
    sc = _tiny_world(agents, edges, lanes)
    sim = oracle_mod.OracleSim(sc)
    coll, band = sim.collide()
    assert list(coll) == [1, 1, 2, 0, 0]
    sim.flags[1] = oracle_mod.VISIBLE  # agent 1 no longer alive: nobody collides with it
    coll, _ = sim.collide()
    assert list(coll) == [0, 0, 2, 0, 0]


def test_polyline_boundary_is_not_a_segment(oracle_mod):
    """The last point of one edge polyline and the first of the next are not joined."""
    agents = [(0, 0, 0, 4.5, 2)]
    edges = [[(-10, -5), (-1, -5)], [(1, 5), (10, 5)]]  # a jump across the agent
    sc = _tiny_world(agents, edges)
    coll, _ = oracle_mod.OracleSim(sc).collide()
    assert coll[0] == 0
    sc = _tiny_world(agents, [[(-10, -5), (-1, -5), (1, 5), (10, 5)]])
    coll, _ = oracle_mod.OracleSim(sc).collide()
    assert coll[0] == 2


def test_near_touch_just_outside_the_band(oracle_mod):
    """Boxes 0.5 mm apart do not collide and boxes overlapping by 0.5 mm do (strict
    overlap, Sec. 3.2 "Termination"); both are outside the 1e-4 m band, so no band bit is
    set.  The same for a road edge 0.5 mm beside a box and one 0.5 mm inside it."""
    for gap, want in ((5e-4, 0), (-5e-4, 1)):
        sc = _tiny_world([(0, 0, 0, 4.5, 2), (4.5 + gap, 0, 0, 4.5, 2)], [])
        coll, band = oracle_mod.OracleSim(sc).collide()
        assert list(coll) == [want, want], gap
        assert not band.any(), gap
    for gap, want in ((5e-4, 0), (-5e-4, 2)):
        sc = _tiny_world([(0, 0, 0, 4.5, 2)], [[(-10, 1 + gap), (10, 1 + gap)]])
        coll, band = oracle_mod.OracleSim(sc).collide()
        assert coll[0] == want and not band.any(), gap
    # within the band the decision is marked
    sc = _tiny_world([(0, 0, 0, 4.5, 2), (4.5 + 5e-5, 0, 0, 4.5, 2)], [])
    _, band = oracle_mod.OracleSim(sc).collide()
    assert np.all(band & 1)
