"""Pins of the oracle's bicycle model (App. B) against closed forms.

None of these re-types the update rule: each compares the oracle with a property the
equations imply (constant-acceleration kinematics, the discrete circle traced under a
constant steer, the continuous turning radii, saturation of the speed clip).
"""
import math

import numpy as np
import pytest

DT = 0.1
L = 4.5


def run(O, x, y, yaw, v, acts, steps, vmax=30.0, dt=DT, length=L):
    n = len(x)
    traj = [np.stack([x, y, yaw, v])]
    for k in range(steps):
        a = acts[k] if acts.ndim == 3 else acts
        x, y, yaw, v = O.dynamics(x, y, yaw, v, np.full(n, length), a, dt=dt, v_max=vmax)
        traj.append(np.stack([x, y, yaw, v]))
    return np.array(traj)  # [steps+1, 4, n]


def test_straight_line_constant_acceleration(oracle_mod):
    """delta = 0: the midpoint-speed rule integrates constant acceleration exactly:
    s(n) = v0 n dt + a (n dt)^2 / 2 along the heading, v(n) = v0 + a n dt."""
    rng = np.random.default_rng(0)
    n = 16
    x0, y0 = rng.uniform(-50, 50, n), rng.uniform(-50, 50, n)
    yaw0 = rng.uniform(-math.pi, math.pi, n)
    v0 = rng.uniform(-5, 5, n)
    a = rng.uniform(-0.2, 0.2, n)  # |v| stays well below v_max over 91 steps
    acts = np.stack([a, np.zeros(n)], -1)
    tr = run(oracle_mod, x0, y0, yaw0, v0, acts, 91)
    for k in range(92):
        tk = k * DT
        s = v0 * tk + 0.5 * a * tk * tk
        np.testing.assert_allclose(tr[k, 0], x0 + s * np.cos(yaw0), rtol=0, atol=1e-9)
        np.testing.assert_allclose(tr[k, 1], y0 + s * np.sin(yaw0), rtol=0, atol=1e-9)
        np.testing.assert_allclose(tr[k, 2], yaw0, rtol=0, atol=0)
        np.testing.assert_allclose(tr[k, 3], v0 + a * tk, rtol=0, atol=1e-11)


def _circle_center(p):
    """Circumcentre of the first three points (x, y arrays)."""
    (ax, bx, cx), (ay, by, cy) = p[0][:3], p[1][:3]
    d = 2 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = ((ax**2 + ay**2) * (by - cy) + (bx**2 + by**2) * (cy - ay) + (cx**2 + cy**2) * (ay - by)) / d
    uy = ((ax**2 + ay**2) * (cx - bx) + (bx**2 + by**2) * (ax - cx) + (cx**2 + cy**2) * (bx - ax)) / d
    return ux, uy


@pytest.mark.parametrize("v,delta", [(10.0, 0.3), (5.0, -0.2), (12.0, 0.05), (-4.0, 0.25)])
def test_constant_steer_discrete_circle(oracle_mod, v, delta):
    """a = 0, constant delta: every step is the same rigid rotation, so the centre of
    gravity lies exactly on a circle of radius |v| dt / (2 sin(phi/2)), the yaw advances by
    phi = v cos(beta) tan(delta) dt / L with beta = atan(tan(delta)/2) (l_r = L/2), and the
    chord of each step points along yaw + beta."""
    tr = run(oracle_mod, np.array([1.0]), np.array([-2.0]), np.array([0.7]), np.array([v]),
             np.array([[0.0, delta]]), 91)
    beta = math.atan(0.5 * math.tan(delta))
    phi = v * math.cos(beta) * math.tan(delta) / L * DT
    np.testing.assert_allclose(np.diff(tr[:, 2, 0]), phi, rtol=0, atol=1e-13)
    xs, ys = tr[:, 0, 0], tr[:, 1, 0]
    cx, cy = _circle_center((xs, ys))
    rad = np.hypot(xs - cx, ys - cy)
    rho = abs(v) * DT / (2 * abs(math.sin(phi / 2)))
    np.testing.assert_allclose(rad, rho, rtol=1e-9)
    chord = np.arctan2(np.diff(ys), np.diff(xs))
    want = tr[:-1, 2, 0] + beta + (math.pi if v < 0 else 0.0)
    err = (chord - want + math.pi) % (2 * math.pi) - math.pi
    np.testing.assert_allclose(err, 0.0, atol=1e-11)


def test_turning_radius_continuous_limit(oracle_mod):
    """As dt -> 0 the centre of gravity turns on L / (cos(beta) tan(delta)) with error
    O(dt^2), and the rear axle (l_r = L/2 behind the CG) on L / tan(delta) with error
    O(dt): halving dt quarters, resp. halves, the error."""
    v, delta = 10.0, 0.3
    beta = math.atan(0.5 * math.tan(delta))
    r_cg = L / (math.cos(beta) * math.tan(delta))
    r_rear = L / math.tan(delta)
    errs_cg, errs_rear = [], []
    for dt in (0.1, 0.05, 0.025, 0.0125):
        steps = int(round(3.0 / dt))
        tr = run(oracle_mod, np.array([0.0]), np.array([0.0]), np.array([0.0]), np.array([v]),
                 np.array([[0.0, delta]]), steps, dt=dt)
        xs, ys, th = tr[:, 0, 0], tr[:, 1, 0], tr[:, 2, 0]
        cx, cy = _circle_center((xs, ys))
        errs_cg.append(abs(np.mean(np.hypot(xs - cx, ys - cy)) - r_cg))
        rx, ry = xs - 0.5 * L * np.cos(th), ys - 0.5 * L * np.sin(th)
        ccx, ccy = _circle_center((rx, ry))
        errs_rear.append(abs(np.mean(np.hypot(rx - ccx, ry - ccy)) - r_rear))
    ratios_cg = np.array(errs_cg[:-1]) / np.array(errs_cg[1:])
    ratios_rear = np.array(errs_rear[:-1]) / np.array(errs_rear[1:])
    assert np.all(np.abs(ratios_cg - 4.0) < 0.2), ratios_cg
    assert np.all(np.abs(ratios_rear - 2.0) < 0.1), ratios_rear
    assert errs_rear[0] / r_rear < 0.01  # ~0.5 % at dt = 0.1


def test_speed_clip_saturation(oracle_mod):
    """|v| is clipped to v_max both in the midpoint speed and in the new speed; once
    saturated the agent advances exactly v_max dt per step (reverse motion allowed)."""
    vmax = 5.0
    v0 = np.array([3.0, -3.0])
    a = np.array([2.0, -2.0])
    acts = np.stack([a, np.zeros(2)], -1)
    tr = run(oracle_mod, np.zeros(2), np.zeros(2), np.zeros(2), v0, acts, 30, vmax=vmax)
    # unclipped: v0 + a t reaches +-5 at t = 1.0 s (step 10); afterwards constant
    t_sat = 1.0
    for k in range(31):
        tk = k * DT
        if tk <= t_sat + 1e-12:
            s = v0 * tk + 0.5 * a * tk * tk
        else:
            s = v0 * t_sat + 0.5 * a * t_sat**2 + np.sign(a) * vmax * (tk - t_sat)
        np.testing.assert_allclose(tr[k, 0], s, atol=1e-12)
        np.testing.assert_allclose(tr[k, 3], np.clip(v0 + a * tk, -vmax, vmax), atol=1e-12)
    # the midpoint speed saturates half a step before the speed itself
    tr2 = run(oracle_mod, np.zeros(1), np.zeros(1), np.zeros(1), np.array([4.95]),
              np.array([[1.0, 0.0]]), 1, vmax=vmax)
    np.testing.assert_allclose(tr2[1, 0, 0], 5.0 * DT, atol=1e-15)   # vbar = min(5.0, 5)
    np.testing.assert_allclose(tr2[1, 3, 0], 5.0, atol=1e-15)        # min(5.05, 5)


def test_inactive_agents_frozen(oracle_mod):
    x, y, yaw, v = (np.array([1.0, 2.0]), np.array([3.0, 4.0]), np.array([0.1, 0.2]),
                    np.array([5.0, 6.0]))
    out = oracle_mod.dynamics(x, y, yaw, v, np.full(2, L), np.array([[1.0, 0.1], [1.0, 0.1]]),
                              alive=np.array([0, 1], np.uint8))
    assert out[0][0] == 1.0 and out[1][0] == 3.0 and out[2][0] == 0.1 and out[3][0] == 5.0
    assert out[0][1] != 2.0


def test_length_dependence(oracle_mod):
    """The yaw rate scales as 1/L (longer vehicles turn slower, Sec. 3.2 "Agent
    dynamics"); positions over one step do not depend on L."""
    outs = [oracle_mod.dynamics([0.0], [0.0], [0.0], [10.0], [Lk], [[0.0, 0.2]]) for Lk in (3.0, 6.0)]
    assert abs(outs[0][2][0] / outs[1][2][0] - 2.0) < 1e-12
    assert outs[0][0][0] == outs[1][0][0] and outs[0][1][0] == outs[1][1][0]
