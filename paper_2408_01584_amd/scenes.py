"""Seeded synthetic scenes and action sequences.

This module only *generates inputs*; it holds none of the simulator's
arithmetic (no dynamics, collision, observation or reward code).  Both the HIP
library and the CPU oracle consume the arrays it returns.

The paper evaluates on Waymo Open Motion Dataset scenes, which represent the
map as road polylines with a type (Sec. 3.2, "Dataset") and agents as boxes
with a goal point (Sec. 3.2, "Rewards").  That dataset is not available here,
so procedural scenes of the same structure stand in for it:

* road polylines of two types, ``LANE`` (centre lines, travel direction) and
  ``EDGE`` (road edges).  Edge polylines run with the drivable area on their
  left; block boundaries are closed loops, blocks cut by the map border are
  open polylines.
* agents are 4.5 x 2.0 m boxes placed on lane centre lines with the heading of
  the lane, speed U(0, 15) m/s and a goal U(30, 80) m straight ahead.
* actions are (acceleration U(-3, 2) m/s^2, steering U(-0.3, 0.3) rad).

Layout (structure of arrays, all worlds concatenated, CSR offsets):

* ``agent_off`` int32 [W+1], ``road_off`` int32 [W+1]
* agents, float32 [A]: ``x y yaw speed length width goal_x goal_y``
* road, [R]: ``road_x road_y road_dir`` float32 and ``road_meta`` int32 with
  bits 0..7 = type (0 lane, 1 edge) and bit 8 = last point of its polyline.
  ``road_dir`` is the angle of the vector to the next point of the polyline
  (the last point repeats its predecessor's angle).

Seeding: world ``w`` of configuration ``c`` draws from
``SeedSequence(1000 + c).spawn(W)[w]`` (so a world does not depend on how many
other worlds are generated) and the actions of configuration ``c`` from
``SeedSequence(2000 + c)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LANE = 0
EDGE = 1
META_LAST = 1 << 8

CAR_LENGTH = 4.5
CAR_WIDTH = 2.0
LANE_WIDTH = 3.5
HALF_ROAD = 2 * LANE_WIDTH  # two lanes per direction -> 14 m roads


@dataclass(frozen=True)
class SimParams:
    """Per-configuration simulator parameters (sizes and constants)."""

    top_k: int
    partners: int  # -1: ragged, A_w - 1 slots per agent
    episode_len: int = 91
    dt: float = 0.1
    obs_radius: float = 50.0
    goal_radius: float = 2.0
    v_max: float = 30.0
    lidar_rays: int = 0
    lidar_range: float = 50.0
    collision_penalty: float = 0.0
    auto_reset: bool = True
    terminate_on_collision: bool = False
    dynamics: int = 0  # 0: bicycle model (App. B); 1: simplified model (Sec. 3.2 "Agent dynamics")
    lidar_fov: float = 0.0  # 0: LIDAR rays around the full circle; > 0: view-cone width (rad)
    min_goal_dist: float = 0.0  # > 0: agents starting within it of their goal are parked


@dataclass(frozen=True)
class ConfigSpec:
    worlds: int
    agents: tuple  # (lo, hi) inclusive; lo == hi for fixed counts
    road: object  # int (fixed) or "lognormal"
    steps: int
    params: SimParams
    layout: str = "grid3x3"


CONFIGS = {
    # single 4-way intersection, 500 points at 1 m spacing
    0: ConfigSpec(1, (8, 8), 500, 91, SimParams(top_k=64, partners=7), layout="cross"),
    # fixed-size batch, 3x3 intersections on 100 m blocks
    1: ConfigSpec(256, (64, 64), 4000, 91, SimParams(top_k=200, partners=63)),
    # uneven batch: agents U{1..128}, road points lognormal(ln 3000, 0.6) in [500, 10000]
    2: ConfigSpec(1024, (1, 128), "lognormal", 91, SimParams(top_k=200, partners=-1)),
    # differentiable rollout
    3: ConfigSpec(512, (32, 32), 2000, 20, SimParams(top_k=64, partners=31)),
    # large mixed with 30-ray planar LIDAR
    4: ConfigSpec(4096, (64, 64), 6000, 91, SimParams(top_k=200, partners=63, lidar_rays=30)),
}


@dataclass
class Scene:
    cfg: int
    params: SimParams
    agent_off: np.ndarray
    road_off: np.ndarray
    x: np.ndarray
    y: np.ndarray
    yaw: np.ndarray
    speed: np.ndarray
    length: np.ndarray
    width: np.ndarray
    goal_x: np.ndarray
    goal_y: np.ndarray
    road_x: np.ndarray
    road_y: np.ndarray
    road_dir: np.ndarray
    road_meta: np.ndarray
    extra: dict = field(default_factory=dict)
    agent_class: np.ndarray | None = None  # uint8 [A]: 0 vehicle, 1 cyclist, 2 pedestrian

    @property
    def num_worlds(self) -> int:
        return len(self.agent_off) - 1

    @property
    def num_agents(self) -> int:
        return int(self.agent_off[-1])

    @property
    def num_road(self) -> int:
        return int(self.road_off[-1])

    def agent_arrays(self):
        return dict(x=self.x, y=self.y, yaw=self.yaw, speed=self.speed, length=self.length,
                    width=self.width, goal_x=self.goal_x, goal_y=self.goal_y)

    def road_arrays(self):
        return dict(road_x=self.road_x, road_y=self.road_y, road_dir=self.road_dir,
                    road_meta=self.road_meta)

    def copy(self) -> "Scene":
        kw = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in self.__dict__.items()}
        kw["extra"] = dict(self.extra)
        return Scene(**kw)


# --------------------------------------------------------------------------------------
# road geometry (exact corner points; resampled afterwards)
# --------------------------------------------------------------------------------------

def _lanes_for_road(axis: str, c: float, lo: float, hi: float):
    """Centre lines of one 4-lane road (right-hand traffic) as (type, corners)."""
    out = []
    for off in (0.5 * LANE_WIDTH, 1.5 * LANE_WIDTH):
        if axis == "v":  # road along y at x = c: northbound on the +x side
            out.append((LANE, [(c + off, lo), (c + off, hi)]))
            out.append((LANE, [(c - off, hi), (c - off, lo)]))
        else:  # road along x at y = c: eastbound on the -y side
            out.append((LANE, [(lo, c - off), (hi, c - off)]))
            out.append((LANE, [(hi, c + off), (lo, c + off)]))
    return out


def _block_edge(xa, xb, ya, yb, border):
    """Edge polyline of the block [xa,xb]x[ya,yb], clockwise (drivable area on the
    left).  ``border`` = (top, right, bottom, left) booleans, True where that side lies
    on the map border and therefore carries no edge."""
    corners = [(xa, yb), (xb, yb), (xb, ya), (xa, ya)]  # clockwise
    sides = [(corners[i], corners[(i + 1) % 4]) for i in range(4)]  # top, right, bottom, left
    if not any(border):
        return [corners[0], corners[1], corners[2], corners[3], corners[0]]
    # start right after a border side so that the road-facing sides are consecutive
    first = next(i for i in range(4) if border[i] and not border[(i + 1) % 4])
    pts = []
    for k in range(1, 4):
        i = (first + k) % 4
        if border[i]:
            break
        a, b = sides[i]
        if not pts:
            pts.append(a)
        pts.append(b)
    return pts


def _grid_geometry(rng: np.random.Generator, jitter: float = 8.0):
    """3x3 intersections on ~100 m blocks spanning +-150 m."""
    span = 150.0
    xs = np.array([-100.0, 0.0, 100.0]) + rng.uniform(-jitter, jitter, 3)
    ys = np.array([-100.0, 0.0, 100.0]) + rng.uniform(-jitter, jitter, 3)
    polys = []
    for c in xs:
        polys += _lanes_for_road("v", float(c), -span, span)
    for c in ys:
        polys += _lanes_for_road("h", float(c), -span, span)
    xcuts = [-span] + [v for c in xs for v in (c - HALF_ROAD, c + HALF_ROAD)] + [span]
    ycuts = [-span] + [v for c in ys for v in (c - HALF_ROAD, c + HALF_ROAD)] + [span]
    for i in range(4):
        xa, xb = float(xcuts[2 * i]), float(xcuts[2 * i + 1])
        for j in range(4):
            ya, yb = float(ycuts[2 * j]), float(ycuts[2 * j + 1])
            border = (j == 3, i == 3, j == 0, i == 0)
            polys.append((EDGE, _block_edge(xa, xb, ya, yb, border)))
    return polys


def _cross_geometry():
    """Single 4-way intersection: lanes to +-22.5 m (46 points each at 1 m), four
    L-shaped corner edges with 16 m legs (33 points each): 8*46 + 4*33 = 500."""
    polys = []
    polys += _lanes_for_road("v", 0.0, -22.5, 22.5)
    polys += _lanes_for_road("h", 0.0, -22.5, 22.5)
    e, f = HALF_ROAD, 23.0
    polys.append((EDGE, [(f, e), (e, e), (e, f)]))        # NE block
    polys.append((EDGE, [(e, -f), (e, -e), (f, -e)]))     # SE block
    polys.append((EDGE, [(-f, -e), (-e, -e), (-e, -f)]))  # SW block
    polys.append((EDGE, [(-e, f), (-e, e), (-f, e)]))     # NW block
    return polys


def _poly_len(pts):
    p = np.asarray(pts, dtype=np.float64)
    return float(np.sum(np.hypot(np.diff(p[:, 0]), np.diff(p[:, 1]))))


def _resample(pts, n):
    """n points uniformly spaced in arc length along the polyline (ends kept)."""
    p = np.asarray(pts, dtype=np.float64)
    seg = np.hypot(np.diff(p[:, 0]), np.diff(p[:, 1]))
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    s = np.linspace(0.0, cum[-1], n)
    return np.interp(s, cum, p[:, 0]), np.interp(s, cum, p[:, 1])


def _allocate_points(lengths, total):
    """Points per polyline (>= 2 each) proportional to length, summing to ``total``."""
    lengths = np.asarray(lengths, dtype=np.float64)
    npoly = len(lengths)
    if total < 2 * npoly:
        raise ValueError("too few road points for the polylines")
    spacing = lengths.sum() / max(total - npoly, 1)
    n = np.maximum(2, np.round(lengths / spacing).astype(np.int64) + 1)
    order = np.argsort(-lengths, kind="stable")
    k = 0
    while n.sum() != total:
        i = order[k % npoly]
        if n.sum() > total:
            if n[i] > 2:
                n[i] -= 1
        else:
            n[i] += 1
        k += 1
    return n


def _build_road(polys, total_points, exact_spacing=False):
    lengths = [_poly_len(p) for _, p in polys]
    if exact_spacing:
        counts = [int(round(L)) + 1 for L in lengths]
        if sum(counts) != total_points:
            raise ValueError("cross layout must give exactly %d points" % total_points)
    else:
        counts = _allocate_points(lengths, total_points)
    xs, ys, dirs, metas = [], [], [], []
    for (typ, pts), n in zip(polys, counts):
        px, py = _resample(pts, int(n))
        d = np.arctan2(np.diff(py), np.diff(px))
        d = np.concatenate([d, d[-1:]])
        m = np.full(len(px), typ, dtype=np.int32)
        m[-1] |= META_LAST
        xs.append(px); ys.append(py); dirs.append(d); metas.append(m)
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(dirs), np.concatenate(metas))


def _build_dense_road(polys, rng, spacing, wobble, wavelength, jitter):
    """Polylines sampled every ``spacing`` m (the paper's source maps are sampled at
    0.1 m, Sec. 3.1) with a smooth lateral wobble (amplitude ``wobble`` m, wavelength
    ``wavelength`` m, random phase per polyline, fading to zero at the ends) and a
    Gaussian jitter of ``jitter`` m, so that nothing is exactly straight."""
    xs, ys, dirs, metas = [], [], [], []
    for typ, pts in polys:
        L = _poly_len(pts)
        n = max(2, int(round(L / spacing)) + 1)
        px, py = _resample(pts, n)
        tx, ty = np.gradient(px), np.gradient(py)
        tn = np.maximum(np.hypot(tx, ty), 1e-12)
        nx, ny = -ty / tn, tx / tn
        sarc = np.linspace(0.0, L, n)
        fade = np.minimum(1.0, np.minimum(sarc, L - sarc) / 10.0)
        off = wobble * fade * np.sin(2 * np.pi * sarc / wavelength + rng.uniform(0, 2 * np.pi))
        px = px + off * nx + rng.normal(0.0, jitter, n)
        py = py + off * ny + rng.normal(0.0, jitter, n)
        d = np.arctan2(np.diff(py), np.diff(px))
        d = np.concatenate([d, d[-1:]])
        m = np.full(n, typ, dtype=np.int32)
        m[-1] |= META_LAST
        xs.append(px); ys.append(py); dirs.append(d); metas.append(m)
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(dirs), np.concatenate(metas))


# --------------------------------------------------------------------------------------
# agents
# --------------------------------------------------------------------------------------

def _place_agents(rng, lanes, n_agents, margin=0.5, max_tries=20000):
    """Agents on lane centre lines, heading along the lane.  A candidate is rejected
    when its centre is closer than (box diagonal + margin) to an earlier agent, which is
    sufficient for the boxes not to touch."""
    lens = np.array([_poly_len(p) for p in lanes])
    prob = lens / lens.sum()
    min_d = math.hypot(CAR_LENGTH, CAR_WIDTH) + margin
    px, py, ph = [], [], []
    tries = 0
    while len(px) < n_agents:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d agents" % n_agents)
        li = rng.choice(len(lanes), p=prob)
        (x0, y0), (x1, y1) = lanes[li][0], lanes[li][-1]
        s = rng.uniform(0.0, 1.0)
        cx, cy = x0 + s * (x1 - x0), y0 + s * (y1 - y0)
        if px:
            d = np.hypot(np.asarray(px) - cx, np.asarray(py) - cy)
            if np.any(d < min_d):
                continue
        px.append(cx); py.append(cy); ph.append(math.atan2(y1 - y0, x1 - x0))
    px, py, ph = np.array(px), np.array(py), np.array(ph)
    speed = rng.uniform(0.0, 15.0, n_agents)
    ahead = rng.uniform(30.0, 80.0, n_agents)
    gx = px + ahead * np.cos(ph)
    gy = py + ahead * np.sin(ph)
    return px, py, ph, speed, gx, gy


def _wrap(a):
    return (a + np.pi) % (2.0 * np.pi) - np.pi


def make_world(cfg: int, w: int, n_worlds: int | None = None, dense: dict | None = None):
    """Arrays of world ``w`` of configuration ``cfg`` (float64, before the float32 cast).
    ``dense`` (keys spacing, wobble, wavelength, jitter) replaces the fixed point count by
    polylines sampled densely as in the paper's source maps (``_build_dense_road``, drawn
    from SeedSequence(4000 + cfg)); agents and geometry are those of the plain world."""
    spec = CONFIGS[cfg]
    W = spec.worlds if n_worlds is None else n_worlds
    ss = np.random.SeedSequence(1000 + cfg).spawn(max(W, w + 1))[w]
    rng = np.random.Generator(np.random.PCG64(ss))
    lo, hi = spec.agents
    n_agents = int(rng.integers(lo, hi + 1)) if lo != hi else lo
    if spec.road == "lognormal":
        n_road = int(np.clip(round(math.exp(math.log(3000.0) + 0.6 * rng.standard_normal())),
                             500, 10000))
    else:
        n_road = int(spec.road)
    if spec.layout == "cross":
        polys = _cross_geometry()
        rx, ry, rd, rm = _build_road(polys, n_road, exact_spacing=True)
        lanes = [p for t, p in polys if t == LANE]
        ax, ay, ah, sp, gx, gy = _place_agents(rng, lanes, n_agents)
    else:
        polys = _grid_geometry(rng)
        if dense is not None:
            rng2 = np.random.Generator(np.random.PCG64(np.random.SeedSequence(4000 + cfg).spawn(max(W, w + 1))[w]))
            rx, ry, rd, rm = _build_dense_road(polys, rng2, **dense)
        else:
            rx, ry, rd, rm = _build_road(polys, n_road)
        lanes = [p for t, p in polys if t == LANE]
        ax, ay, ah, sp, gx, gy = _place_agents(rng, lanes, n_agents)
        # a seeded rigid motion per world so that no two worlds share coordinates
        th = rng.uniform(-math.pi, math.pi)
        tx, ty = rng.uniform(-50.0, 50.0, 2)
        c, s = math.cos(th), math.sin(th)

        def mv(x, y):
            return c * x - s * y + tx, s * x + c * y + ty

        rx, ry = mv(rx, ry)
        ax, ay = mv(ax, ay)
        gx, gy = mv(gx, gy)
        rd = _wrap(rd + th)
        ah = _wrap(ah + th)
    return dict(x=ax, y=ay, yaw=ah, speed=sp, length=np.full(n_agents, CAR_LENGTH),
                width=np.full(n_agents, CAR_WIDTH), goal_x=gx, goal_y=gy,
                road_x=rx, road_y=ry, road_dir=rd, road_meta=rm)


def make_scene(cfg: int, worlds=None, dense: dict | None = None) -> Scene:
    """Scene of configuration ``cfg``.  ``worlds`` (an iterable of world indices or
    an int n meaning range(n)) selects a subset; each world is identical to the same
    world in the full batch.  ``dense``: see ``make_world``."""
    spec = CONFIGS[cfg]
    if worlds is None:
        idx = list(range(spec.worlds))
    elif isinstance(worlds, (int, np.integer)):
        idx = list(range(int(worlds)))
    else:
        idx = [int(i) for i in worlds]
    parts = [make_world(cfg, w, spec.worlds, dense) for w in idx]
    return assemble(cfg, parts, spec.params, world_ids=idx)


def assemble(cfg, parts, params: SimParams, world_ids=None) -> Scene:
    """Concatenate per-world dicts into a CSR-batched float32 Scene."""
    a_counts = [len(p["x"]) for p in parts]
    r_counts = [len(p["road_x"]) for p in parts]
    agent_off = np.concatenate([[0], np.cumsum(a_counts)]).astype(np.int32)
    road_off = np.concatenate([[0], np.cumsum(r_counts)]).astype(np.int32)
    cat = lambda k, dt=np.float32: np.ascontiguousarray(
        np.concatenate([np.asarray(p[k]) for p in parts]).astype(dt))
    return Scene(cfg=cfg, params=params, agent_off=agent_off, road_off=road_off,
                 x=cat("x"), y=cat("y"), yaw=cat("yaw"), speed=cat("speed"),
                 length=cat("length"), width=cat("width"), goal_x=cat("goal_x"),
                 goal_y=cat("goal_y"), road_x=cat("road_x"), road_y=cat("road_y"),
                 road_dir=cat("road_dir"), road_meta=cat("road_meta", np.int32),
                 extra={"world_ids": list(world_ids) if world_ids is not None else None})


def make_delta_actions(cfg: int, steps: int, num_agents: int) -> np.ndarray:
    """float32 [steps, num_agents, 2] for the simplified model: (accel U(-3,2) m/s^2,
    curvature command U(-0.06,0.06) 1/m, i.e. turning radii of 17 m and more), drawn from
    SeedSequence(3000 + cfg)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(3000 + cfg)))
    acc = rng.uniform(-3.0, 2.0, size=(steps, num_agents))
    curv = rng.uniform(-0.06, 0.06, size=(steps, num_agents))
    return np.ascontiguousarray(np.stack([acc, curv], axis=-1).astype(np.float32))


def make_actions(cfg: int, steps: int, num_agents: int) -> np.ndarray:
    """float32 [steps, num_agents, 2]: (accel U(-3,2) m/s^2, steer U(-0.3,0.3) rad)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(2000 + cfg)))
    acc = rng.uniform(-3.0, 2.0, size=(steps, num_agents))
    steer = rng.uniform(-0.3, 0.3, size=(steps, num_agents))
    return np.ascontiguousarray(np.stack([acc, steer], axis=-1).astype(np.float32))
