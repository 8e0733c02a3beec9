"""ctypes front end of the FP64 CPU oracle (``gd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the CPU-baseline
leg of ``bench.py``; never by the product path.  It shares no code with the HIP library
and takes its inputs from scene objects produced by the seeded input generator (any
object with the Scene attributes works).

``build()`` compiles ``liboracle.so`` with gcc (``-O2 -fopenmp -ffp-contract=off``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gd_oracle.c")
# GD_ORACLE_LIB points the loader at another build of the same source (the mutation
# check of the oracle's pins builds planted-mistake copies there)
LIB = os.environ.get("GD_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))

COLL_AGENT, COLL_EDGE, GOAL, DONE, ALIVE, VISIBLE, STATIC = 1, 2, 4, 8, 16, 32, 64
VEHICLE, CYCLIST, PEDESTRIAN = 0, 1, 2
AUTO_RESET, TERM_ON_COLLISION = 1, 2
MODEL_BICYCLE, MODEL_DELTA = 0, 1
INV_MIN_DIST = 1e-3  # the inversion's distance threshold (m), as in gd_oracle.c


def build(force: bool = True) -> str:
    if "GD_ORACLE_LIB" in os.environ and os.path.exists(LIB):
        return LIB  # a prebuilt copy chosen by the caller
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


class Config(C.Structure):
    _fields_ = [("top_k", C.c_int32), ("partners", C.c_int32), ("episode_len", C.c_int32),
                ("lidar_rays", C.c_int32), ("flags", C.c_uint32), ("dt", C.c_double),
                ("obs_radius", C.c_double), ("goal_radius", C.c_double), ("v_max", C.c_double),
                ("lidar_range", C.c_double), ("collision_penalty", C.c_double),
                ("model", C.c_int32), ("lidar_fov", C.c_double), ("min_goal_dist", C.c_double),
                ("decide32", C.c_int32)]


class Batch(C.Structure):
    _fields_ = [("W", C.c_int32), ("agent_off", C.c_void_p), ("road_off", C.c_void_p)] + \
        [(n, C.c_void_p) for n in ("x", "y", "yaw", "v", "len", "wid", "gx", "gy", "snap_x",
                                   "snap_y", "snap_yaw", "snap_v", "rx", "ry", "rdir", "rmeta",
                                   "flags", "t", "head", "cls")]


class Outputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("ego", "partner", "pmask", "road", "road_idx", "lidar",
                                         "lidar_hit", "reward", "world_done", "band",
                                         "lidar_band")]


def _declare(L):
    vp, i32, d = C.c_void_p, C.c_int, C.c_double
    L.or_dynamics.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, d, d]
    L.or_delta.argtypes = [i32, vp, vp, vp, vp, vp, vp, d]
    L.or_delta_invert.argtypes = [i32, i32, vp, d, vp, vp]
    L.or_decimate.argtypes = [i32, vp, vp, vp, C.c_float, vp, vp]
    L.or_box_box_sep.argtypes = [vp, vp]
    L.or_box_box_sep.restype = d
    L.or_box_seg_sep.argtypes = [vp, d, d, d, d]
    L.or_box_seg_sep.restype = d
    L.or_ray_segment.argtypes = [d] * 9
    L.or_ray_segment.restype = d
    L.or_obs.argtypes = [vp, vp, vp]
    L.or_collide.argtypes = [vp, vp, vp]
    L.or_reset.argtypes = [vp, vp, vp, vp]
    L.or_step.argtypes = [vp, vp, vp, vp]
    L.or_rollout.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, d]
    L.or_rollout_vjp.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
    L.or_rollout_obs.argtypes = [vp, vp, i32, vp, vp, vp]


def _p(a):
    return None if a is None else a.ctypes.data


def config_from_params(p, decide32: bool = False) -> Config:
    """decide32: take the distance decisions (radius filters, goal and parking tests, road
    ranking key) in binary32 with the fixed operation order instead of FP64."""
    flags = (AUTO_RESET if p.auto_reset else 0) | (TERM_ON_COLLISION if p.terminate_on_collision else 0)
    return Config(p.top_k, p.partners, p.episode_len, p.lidar_rays, flags, p.dt, p.obs_radius,
                  p.goal_radius, p.v_max, p.lidar_range, p.collision_penalty,
                  getattr(p, "dynamics", MODEL_BICYCLE), getattr(p, "lidar_fov", 0.0),
                  getattr(p, "min_goal_dist", 0.0), 1 if decide32 else 0)


def partner_slots(agent_off: np.ndarray, partners: int) -> int:
    n = np.diff(agent_off.astype(np.int64))
    return int(n.sum() * partners) if partners >= 0 else int((n * (n - 1)).sum())


# --------------------------------------------------------------------------- primitives

def dynamics(x, y, yaw, v, length, actions, dt=0.1, v_max=30.0, alive=None):
    """One explicit-Euler bicycle step (App. B) in FP64; returns new arrays."""
    x, y, yaw, v = (np.array(a, dtype=np.float64, copy=True) for a in (x, y, yaw, v))
    length = np.ascontiguousarray(length, dtype=np.float64)
    act = np.ascontiguousarray(actions, dtype=np.float64).reshape(-1, 2)
    al = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    lib().or_dynamics(len(x), _p(x), _p(y), _p(yaw), _p(v), _p(length), _p(act), _p(al), dt, v_max)
    return x, y, yaw, v


def delta_dynamics(x, y, yaw, v, actions, dt=0.1, alive=None):
    """One step of the simplified bicycle model (Sec. 3.2 "Agent dynamics") in FP64: actions are
    (acceleration m/s^2, curvature command 1/m); returns new arrays."""
    x, y, yaw, v = (np.array(a, dtype=np.float64, copy=True) for a in (x, y, yaw, v))
    act = np.ascontiguousarray(actions, dtype=np.float64).reshape(-1, 2)
    al = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    lib().or_delta(len(x), _p(x), _p(y), _p(yaw), _p(v), _p(act), _p(al), dt)
    return x, y, yaw, v


def invert_actions(states, dt=0.1):
    """Actions [T, n, 2] of the simplified model that carry states[t] to states[t+1]
    (states [T+1, 4, n]: x, y, yaw, speed), and a band mask [T, n] of the steps whose
    command sits at a decision threshold (see ``or_delta_invert``)."""
    st = np.ascontiguousarray(states, dtype=np.float64)
    T, n = st.shape[0] - 1, st.shape[2]
    act = np.zeros((max(T, 0), n, 2))
    band = np.zeros((max(T, 0), n), np.uint8)
    lib().or_delta_invert(n, T, _p(st), dt, _p(act), _p(band))
    return act, band


def decimate(poly_off, x, y, min_area):
    """Visvalingam-Whyatt decimation (Sec. 3.1) of the polylines with CSR offsets
    poly_off over binary32 points x, y: (keep [n] uint8, dir [n] float64 for kept points)."""
    po = np.ascontiguousarray(poly_off, dtype=np.int32)
    xs = np.ascontiguousarray(x, dtype=np.float32)
    ys = np.ascontiguousarray(y, dtype=np.float32)
    keep = np.zeros(len(xs), np.uint8)
    dr = np.zeros(len(xs))
    lib().or_decimate(len(po) - 1, _p(po), _p(xs), _p(ys), float(min_area), _p(keep), _p(dr))
    return keep, dr


def box_box_sep(a, b) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return lib().or_box_box_sep(_p(a), _p(b))


def box_seg_sep(a, x0, y0, x1, y1) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return lib().or_box_seg_sep(_p(a), x0, y0, x1, y1)


def ray_segment(ox, oy, dx, dy, x0, y0, x1, y1, tmax) -> float:
    return lib().or_ray_segment(ox, oy, dx, dy, x0, y0, x1, y1, tmax)


# --------------------------------------------------------------------------- simulator

# band bits (per agent) of the oracle's outputs: a decision within 1e-4 m of its threshold
BAND_COLL, BAND_GOAL, BAND_PARTNER_R, BAND_KTH, BAND_LIDAR, BAND_ROAD_R = 1, 2, 4, 8, 16, 32


class OracleSim:
    """FP64 simulator over a CSR-batched scene.  State and outputs are numpy arrays.

    decide32=True switches the distance decisions to the binary32 emulation (secondary
    check); the default takes them in FP64, the plain definition."""

    def __init__(self, scene, params=None, decide32=False):
        self.params = params if params is not None else scene.params
        self.cfg = config_from_params(self.params, decide32)
        self.agent_off = np.ascontiguousarray(scene.agent_off, dtype=np.int32)
        self.road_off = np.ascontiguousarray(scene.road_off, dtype=np.int32)
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64).copy()
        self.x, self.y, self.yaw, self.v = f64(scene.x), f64(scene.y), f64(scene.yaw), f64(scene.speed)
        self.len, self.wid = f64(scene.length), f64(scene.width)
        self.gx, self.gy = f64(scene.goal_x), f64(scene.goal_y)
        self.snap = [self.x.copy(), self.y.copy(), self.yaw.copy(), self.v.copy()]
        self.rx, self.ry, self.rdir = f64(scene.road_x), f64(scene.road_y), f64(scene.road_dir)
        self.rmeta = np.ascontiguousarray(scene.road_meta, dtype=np.int32).copy()
        self.W = len(self.agent_off) - 1
        self.A = int(self.agent_off[-1])
        self.flags = np.full(self.A, ALIVE | VISIBLE, dtype=np.uint8)
        cls = getattr(scene, "agent_class", None)
        self.cls = None if cls is None else np.ascontiguousarray(cls, dtype=np.uint8).copy()
        self.head = np.zeros(self.A)  # view-cone head angles (rad, from the heading)
        self.t = np.zeros(self.W, dtype=np.int32)
        p = self.params
        self.K, self.N = p.top_k, p.lidar_rays
        self.S = partner_slots(self.agent_off, p.partners)
        self._alloc_outputs()
        if getattr(p, "min_goal_dist", 0.0) > 0.0:  # start flags of the first episode
            lib().or_reset(C.byref(self._batch()), C.byref(self.cfg), None, None)

    def _alloc_outputs(self):
        A, K, N, S = self.A, self.K, self.N, self.S
        self.out = dict(ego=np.zeros((A, 8)), partner=np.zeros((S, 6)),
                        pmask=np.zeros(S, np.uint8), road=np.zeros((A, K, 4)),
                        road_idx=np.zeros((A, K), np.int32), lidar=np.zeros((A, max(N, 1))),
                        lidar_hit=np.zeros((A, max(N, 1)), np.int32), reward=np.zeros(A),
                        world_done=np.zeros(self.W, np.uint8), band=np.zeros(A, np.uint8),
                        lidar_band=np.zeros((A, max(N, 1)), np.uint8))

    def _batch(self):
        b = Batch()
        b.W = self.W
        b.agent_off, b.road_off = _p(self.agent_off), _p(self.road_off)
        b.x, b.y, b.yaw, b.v = _p(self.x), _p(self.y), _p(self.yaw), _p(self.v)
        b.len, b.wid, b.gx, b.gy = _p(self.len), _p(self.wid), _p(self.gx), _p(self.gy)
        b.snap_x, b.snap_y, b.snap_yaw, b.snap_v = (_p(a) for a in self.snap)
        b.rx, b.ry, b.rdir, b.rmeta = _p(self.rx), _p(self.ry), _p(self.rdir), _p(self.rmeta)
        b.flags, b.t = _p(self.flags), _p(self.t)
        b.head = _p(self.head)
        b.cls = _p(self.cls)
        self._keep = b
        return b

    def _outputs(self):
        o = Outputs()
        for k in ("ego", "partner", "pmask", "road", "road_idx", "lidar", "lidar_hit", "reward",
                  "world_done", "band", "lidar_band"):
            setattr(o, k, _p(self.out[k]))
        self._keep_o = o
        return o

    def _result(self):
        r = {k: v.copy() for k, v in self.out.items()}
        if self.N == 0:
            r["lidar"] = r["lidar"][:, :0]
            r["lidar_hit"] = r["lidar_hit"][:, :0]
            r["lidar_band"] = r["lidar_band"][:, :0]
        r["flags"] = self.flags.copy()
        r["t"] = self.t.copy()
        r["state"] = np.stack([self.x, self.y, self.yaw, self.v]).copy()
        # the scene geometry (shared, not copied), for comparisons that need FP64
        # distances of points the oracle did not select
        r["geom"] = dict(agent_off=self.agent_off, road_off=self.road_off, road_x=self.rx,
                         road_y=self.ry, partners=self.params.partners)
        return r

    # -- state access (teacher forcing) --
    def set_state(self, x=None, y=None, yaw=None, v=None, flags=None, t=None, head=None):
        for name, val in (("x", x), ("y", y), ("yaw", yaw), ("v", v), ("head", head)):
            if val is not None:
                getattr(self, name)[:] = np.asarray(val, dtype=np.float64)
        if flags is not None:
            self.flags[:] = np.asarray(flags, dtype=np.uint8)
        if t is not None:
            self.t[:] = np.asarray(t, dtype=np.int32)

    def reset(self, mask=None):
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        self.out["band"][:] = 0
        lib().or_reset(C.byref(self._batch()), C.byref(self.cfg), _p(m), C.byref(self._outputs()))
        return self._result()

    def step(self, actions):
        act = np.ascontiguousarray(actions, dtype=np.float64).reshape(self.A, 2)
        self.out["band"][:] = 0
        lib().or_step(C.byref(self._batch()), C.byref(self.cfg), _p(act), C.byref(self._outputs()))
        return self._result()

    def obs(self):
        self.out["band"][:] = 0
        lib().or_obs(C.byref(self._batch()), C.byref(self.cfg), C.byref(self._outputs()))
        return self._result()

    def collide(self):
        coll = np.zeros(self.A, np.uint8)
        band = np.zeros(self.A, np.uint8)
        lib().or_collide(C.byref(self._batch()), _p(coll), _p(band))
        return coll, band

    # -- differentiable rollout --
    def rollout(self, actions, tol=1e-6, obs=False):
        T = actions.shape[0]
        act = np.ascontiguousarray(actions, dtype=np.float64)
        rew = np.zeros((T, self.A))
        states = np.zeros((T + 1, 4, self.A))
        seg = np.zeros((T, self.A), np.int32)
        un = np.zeros(self.A, np.uint8)
        lib().or_rollout(C.byref(self._batch()), C.byref(self.cfg), T, _p(act), _p(rew),
                         _p(states), _p(seg), _p(un), tol)
        out = dict(rewards=rew, states=states, seg=seg, unstable=un)
        if obs:
            out["obs"], out["obs_band"] = self.rollout_obs(states)
        return out

    def obs_features(self) -> int:
        """Features per agent-step of the rollout observation (speed, goal x', goal y',
        then x', y', heading difference, speed of each of the P partner slots)."""
        if self.params.partners < 0:
            raise ValueError("the rollout observation needs a fixed number of partner slots")
        return 3 + 4 * self.params.partners

    def rollout_obs(self, states):
        """Observation [T, A, F] of the states [T + 1, 4, A] after each step, and the band
        [T, A] of its mask and wrap decisions."""
        T = states.shape[0] - 1
        st = np.ascontiguousarray(states, dtype=np.float64)
        obs = np.zeros((T, self.A, self.obs_features()))
        band = np.zeros((T, self.A), np.uint8)
        lib().or_rollout_obs(C.byref(self._batch()), C.byref(self.cfg), T, _p(st), _p(obs), _p(band))
        return obs, band

    def rollout_vjp(self, actions, grad_rewards, grad_obs=None):
        T = actions.shape[0]
        act = np.ascontiguousarray(actions, dtype=np.float64)
        gr = np.ascontiguousarray(grad_rewards, dtype=np.float64)
        go = None
        if grad_obs is not None:
            go = np.ascontiguousarray(grad_obs, dtype=np.float64)
            assert go.shape == (T, self.A, self.obs_features())
        ga = np.zeros((T, self.A, 2))
        g0 = np.zeros((4, self.A))
        lib().or_rollout_vjp(C.byref(self._batch()), C.byref(self.cfg), T, _p(act), _p(gr),
                             _p(go), _p(ga), _p(g0))
        return ga, g0
