"""ctypes binding of libgd.so with the same entry-point names as include/gd.h.

Argument marshalling only: every step of the simulator runs in the HIP kernels of the
library.  Importing this module loads ``libgd.so`` from the package directory and fails
loudly when it is missing (build it with ``python -m paper_2408_01584_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgd.so")

GD_OK, GD_E_ARG, GD_E_SIZE, GD_E_HIP, GD_E_STATE, GD_E_NONFINITE, GD_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "GD_OK", -1: "GD_E_ARG", -2: "GD_E_SIZE", -3: "GD_E_HIP", -4: "GD_E_STATE",
                -5: "GD_E_NONFINITE", -6: "GD_E_UNSUPPORTED"}

GD_FLAG_COLL_AGENT, GD_FLAG_COLL_EDGE, GD_FLAG_GOAL, GD_FLAG_DONE, GD_FLAG_ALIVE, GD_FLAG_VISIBLE = 1, 2, 4, 8, 16, 32
GD_FLAG_STATIC = 64
GD_CLASS_VEHICLE, GD_CLASS_CYCLIST, GD_CLASS_PEDESTRIAN = 0, 1, 2
GD_AUTO_RESET, GD_TERMINATE_ON_COLLISION, GD_CHECK_FINITE, GD_USE_GRAPH = 1, 2, 4, 8

ENTRY_POINTS = ("gd_partner_slots", "gd_workspace_size", "gd_create", "gd_reset", "gd_step",
                "gd_obs", "gd_rollout_fwd", "gd_rollout_obs_features", "gd_rollout_bwd",
                "gd_invert_actions",
                "gd_decimate_workspace_size", "gd_decimate", "gd_decimate_noalloc",
                "gd_set_obs_buffers", "gd_set_timing",
                "gd_get_timing", "gd_check", "gd_destroy", "gd_last_error")
GD_ROAD_AUTO, GD_ROAD_LDS, GD_ROAD_GLOBAL = 0, 1, 2
GD_ROAD_LANE, GD_ROAD_EDGE, GD_META_LAST = 0, 1, 1 << 8
GD_DYN_BICYCLE, GD_DYN_DELTA = 0, 1
GD_PHASE_STEP, GD_PHASE_LIDAR, GD_PHASE_ROLLOUT_FWD, GD_PHASE_ROLLOUT_BWD, GD_PHASE_INVERT = range(5)
GD_NUM_PHASES = 5
GD_DECIMATE_NOALLOC_MAX_POINTS = 1 << 22


class GDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class gd_config(C.Structure):
    _fields_ = [("num_worlds", C.c_int32), ("top_k", C.c_int32), ("partners", C.c_int32),
                ("episode_len", C.c_int32), ("lidar_rays", C.c_int32), ("flags", C.c_uint32),
                ("dt", C.c_float), ("obs_radius", C.c_float), ("goal_radius", C.c_float),
                ("v_max", C.c_float), ("lidar_range", C.c_float), ("collision_penalty", C.c_float),
                ("cell_size", C.c_float), ("obs_waves", C.c_int32), ("obs_bins", C.c_int32),
                ("obs_cands", C.c_int32), ("obs_road", C.c_int32), ("dynamics", C.c_int32),
                ("lidar_fov", C.c_float), ("min_goal_dist", C.c_float)]


_BUF_FIELDS = ("agent_off", "road_off", "x", "y", "yaw", "speed", "length", "width", "goal_x",
               "goal_y", "road_x", "road_y", "road_dir", "road_meta", "obs_ego", "obs_partner",
               "partner_mask", "obs_road", "road_idx", "lidar", "lidar_hit", "reward", "flags",
               "world_done", "t", "lidar_head", "agent_class", "workspace")


class gd_buffers(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in _BUF_FIELDS] + [("workspace_bytes", C.c_size_t)]


_lib = None


def lib():
    """The loaded libgd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgd.so not found at %s: build it with "
                               "`python -m paper_2408_01584_amd.build`" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, i32, i64p, szp = C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)
        cfgp = C.POINTER(gd_config)
        sig = {
            "gd_partner_slots": [cfgp, vp, i64p],
            "gd_workspace_size": [cfgp, vp, vp, szp],
            "gd_create": [cfgp, vp, vp, C.POINTER(gd_buffers), vp, C.POINTER(vp)],
            "gd_reset": [vp, vp, vp],
            "gd_step": [vp, vp, vp],
            "gd_obs": [vp, vp],
            "gd_rollout_fwd": [vp, vp, i32, i32, vp, vp, vp, vp, vp],
            "gd_rollout_obs_features": [vp, C.POINTER(C.c_int32)],
            "gd_rollout_bwd": [vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp],
            "gd_invert_actions": [vp, vp, i32, vp, vp],
            "gd_decimate_workspace_size": [i32, szp],
            "gd_decimate": [vp, i32, i32, vp, vp, C.c_float, vp, vp, vp, C.c_size_t, vp],
            "gd_decimate_noalloc": [vp, i32, i32, vp, vp, C.c_float, vp, vp, vp],
            "gd_set_obs_buffers": [vp, C.POINTER(gd_buffers)],
            "gd_set_timing": [vp, i32],
            "gd_get_timing": [vp, vp, vp],
            "gd_check": [vp, vp],
            "gd_destroy": [vp],
            "gd_last_error": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.gd_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def gd_last_error() -> str:
    return lib().gd_last_error().decode()


def _check(status: int) -> int:
    if status != GD_OK:
        raise GDError(status, gd_last_error())
    return status


def gd_partner_slots(cfg: gd_config, h_agent_off) -> int:
    out = C.c_int64(0)
    _check(lib().gd_partner_slots(C.byref(cfg), h_agent_off.ctypes.data, C.byref(out)))
    return out.value


def gd_workspace_size(cfg: gd_config, h_agent_off, h_road_off) -> int:
    out = C.c_size_t(0)
    _check(lib().gd_workspace_size(C.byref(cfg), h_agent_off.ctypes.data, h_road_off.ctypes.data,
                                   C.byref(out)))
    return out.value


def gd_create(cfg: gd_config, h_agent_off, h_road_off, bufs: gd_buffers, stream: int):
    h = C.c_void_p(0)
    _check(lib().gd_create(C.byref(cfg), h_agent_off.ctypes.data, h_road_off.ctypes.data,
                           C.byref(bufs), C.c_void_p(stream), C.byref(h)))
    return h


def gd_reset(sim, world_mask_ptr: int | None, stream: int):
    _check(lib().gd_reset(sim, C.c_void_p(world_mask_ptr or 0), C.c_void_p(stream)))


def gd_step(sim, actions_ptr: int, stream: int):
    _check(lib().gd_step(sim, C.c_void_p(actions_ptr), C.c_void_p(stream)))


def gd_obs(sim, stream: int):
    _check(lib().gd_obs(sim, C.c_void_p(stream)))


def gd_rollout_fwd(sim, actions_ptr: int, T: int, ckpt_every: int, rewards_ptr: int,
                   ckpt_ptr: int, states_ptr: int | None, obs_ptr: int | None, stream: int):
    _check(lib().gd_rollout_fwd(sim, C.c_void_p(actions_ptr), T, ckpt_every,
                                C.c_void_p(rewards_ptr), C.c_void_p(ckpt_ptr),
                                C.c_void_p(states_ptr or 0), C.c_void_p(obs_ptr or 0),
                                C.c_void_p(stream)))


def gd_rollout_obs_features(sim) -> int:
    out = C.c_int32(0)
    _check(lib().gd_rollout_obs_features(sim, C.byref(out)))
    return out.value


def gd_rollout_bwd(sim, actions_ptr: int, ckpt_ptr: int, T: int, ckpt_every: int,
                   grad_rewards_ptr: int, grad_obs_ptr: int | None, states_ptr: int | None,
                   grad_actions_ptr: int, grad_state0_ptr: int | None, stream: int):
    _check(lib().gd_rollout_bwd(sim, C.c_void_p(actions_ptr), C.c_void_p(ckpt_ptr), T, ckpt_every,
                                C.c_void_p(grad_rewards_ptr), C.c_void_p(grad_obs_ptr or 0),
                                C.c_void_p(states_ptr or 0), C.c_void_p(grad_actions_ptr),
                                C.c_void_p(grad_state0_ptr or 0), C.c_void_p(stream)))


def gd_invert_actions(sim, states_ptr: int, T: int, actions_ptr: int, stream: int):
    _check(lib().gd_invert_actions(sim, C.c_void_p(states_ptr), T, C.c_void_p(actions_ptr),
                                   C.c_void_p(stream)))


def gd_decimate_workspace_size(n_points: int) -> int:
    out = C.c_size_t(0)
    _check(lib().gd_decimate_workspace_size(n_points, C.byref(out)))
    return out.value


def gd_decimate(poly_off_ptr: int, n_poly: int, n_points: int, x_ptr: int, y_ptr: int,
                min_area: float, keep_ptr: int, dir_ptr: int, ws_ptr: int, ws_bytes: int, stream: int):
    _check(lib().gd_decimate(C.c_void_p(poly_off_ptr), n_poly, n_points, C.c_void_p(x_ptr),
                             C.c_void_p(y_ptr), min_area, C.c_void_p(keep_ptr), C.c_void_p(dir_ptr),
                             C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream)))


def gd_decimate_noalloc(poly_off_ptr: int, n_poly: int, n_points: int, x_ptr: int, y_ptr: int,
                        min_area: float, keep_ptr: int, dir_ptr: int, stream: int):
    _check(lib().gd_decimate_noalloc(C.c_void_p(poly_off_ptr), n_poly, n_points, C.c_void_p(x_ptr),
                                     C.c_void_p(y_ptr), min_area, C.c_void_p(keep_ptr),
                                     C.c_void_p(dir_ptr), C.c_void_p(stream)))


def gd_set_obs_buffers(sim, bufs: gd_buffers):
    _check(lib().gd_set_obs_buffers(sim, C.byref(bufs)))


def gd_set_timing(sim, enable: bool):
    _check(lib().gd_set_timing(sim, 1 if enable else 0))


def gd_get_timing(sim):
    """(ms[GD_NUM_PHASES], count[GD_NUM_PHASES]) accumulated since the last call."""
    ms = (C.c_double * GD_NUM_PHASES)()
    cnt = (C.c_int64 * GD_NUM_PHASES)()
    _check(lib().gd_get_timing(sim, C.cast(ms, C.c_void_p), C.cast(cnt, C.c_void_p)))
    return list(ms), list(cnt)


def gd_check(sim, stream: int):
    _check(lib().gd_check(sim, C.c_void_p(stream)))


def gd_destroy(sim):
    _check(lib().gd_destroy(sim))
