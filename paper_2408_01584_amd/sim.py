"""torch convenience layer over the C-ABI: device buffers, the ``Sim`` handle and the
``DiffRollout`` autograd function.

torch is used for device memory and streams only; every step of the simulator runs in
the HIP kernels of libgd.so, called through ``paper_2408_01584_amd.gd``.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gd as G


def config_from_params(p, num_worlds: int, graph: bool = False, check_finite: bool = False,
                       cell_size: float = 0.0, obs_waves: int = 0, obs_bins: int = 0,
                       obs_cands: int = 0, obs_road: int = 0) -> G.gd_config:
    flags = (G.GD_AUTO_RESET if p.auto_reset else 0) | \
        (G.GD_TERMINATE_ON_COLLISION if p.terminate_on_collision else 0) | \
        (G.GD_CHECK_FINITE if check_finite else 0) | (G.GD_USE_GRAPH if graph else 0)
    c = G.gd_config()
    c.num_worlds = num_worlds
    c.top_k = p.top_k
    c.partners = p.partners
    c.episode_len = p.episode_len
    c.lidar_rays = p.lidar_rays
    c.flags = flags
    c.dt = p.dt
    c.obs_radius = p.obs_radius
    c.goal_radius = p.goal_radius
    c.v_max = p.v_max
    c.lidar_range = p.lidar_range
    c.collision_penalty = p.collision_penalty
    c.cell_size = cell_size
    c.obs_waves = obs_waves
    c.obs_bins = obs_bins
    c.obs_cands = obs_cands
    c.obs_road = obs_road
    c.dynamics = getattr(p, "dynamics", G.GD_DYN_BICYCLE)
    c.lidar_fov = getattr(p, "lidar_fov", 0.0)
    c.min_goal_dist = getattr(p, "min_goal_dist", 0.0)
    return c


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Sim:
    """A batch of worlds on one GPU.  ``scene`` is a CSR-batched Scene (see
    ``paper_2408_01584_amd.scenes``); its arrays are copied to the device once.

    Buffers are exposed as torch tensors in ``self.buf``; ``gd_step`` and friends update
    them in place on the current stream."""

    def __init__(self, scene, params=None, device="cuda", tuned=True, emit_road_idx=True, **launch):
        """``launch``: explicit launch-shape fields (cell_size, obs_waves, obs_bins,
        obs_cands, obs_road) and graph; without shape fields and with ``tuned``, the shape
        the autotuner cached for this workload on this device is used when there is one
        (every shape gives the same results).  ``emit_road_idx=False`` leaves the road
        point indices unwritten (no ``road_idx`` buffer)."""
        self.params = params if params is not None else scene.params
        shape_keys = ("cell_size", "obs_waves", "obs_bins", "obs_cands", "obs_road")
        if tuned and not any(k in launch for k in shape_keys):
            from .tune import cached_shape
            cs = cached_shape(scene, self.params, bool(launch.get("graph", False)))
            if cs:
                launch = {**launch, **cs}
        self.launch = {k: v for k, v in launch.items() if k in shape_keys}
        self.device = torch.device(device)
        self.h_agent_off = np.ascontiguousarray(scene.agent_off, dtype=np.int32)
        self.h_road_off = np.ascontiguousarray(scene.road_off, dtype=np.int32)
        self.W = len(self.h_agent_off) - 1
        self.A = int(self.h_agent_off[-1])
        self.R = int(self.h_road_off[-1])
        self.cfg = config_from_params(self.params, self.W, **launch)
        self.S = G.gd_partner_slots(self.cfg, self.h_agent_off)
        ws = G.gd_workspace_size(self.cfg, self.h_agent_off, self.h_road_off)
        dev = self.device
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev).contiguous()
        K, N = self.params.top_k, self.params.lidar_rays
        b = {}
        b["agent_off"] = torch.as_tensor(self.h_agent_off, device=dev)
        b["road_off"] = torch.as_tensor(self.h_road_off, device=dev)
        for k, src in (("x", scene.x), ("y", scene.y), ("yaw", scene.yaw), ("speed", scene.speed),
                       ("length", scene.length), ("width", scene.width), ("goal_x", scene.goal_x),
                       ("goal_y", scene.goal_y), ("road_x", scene.road_x), ("road_y", scene.road_y),
                       ("road_dir", scene.road_dir)):
            b[k] = f32(src)
        b["road_meta"] = torch.as_tensor(np.ascontiguousarray(scene.road_meta, dtype=np.int32), device=dev)
        A, W, S = self.A, self.W, self.S
        b["obs_ego"] = torch.zeros((A, 8), dtype=torch.float32, device=dev)
        b["obs_partner"] = torch.zeros((max(S, 1), 6), dtype=torch.float32, device=dev)
        b["partner_mask"] = torch.zeros(max(S, 1), dtype=torch.uint8, device=dev)
        b["obs_road"] = torch.zeros((A, max(K, 1), 4), dtype=torch.float32, device=dev)
        b["road_idx"] = torch.zeros((A, max(K, 1)), dtype=torch.int32, device=dev) if emit_road_idx else None
        b["lidar"] = torch.zeros((A, max(N, 1)), dtype=torch.float32, device=dev)
        b["lidar_hit"] = torch.zeros((A, max(N, 1)), dtype=torch.int32, device=dev)
        b["reward"] = torch.zeros(A, dtype=torch.float32, device=dev)
        b["flags"] = torch.zeros(A, dtype=torch.uint8, device=dev)
        b["world_done"] = torch.zeros(W, dtype=torch.uint8, device=dev)
        b["t"] = torch.zeros(W, dtype=torch.int32, device=dev)
        b["lidar_head"] = torch.zeros(max(A, 1), dtype=torch.float32, device=dev)  # head angles
        cls = getattr(scene, "agent_class", None)
        b["agent_class"] = None if cls is None else \
            torch.as_tensor(np.ascontiguousarray(cls, dtype=np.uint8), device=dev)
        b["workspace"] = torch.empty(ws + 256, dtype=torch.uint8, device=dev)
        self.buf = b
        bufs = G.gd_buffers()
        for name in G._BUF_FIELDS:
            if name == "workspace":
                continue
            t = b[name]
            setattr(bufs, name, None if t is None else t.data_ptr())
        if N == 0:
            bufs.lidar = None
            bufs.lidar_hit = None
        wptr = b["workspace"].data_ptr()
        pad = (-wptr) % 256
        bufs.workspace = wptr + pad
        bufs.workspace_bytes = ws
        self._bufs = bufs
        self.workspace_bytes = ws
        self.handle = G.gd_create(self.cfg, self.h_agent_off, self.h_road_off, bufs, _stream())

    # ---- stepping
    def step(self, actions: torch.Tensor):
        assert actions.dtype == torch.float32 and actions.is_contiguous() and actions.numel() == 2 * self.A
        G.gd_step(self.handle, actions.data_ptr(), _stream())

    def reset(self, mask: torch.Tensor | None = None):
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.numel() == self.W and mask.is_contiguous()
        G.gd_reset(self.handle, None if mask is None else mask.data_ptr(), _stream())

    def obs(self):
        G.gd_obs(self.handle, _stream())

    def set_obs_buffers(self, ego, partner, pmask, road, road_idx, lidar=None, lidar_hit=None):
        """Write the next observations into these tensors (e.g. a slot of a rollout ring)."""
        b = G.gd_buffers()
        b.obs_ego, b.obs_partner, b.partner_mask = ego.data_ptr(), partner.data_ptr(), pmask.data_ptr()
        b.obs_road, b.road_idx = road.data_ptr(), None if road_idx is None else road_idx.data_ptr()
        if lidar is not None:
            b.lidar, b.lidar_hit = lidar.data_ptr(), lidar_hit.data_ptr()
        G.gd_set_obs_buffers(self.handle, b)

    def set_timing(self, enable: bool):
        G.gd_set_timing(self.handle, enable)

    def get_timing(self):
        return G.gd_get_timing(self.handle)

    def check(self):
        G.gd_check(self.handle, _stream())

    def close(self):
        if getattr(self, "handle", None) is not None:
            G.gd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- views
    def state(self) -> torch.Tensor:
        b = self.buf
        return torch.stack([b["x"], b["y"], b["yaw"], b["speed"]])

    def outputs(self) -> dict:
        b = self.buf
        K, N, S = self.params.top_k, self.params.lidar_rays, self.S
        return dict(ego=b["obs_ego"], partner=b["obs_partner"][:S], pmask=b["partner_mask"][:S],
                    road=b["obs_road"][:, :K],
                    road_idx=None if b["road_idx"] is None else b["road_idx"][:, :K],
                    lidar=b["lidar"][:, :N], lidar_hit=b["lidar_hit"][:, :N], reward=b["reward"],
                    flags=b["flags"], world_done=b["world_done"], t=b["t"])

    def host_outputs(self) -> dict:
        torch.cuda.current_stream().synchronize()
        out = {k: v.cpu().numpy() for k, v in self.outputs().items() if v is not None}
        out["state"] = self.state().cpu().numpy()
        return out

    # ---- differentiable rollout
    def rollout_fwd(self, actions: torch.Tensor, ckpt_every: int = 10, obs: bool = False):
        """rewards [T, A] and checkpoints; with obs=True also the state log [T, 4, A] and
        the observation [T, A, 3 + 4P] (returned as a third and fourth value)."""
        T = actions.shape[0]
        rewards = torch.empty((T, self.A), dtype=torch.float32, device=self.device)
        nck = max(1, math.ceil(T / ckpt_every))
        ckpt = torch.empty((nck, 4, self.A), dtype=torch.float32, device=self.device)
        states = o = None
        if obs:
            F = G.gd_rollout_obs_features(self.handle)
            states = torch.empty((T, 4, self.A), dtype=torch.float32, device=self.device)
            o = torch.empty((T, self.A, F), dtype=torch.float32, device=self.device)
        G.gd_rollout_fwd(self.handle, actions.data_ptr(), T, ckpt_every, rewards.data_ptr(),
                         ckpt.data_ptr(), None if states is None else states.data_ptr(),
                         None if o is None else o.data_ptr(), _stream())
        if obs:
            return rewards, ckpt, states, o
        return rewards, ckpt

    def rollout_bwd(self, actions, ckpt, grad_rewards, ckpt_every: int = 10, want_state0=False,
                    grad_obs=None, states=None):
        T = actions.shape[0]
        ga = torch.empty((T, self.A, 2), dtype=torch.float32, device=self.device)
        g0 = torch.empty((4, self.A), dtype=torch.float32, device=self.device) if want_state0 else None
        if grad_obs is not None:
            assert states is not None and states.shape == (T, 4, self.A)
            grad_obs = grad_obs.contiguous()
        G.gd_rollout_bwd(self.handle, actions.data_ptr(), ckpt.data_ptr(), T, ckpt_every,
                         grad_rewards.contiguous().data_ptr(),
                         None if grad_obs is None else grad_obs.data_ptr(),
                         None if grad_obs is None else states.data_ptr(), ga.data_ptr(),
                         None if g0 is None else g0.data_ptr(), _stream())
        return ga, g0


    # ---- expert-action inversion (simplified model)
    def invert_actions(self, states: torch.Tensor) -> torch.Tensor:
        """states [T+1, 4, A] (x, y, yaw, speed) -> actions [T, A, 2] that replay them."""
        assert states.dtype == torch.float32 and states.is_contiguous()
        assert states.dim() == 3 and states.shape[1] == 4 and states.shape[2] == self.A
        T = states.shape[0] - 1
        actions = torch.empty((max(T, 0), self.A, 2), dtype=torch.float32, device=self.device)
        G.gd_invert_actions(self.handle, states.data_ptr(), T, actions.data_ptr(), _stream())
        return actions


class DiffRollout(torch.autograd.Function):
    """rewards [T, A] = rollout(actions [T, A, 2]) from the simulator's current state,
    differentiable with respect to the actions through the hand-written backward kernel
    (checkpoints every ``ckpt_every`` steps, recomputed in the backward pass).  With
    ``obs=True`` it returns (rewards, obs [T, A, 3 + 4P]), both differentiable."""

    @staticmethod
    def forward(ctx, actions: torch.Tensor, sim: Sim, ckpt_every: int = 10, obs: bool = False):
        actions = actions.detach().contiguous()
        ctx.sim = sim
        ctx.ckpt_every = ckpt_every
        ctx.obs = obs
        if obs:
            rewards, ckpt, states, o = sim.rollout_fwd(actions, ckpt_every, obs=True)
            ctx.save_for_backward(actions, ckpt, states)
            return rewards, o
        rewards, ckpt = sim.rollout_fwd(actions, ckpt_every)
        ctx.save_for_backward(actions, ckpt)
        return rewards

    @staticmethod
    def backward(ctx, grad_rewards, grad_obs=None):
        if ctx.obs:
            actions, ckpt, states = ctx.saved_tensors
            if grad_rewards is None:
                grad_rewards = torch.zeros(actions.shape[:2], dtype=torch.float32, device=actions.device)
            ga, _ = ctx.sim.rollout_bwd(actions, ckpt, grad_rewards.contiguous(), ctx.ckpt_every,
                                        grad_obs=grad_obs, states=states if grad_obs is not None else None)
        else:
            actions, ckpt = ctx.saved_tensors
            ga, _ = ctx.sim.rollout_bwd(actions, ckpt, grad_rewards.contiguous(), ctx.ckpt_every)
        return ga, None, None, None
