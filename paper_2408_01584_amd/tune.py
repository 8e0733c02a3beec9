"""Autotuner for the launch shape of the fused step kernel.

The kernel has five free parameters that do not change its results (the GPU tests check
that every shape gives the same bits): waves per workgroup, number of distance bins of
the top-K selection, candidate-list entries per wave, the cell size of the per-world road
grid, and whether the road is staged in LDS or read through the caches.  Which shape is fastest depends on the batch (agents and road points per
world, K) and on the device, so it is measured: every candidate shape steps the given
scene a few times and the one with the lowest mean step time wins.

Results are cached in a JSON file keyed by the workload signature and the device name.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

CACHE = os.environ.get("GD_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                     "tuned_shapes.json"))

DEFAULT_SPACE = [
    dict(obs_waves=w, obs_bins=b, obs_cands=c, cell_size=cs, obs_road=rd)
    for rd in (1, 2)  # GD_ROAD_LDS, GD_ROAD_GLOBAL
    for w in (16, 12, 8)
    for c in (512, 768)
    for b in (256, 512, 1024)
    for cs in (10.0, 15.0)
]


def signature(scene, params, graph: bool) -> str:
    """Workload key: sizes of every world, observation parameters, graph mode."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.diff(scene.agent_off), np.int32).tobytes())
    h.update(np.ascontiguousarray(np.diff(scene.road_off), np.int32).tobytes())
    h.update(repr((params.top_k, params.partners, params.lidar_rays, params.obs_radius,
                   params.lidar_range, graph)).encode())
    return h.hexdigest()[:20]


def _device_name() -> str:
    """Device key: architecture and compute-unit count (the marketing name is left out: it
    depends on whether the driver's ID table is installed, and a profiler can change it)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    return "%s:%d" % (getattr(p, "gcnArchName", ""), p.multi_processor_count)


def _load():
    try:
        return json.load(open(CACHE))
    except (OSError, ValueError):
        return {}


def time_shape(scene, params, shape, actions, steps=20, warmup=5, graph=False) -> float:
    """Mean milliseconds per gd_step of `scene` with launch `shape`."""
    import torch

    from .sim import Sim
    sim = Sim(scene, params=params, graph=graph, **shape)
    try:
        for k in range(warmup):
            sim.step(actions[k % actions.shape[0]])
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for k in range(steps):
            sim.step(actions[(warmup + k) % actions.shape[0]])
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps
    finally:
        sim.close()


def cached_shape(scene, params=None, graph=False):
    """The launch shape the autotuner found for this workload on this device, or None."""
    params = params if params is not None else scene.params
    cache, dev = _load(), "@" + _device_name()
    rec = cache.get(signature(scene, params, graph) + dev)
    if rec is None and graph:
        # a launch shape is a property of the kernel, not of how it is launched: without a
        # record of its own, a graph-mode simulator takes the direct-launch shape
        rec = cache.get(signature(scene, params, False) + dev)
    return None if rec is None else dict(rec["shape"])


def autotune(scene, params=None, space=None, steps=20, warmup=5, graph=False, use_cache=True,
             verbose=False) -> dict:
    """Fastest launch shape for this scene on this device (cached)."""
    import torch

    from .scenes import make_actions
    params = params if params is not None else scene.params
    key = signature(scene, params, graph) + "@" + _device_name()
    cache = _load() if use_cache else {}
    if key in cache:
        return dict(cache[key]["shape"])
    space = space if space is not None else DEFAULT_SPACE
    acts = torch.as_tensor(make_actions(scene.cfg, steps + warmup, scene.num_agents), device="cuda")
    results = []
    for shape in space:
        try:
            ms = time_shape(scene, params, shape, acts, steps, warmup, graph)
        except RuntimeError as e:  # a shape that does not fit this workload
            if verbose:
                print("tune: skip", shape, e, flush=True)
            continue
        results.append((ms, shape))
        if verbose:
            print("tune: %.4f ms %s" % (ms, shape), flush=True)
    if not results:
        return {}
    ms, best = min(results, key=lambda r: r[0])
    if use_cache:
        cache = _load()
        cache[key] = {"shape": best, "ms_per_step": ms, "candidates": len(results)}
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    return dict(best)


def main():
    """python -m paper_2408_01584_amd.tune --config N [...]: tune the workload's launch
    shape on this device and cache it (GD_TUNE_CACHE names the cache file)."""
    import argparse

    from .scenes import make_scene
    ap = argparse.ArgumentParser(description=main.__doc__.split(":")[0])
    ap.add_argument("--config", type=int, nargs="+", default=[1])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--graph", action="store_true")
    args = ap.parse_args()
    for c in args.config:
        scene = make_scene(c)
        best = autotune(scene, steps=args.steps, graph=args.graph, verbose=True)
        print(json.dumps({"config": c, "shape": best}), flush=True)


if __name__ == "__main__":
    main()
