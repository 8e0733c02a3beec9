#!/usr/bin/env python3
"""Throughput of the batched driving-simulator step on one MI355X.

Metric: agent steps per second (ASPS = S * sum_k |A_k| / dT, Sec. 4.1) of the full step
(dynamics, collision, reward/done/auto-reset, ego + partner + road top-K observation).

Default workload: 256 worlds x 64 agents, 4000 road points per world (seeded 3x3
intersection grids on 100 m blocks), top-K 200 road points, 63 partner slots, radius
50 m, dt 0.1 s, 91-step episodes with auto-reset, random actions.  Inputs are resident in
HBM before the timed region; each step writes its observation into the next slot of a
rollout ring larger than the 256 MB Infinity Cache, as a training loop would.

Prints one JSON line.  `--gpus N` with N > 1 exits: this benchmark uses one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, B/s
# Vector-ALU ceiling of MI355X: the published FP32 vector rate, 157.3 TFLOP/s = 256 CUs x
# 2.4 GHz x 256 FLOP per clock, i.e. 128 lane-operations per CU per clock counting an FMA as
# one operation (two wave64 instructions per CU per clock).  Measured on the part: simple
# integer and min/max instructions issue at up to 1.4 wave64 instructions per CU per clock,
# FP32 FMA (without packed FP32, which this build never emits) at 0.9
VALU_PEAK = 256 * 128 * 2.4e9
WORKLOAD_TAG = "256w_64a_4000r_k200"
WORKLOADS = {0: "1w_8a_500r_k64", 1: WORKLOAD_TAG, 2: "1024w_uneven", 3: "512w_32a_2000r_k64",
             4: "4096w_64a_6000r_n30"}
PMC_FILE = os.path.join(ROOT, "profiles", "k_step_%s_hbm_counters.json" % WORKLOAD_TAG)
COPY_ELEMS = 1 << 28  # float32 elements of the calibration copy (1 GiB each way)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=91)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--ring-mb", type=int, default=1536, help="observation ring size (MB)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--graph", action="store_true",
                    help="replay a HIP graph per step instead of launching the kernel directly")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--cpu-baselines", action="store_true",
                    help="time the oracle on bounded samples of every workload (host cores only)")
    ap.add_argument("--ingest", action="store_true",
                    help="time the road decimation of the headline workload's map sampled every "
                         "0.1 m, and the step on the decimated map")
    ap.add_argument("--config", type=int, default=1, choices=(0, 1, 2, 3, 4),
                    help="1 (default): the headline workload; 0, 2, 3, 4: the secondary "
                         "workloads (latency, uneven batch, differentiable rollout, LIDAR + "
                         "rollout at 4096 worlds), one JSON line each")
    ap.add_argument("--profile-run", action="store_true",
                    help="no timing: a few steps of workload --config (and, for 3 and 4, two rollouts "
                         "forward + backward) for a profiler to record; the 4096-world workload repeats "
                         "its first 64 worlds (same sizes, 1/64 of the generation time)")
    ap.add_argument("--ingest-sq", nargs="+", metavar="ARG",
                    help="KERNEL TAG FOLDER SOURCE...: turn a rocprofv3 --pmc folder (SQ_INSTS_VALU, "
                         "SQ_ACTIVE_INST_VALU, ...) into the instruction-counter record of KERNEL on "
                         "workload TAG, keyed by the digest of the SOURCE files, then exit")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc output folders (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-calibration run into the HBM-traffic record, then exit")
    return ap.parse_args()


def source_digest(*names):
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(ROOT, "paper_2408_01584_amd", "csrc", n), "rb").read())
    return h.hexdigest()[:16]


def _counter_rows(folder, counter):
    """{dispatch id: (kernel name, value)} of one counter from a rocprofv3 --pmc folder."""
    import csv
    import glob
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % folder)
    out = {}
    for f in files:
        for row in csv.DictReader(open(f)):
            if row["Counter_Name"] != counter:
                continue
            key = (f, row["Dispatch_Id"])
            name, v = out.get(key, (row["Kernel_Name"], 0.0))
            out[key] = (name, v + float(row["Counter_Value"]))
    return out


def ingest_counters(fetch_dir, write_dir):
    """HBM bytes per k_step launch: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each
    scaled by what the same counter reads for the 1 GiB calibration copy."""
    res = {}
    for counter, folder in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(folder, counter)
        step = [v for n, v in rows.values() if "k_step" in n]
        copies = [v for n, v in rows.values() if "copyBuffer" in n or "copy" in n.lower()]
        if not step or not copies:
            raise SystemExit("%s: k_step or copy dispatches missing" % counter)
        big = max(copies)
        calib = [v for v in copies if v > 0.5 * big]
        ideal_kib = COPY_ELEMS * 4 / 1024.0
        factor = (sum(calib) / len(calib)) / ideal_kib
        res[counter] = {"kib_per_launch": sum(step) / len(step), "launches": len(step),
                        "copy_kib": sum(calib) / len(calib), "copy_ideal_kib": ideal_kib,
                        "factor": factor}
    hbm = sum(r["kib_per_launch"] / r["factor"] for r in res.values()) * 1024.0
    rec = {"kernel": "k_step", "workload": WORKLOAD_TAG,
           "source_digest": source_digest("gd_step.hip", "gd_internal.h"),
           "hbm_bytes_per_launch": round(hbm), "counters": res}
    with open(PMC_FILE, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec))


def ingest_sq(kernel, tag, folder, *sources):
    """Mean per dispatch of every counter in the folder for `kernel` (dispatches whose
    name contains it), written to profiles/<kernel>_<tag>_sq_counters.json."""
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            if kernel not in row["Kernel_Name"]:
                continue
            d = per.setdefault((f, row["Dispatch_Id"]), {})
            d[row["Counter_Name"]] = d.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    if not per:
        raise SystemExit("no %s dispatches under %s" % (kernel, folder))
    names = sorted({k for d in per.values() for k in d})
    mean = {k: sum(d.get(k, 0.0) for d in per.values()) / len(per) for k in names}
    rec = {"kernel": kernel, "workload": tag, "sources": list(sources),
           "source_digest": source_digest(*sources), "dispatches": len(per),
           "counters_per_launch": mean,
           "valu_insts_per_launch": mean.get("SQ_INSTS_VALU")}
    with open(os.path.join(ROOT, "profiles", "%s_%s_sq_counters.json" % (kernel, tag)), "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec))


def profile_run(args):
    import torch

    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim
    c = args.config
    torch.cuda.set_device(0)
    if c == 4:
        spec = S.CONFIGS[4]
        base = [S.make_world(4, w, spec.worlds) for w in range(64)]
        scene = S.assemble(4, [base[i % 64] for i in range(spec.worlds)], spec.params,
                           world_ids=[i % 64 for i in range(spec.worlds)])
    else:
        scene = S.make_scene(c)
    print("[bench] profile run: workload %d, %d agents" % (c, scene.num_agents), file=sys.stderr, flush=True)
    sim = Sim(scene)
    T = S.CONFIGS[c].steps
    acts = torch.as_tensor(S.make_actions(c, T + 4, scene.num_agents), device="cuda")
    for k in range(min(args.steps, T + 4)):
        sim.step(acts[k])
    if c in (3, 4):
        ra = acts[:T].contiguous()
        for _ in range(2):
            r, ck = sim.rollout_fwd(ra, 10)
            sim.rollout_bwd(ra, ck, torch.ones_like(r), 10)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": c, "steps": min(args.steps, T + 4)}), flush=True)


def main():
    args = parse()
    if args.profile_run:
        profile_run(args)
        return
    if args.ingest_sq:
        ingest_sq(*args.ingest_sq)
        return
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the simulator step shards by whole worlds with "
              "no exchange between GPUs, and this build measures one GPU's share (--gpus 1).",
              file=sys.stderr)
        sys.exit(2)
    if args.ingest:
        ingest_leg(args)
        return
    if args.cpu_baselines:
        print(json.dumps(cpu_baselines_all()), flush=True)
        return
    if args.config != 1:
        secondary(args)
        return
    import numpy as np
    import torch

    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg_id = 1
    scene = S.make_scene(cfg_id)
    p = scene.params
    A, W = scene.num_agents, scene.num_worlds
    K, P = p.top_k, p.partners
    sim = Sim(scene, graph=args.graph)
    T = args.steps + args.warmup
    actions = torch.as_tensor(S.make_actions(cfg_id, T, A), device=dev)

    # observation ring (> Infinity Cache) so every step's writes reach HBM
    Sl = sim.S
    step_obs_bytes = A * 8 * 4 + Sl * 6 * 4 + Sl + A * K * 16 + A * K * 4
    n_slots = max(2, math.ceil(args.ring_mb * 1e6 / step_obs_bytes))
    ring = dict(ego=torch.empty((n_slots, A, 8), device=dev), partner=torch.empty((n_slots, Sl, 6), device=dev),
                pmask=torch.empty((n_slots, Sl), dtype=torch.uint8, device=dev),
                road=torch.empty((n_slots, A, K, 4), device=dev),
                road_idx=torch.empty((n_slots, A, K), dtype=torch.int32, device=dev))

    def bind(k, target=None):
        s = k % n_slots
        (target or sim).set_obs_buffers(ring["ego"][s], ring["partner"][s], ring["pmask"][s],
                                        ring["road"][s], ring["road_idx"][s])

    for k in range(args.warmup):
        bind(k)
        sim.step(actions[k])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for k in range(args.steps):
        bind(args.warmup + k)
        sim.step(actions[args.warmup + k])
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)

    # controlled-agent (CASPS-like) share: agents observed per step, untimed replay
    vis = 0
    for k in range(min(args.steps, 91)):
        sim.step(actions[k % T])
        vis += int(((sim.buf["flags"] & 32) != 0).sum().item())
    vis_frac = vis / (A * min(args.steps, 91))

    value = A * args.steps / (ms / 1e3)
    # the fused step kernel; algorithmic bytes per agent-step:
    #   state read + write 32, length/width/goal 16, action 8, flags 2, reward 4, ego 32,
    #   partners 25 P (24 B features + mask), road observation 20 K (16 B row + index),
    #   the world's road read once (16 B per point: x, y, direction, type)
    R_w = scene.num_road / W
    A_w = A / W
    unit_bytes = 32 + 16 + 8 + 2 + 4 + 32 + 25 * P + 20 * K + 16 * R_w / A_w
    launch_bytes = unit_bytes * A
    # the timed region holds nothing but back-to-back step-kernel launches on this stream,
    # so its event-timed length per step is the kernel's average launch duration
    step_ms = ms / args.steps
    achieved = launch_bytes / (step_ms / 1e3)
    traffic = None
    if os.path.exists(PMC_FILE):
        pm = json.load(open(PMC_FILE))
        if pm.get("source_digest") == source_digest("gd_step.hip", "gd_internal.h") and \
                pm.get("workload") == WORKLOAD_TAG:
            traffic = pm["hbm_bytes_per_launch"]
    out = {
        "metric": "agent-steps/sec (full step) on 1 MI355X",
        "value": round(value, 1),
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256 worlds x 64 agents, 4000 road points per world (3x3 intersection "
                               "grid, 100 m blocks), top-K 200, 63 partners, radius 50 m, dt 0.1 s, "
                               "91-step episodes with auto-reset, random actions",
                   "worlds": W, "agents": A, "road_points_per_world": int(R_w), "top_k": K,
                   "partners": P, "obs_ring_slots": n_slots},
        "roofline": {"kernel": "k_step", "bound": "hbm", "achieved": round(achieved / 1e9, 1),
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4),
                     "traffic": traffic, "algorithmic_bytes_per_launch": int(launch_bytes),
                     "bytes_per_agent_step": round(unit_bytes, 1), "avg_launch_ms": round(step_ms, 5),
                     "launches_timed": args.steps},
        # the same kernel against the vector-ALU ceiling (its instruction counters)
        "roofline_alu": alu_roofline("k_step", WORKLOAD_TAG, step_ms),
        "step": {"launch": "graph" if args.graph else "direct",
                 "launch_shape": sim.launch or "library default",
                 "observed_agent_fraction": round(vis_frac, 4),
                 "active_agent_steps_per_s": round(value * vis_frac, 1)},
        # the paper's own figure, for context only: another simulator implementation, other
        # hardware and other scenes (vs_baseline stays null)
        "context": {"paper_peak_agent_steps_per_s": 2.3e6,
                    "paper_source": "Sec. 4.1, Fig. 3 (peak ASPS over the number of worlds)",
                    "paper_hardware": "NVIDIA consumer and datacenter GPUs (RTX 4080 / A100 class); "
                                      "precision not stated",
                    "paper_workload": "Waymo Open Motion Dataset scenes, radius-filter observation"},
    }
    if args.copy_calibration:
        a = torch.empty(COPY_ELEMS, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * a.numel() * 4
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg_id, args.cpu_steps)
    print(json.dumps(out), flush=True)


def edge_segments(scene) -> int:
    """Road-edge segments of a scene: consecutive edge points of one polyline."""
    import numpy as np
    m = np.asarray(scene.road_meta)
    is_edge = (m & 0xFF) == 1
    last = (m & 0x100) != 0
    return int((is_edge[:-1] & is_edge[1:] & ~last[:-1]).sum())


def step_bytes(scene, slots):
    """Algorithmic bytes of one step-kernel launch: per agent state read + write 32,
    length/width/goal 16, action 8, flags 2, reward 4, ego 32, road observation 20 K;
    25 per partner slot (24 B features + mask); each world's road read once (16 B per
    point)."""
    p = scene.params
    A = scene.num_agents
    return A * (32 + 16 + 8 + 2 + 4 + 32 + 20 * p.top_k) + 25 * slots + 16 * scene.num_road


def lidar_bytes(scene):
    """Algorithmic bytes of one LIDAR launch: per agent 8 B per ray written (distance,
    hit type) and its pose and box read (24 B); each world's edge segments read once
    (16 B)."""
    return scene.num_agents * (8 * scene.params.lidar_rays + 24) + 16 * edge_segments(scene)


def counters_record(kernel, tag):
    """Instruction counters of `kernel` on workload `tag` from profiles/, when they were
    taken on the current kernel source."""
    f = os.path.join(ROOT, "profiles", "%s_%s_sq_counters.json" % (kernel, tag))
    if not os.path.exists(f):
        return None
    rec = json.load(open(f))
    if rec.get("source_digest") != source_digest(*rec.get("sources", [])):
        return None
    return rec


def alu_roofline(kernel, tag, avg_ms):
    """VALU issue rate of a kernel: wave instructions per launch (from the committed
    counters) x 64 lanes / its average launch time, against VALU_PEAK."""
    rec = counters_record(kernel, tag)
    if rec is None:
        return {"kernel": kernel, "bound": "alu", "achieved": None, "peak": VALU_PEAK / 1e12,
                "unit": "TOP/s", "frac": None, "note": "no counters for the current source"}
    ops = rec["valu_insts_per_launch"] * 64
    ach = ops / (avg_ms / 1e3)
    return {"kernel": kernel, "bound": "alu", "achieved": round(ach / 1e12, 3), "peak": VALU_PEAK / 1e12,
            "unit": "TOP/s", "frac": round(ach / VALU_PEAK, 4), "avg_launch_ms": round(avg_ms, 5),
            "valu_wave_insts_per_launch": rec["valu_insts_per_launch"]}


def hbm_roofline(kernel, nbytes, avg_ms):
    ach = nbytes / (avg_ms / 1e3)
    return {"kernel": kernel, "bound": "hbm", "achieved": round(ach / 1e9, 1), "peak": HBM_PEAK / 1e9,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK, 4), "traffic": None,
            "algorithmic_bytes_per_launch": int(nbytes), "avg_launch_ms": round(avg_ms, 5)}


def _timed(fn, reps=5):
    """Median over `reps` event-timed calls of fn() on the current stream (ms)."""
    import torch
    out = []
    for _ in range(reps):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        fn()
        t1.record()
        torch.cuda.synchronize()
        out.append(t0.elapsed_time(t1))
    return sorted(out)[len(out) // 2]


def secondary(args):
    """Secondary workloads: config 0 (one world, launch latency), 2 (1024 uneven worlds,
    direct launches against a HIP graph per step), 3 (512 x 32, T = 20: step, and the
    differentiable rollout forward against forward + backward) and 4 (4096 x 64 with
    30-ray LIDAR, T = 91 rollout with checkpoints every 10 steps); for 3 and 4 also the
    simplified model's step and its action inversion.  Median of 5 repeats."""
    import torch

    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim

    c = args.config
    torch.cuda.set_device(0)
    print("[bench] generating workload %d" % c, file=sys.stderr, flush=True)
    scene = S.make_scene(c)
    print("[bench] workload %d ready: %d worlds, %d agents" % (c, scene.num_worlds, scene.num_agents),
          file=sys.stderr, flush=True)
    p = scene.params
    A, W = scene.num_agents, scene.num_worlds
    T = S.CONFIGS[c].steps
    acts = torch.as_tensor(S.make_actions(c, T + 10, A), device="cuda")
    out = {"metric": "agent-steps/sec (full step) on 1 MI355X", "config_id": c, "worlds": W,
           "agents": A, "road_points": scene.num_road, "top_k": p.top_k, "partners": p.partners,
           "lidar_rays": p.lidar_rays, "steps": T, "unit": "agent-steps/s"}

    def run_steps(sim, n):
        def f():
            for k in range(n):
                sim.step(acts[k])
        return f

    modes = (("direct", False), ("graph", True)) if c in (0, 2) else (("direct", False),)
    for name, graph in modes:
        sim = Sim(scene, graph=graph)
        run_steps(sim, 10)()
        ms = _timed(run_steps(sim, T))
        out[name] = {"ms_per_step": round(ms / T, 5), "value": round(A * T / (ms / 1e3), 1),
                     "launch_shape": sim.launch or "library default"}
        if name == "direct":
            out["value"] = out[name]["value"]
            out["ms_per_step"] = out[name]["ms_per_step"]
            # per-kernel launch times (HIP events around each launch), then the rooflines:
            # the step kernel against HBM, the LIDAR kernel against HBM and VALU issue
            from paper_2408_01584_amd import gd as G
            sim.set_timing(True)
            sim.get_timing()
            run_steps(sim, T)()
            torch.cuda.synchronize()
            tms, tcnt = sim.get_timing()
            sim.set_timing(False)
            k_ms = tms[G.GD_PHASE_STEP] / max(tcnt[G.GD_PHASE_STEP], 1)
            sb = step_bytes(scene, sim.S)
            out["roofline"] = hbm_roofline("k_step", sb, k_ms)
            out["roofline"]["bytes_per_agent_step"] = round(sb / A, 1)
            if p.lidar_rays > 0:
                l_ms = tms[G.GD_PHASE_LIDAR] / max(tcnt[G.GD_PHASE_LIDAR], 1)
                lb = lidar_bytes(scene)
                out["roofline_lidar"] = hbm_roofline("k_lidar", lb, l_ms)
                out["roofline_lidar_alu"] = alu_roofline("k_lidar", WORKLOADS[c], l_ms)
                out["roofline_step"] = hbm_roofline("k_step + k_lidar", sb + lb, ms / T)
        sim.close()
        del sim
        torch.cuda.empty_cache()

    if c in (0, 2):
        # the caller captures a whole episode's direct-launch steps in one HIP graph
        sim = Sim(scene)
        run_steps(sim, 10)()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            run_steps(sim, T)()
        torch.cuda.synchronize()
        ms = _timed(g.replay)
        out["captured"] = {"ms_per_step": round(ms / T, 5), "value": round(A * T / (ms / 1e3), 1),
                           "note": "%d steps captured by the caller in one HIP graph (torch.cuda.graph)" % T}
        del g
        sim.close()
        del sim
        torch.cuda.empty_cache()

    if c in (3, 4):
        C = 10
        sim = Sim(scene)
        ra = acts[:T].contiguous()
        rewards, ckpt = sim.rollout_fwd(ra, C)
        gr = torch.ones_like(rewards)
        sim.rollout_bwd(ra, ckpt, gr, C)
        fwd = _timed(lambda: sim.rollout_fwd(ra, C))
        rewards, ckpt = sim.rollout_fwd(ra, C)

        def fb():
            r, ck = sim.rollout_fwd(ra, C)
            sim.rollout_bwd(ra, ck, gr, C)
        fwdbwd = _timed(fb)
        from paper_2408_01584_amd import gd as G
        sim.set_timing(True)
        sim.get_timing()
        fb()
        torch.cuda.synchronize()
        tms, tcnt = sim.get_timing()
        sim.set_timing(False)
        f_ms = tms[G.GD_PHASE_ROLLOUT_FWD] / max(tcnt[G.GD_PHASE_ROLLOUT_FWD], 1)
        b_ms = tms[G.GD_PHASE_ROLLOUT_BWD] / max(tcnt[G.GD_PHASE_ROLLOUT_BWD], 1)
        rollout_alu = {"fwd": alu_roofline("k_rollout_fwd", WORKLOADS[c], f_ms),
                       "bwd": alu_roofline("k_rollout_bwd", WORKLOADS[c], b_ms)}
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        fb()
        torch.cuda.synchronize()
        peak_ck = torch.cuda.max_memory_allocated() - base
        out["rollout"] = {
            "T": T, "ckpt_every": C,
            "fwd_agent_steps_per_s": round(A * T / (fwd / 1e3), 1),
            "fwd_bwd_agent_steps_per_s": round(A * T / (fwdbwd / 1e3), 1),
            "fwd_bwd_over_fwd_time": round(fwdbwd / fwd, 3),
            "checkpoint_bytes": int(ckpt.numel() * 4),
            "checkpoint_bytes_every_step": int(T * 4 * A * 4),
            "peak_extra_bytes_fwd_bwd": int(peak_ck),
            "roofline_alu": rollout_alu}
        sim.close()
        del sim
        torch.cuda.empty_cache()
        out["delta"] = delta_model_legs(scene, T, c)
        if p.lidar_rays > 0:
            out["view_cone"] = view_cone_leg(scene, T, c)
    print(json.dumps(out), flush=True)


def view_cone_leg(scene, T, c):
    """The full step with the LIDAR as a 120-degree view cone of the same ray count, the
    head of every agent turned at random before each step (the head-rotation input)."""
    import dataclasses
    import math

    import numpy as np
    import torch

    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim

    A = scene.num_agents
    acts = torch.as_tensor(S.make_actions(c, T + 10, A), device="cuda")
    heads = torch.as_tensor(np.random.default_rng(5).uniform(-1.5, 1.5, (T + 10, A)).astype(np.float32),
                            device="cuda")
    sim = Sim(scene, params=dataclasses.replace(scene.params, lidar_fov=math.radians(120.0)))
    head = sim.buf["lidar_head"]

    def steps(n):
        def f():
            for k in range(n):
                head[:A].copy_(heads[k])
                sim.step(acts[k])
        return f
    steps(10)()
    ms = _timed(steps(T))
    sim.close()
    return {"fov_deg": 120.0, "rays": scene.params.lidar_rays, "ms_per_step": round(ms / T, 5),
            "agent_steps_per_s": round(A * T / (ms / 1e3), 1),
            "note": "includes one device copy of the head angles per step"}


def ingest_leg(args):
    """Road decimation at ingest (Sec. 3.1) on the headline workload's 256 worlds with the
    road polylines sampled every 0.1 m (about 103 000 points per world, 26.4 M in all):
    Visvalingam-Whyatt with min_area 0.01 m^2 (median of 5 launches, inputs resident),
    then 91 steps of the simulator on the decimated map.  Latency-bound (each polyline's
    removals are sequential); algorithmic bytes 13 per input point (x, y read; keep, dir
    written)."""
    import numpy as np
    import torch

    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.ingest import decimate_road, decimate_scene, polyline_offsets
    from paper_2408_01584_amd.sim import Sim

    torch.cuda.set_device(0)
    min_area = 0.01
    dense = dict(spacing=0.1, wobble=0.3, wavelength=40.0, jitter=0.002)
    print("[bench] generating the dense map", file=sys.stderr, flush=True)
    sc = S.make_scene(1, dense=dense)
    po = polyline_offsets(sc.road_meta)
    dev = torch.device("cuda")
    x = torch.as_tensor(sc.road_x, device=dev)
    y = torch.as_tensor(sc.road_y, device=dev)
    pot = torch.as_tensor(po, device=dev)
    decimate_road(x, y, pot, min_area)
    ms = _timed(lambda: decimate_road(x, y, pot, min_area))
    dsc, keep = decimate_scene(sc, min_area)
    n = sc.num_road
    out = {"metric": "road points decimated/s on 1 MI355X", "unit": "points/s",
           "value": round(n / (ms / 1e3), 1), "ms_per_launch": round(ms, 3),
           "config": {"workload": "256 worlds of the headline map, polylines sampled every 0.1 m "
                                  "with a 0.3 m wobble and 2 mm jitter; Visvalingam-Whyatt, "
                                  "min_area 0.01 m^2", "points": n, "polylines": len(po) - 1,
                      "longest_polyline": int(np.diff(po).max())},
           "kept": int(keep.sum()), "reduction": round(n / max(int(keep.sum()), 1), 2),
           "bound": "latency", "algorithmic_bytes_per_launch": 13 * n}
    del x, y, pot
    # the step on the decimated map against the fixed 4000-point map of the headline
    A = dsc.num_agents
    acts = torch.as_tensor(S.make_actions(1, 101, A), device=dev)
    for name, scene in (("decimated", dsc), ("fixed_4000", S.make_scene(1))):
        sim = Sim(scene)

        def run(k0, n_steps):
            def f():
                for k in range(n_steps):
                    sim.step(acts[k0 + k])
            return f
        run(0, 10)()
        ms_s = _timed(run(10, 91))
        out["step_" + name] = {"road_points_per_world": round(scene.num_road / scene.num_worlds, 1),
                               "ms_per_step": round(ms_s / 91, 5),
                               "agent_steps_per_s": round(A * 91 / (ms_s / 1e3), 1)}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    out["cpu_baseline"] = cpu_baseline_decimation(dense, min_area)
    print(json.dumps(out), flush=True)


def delta_model_legs(scene, T, c):
    """The simplified (invertible) bicycle model on the same workload: the full step with
    it, and the expert-action inversion of a T-step log of every agent (one launch, HBM
    bound: reads heading and speed of T+1 states, writes T actions, 16 B per agent-step)."""
    import dataclasses

    import torch

    from paper_2408_01584_amd import gd as G
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim

    A = scene.num_agents
    acts = torch.as_tensor(S.make_delta_actions(c, T + 10, A), device="cuda")
    sim = Sim(scene, params=dataclasses.replace(scene.params, dynamics=G.GD_DYN_DELTA))

    def steps(n):
        def f():
            for k in range(n):
                sim.step(acts[k])
        return f
    steps(10)()
    ms = _timed(steps(T))
    _, log = sim.rollout_fwd(acts[:T + 1].contiguous(), 1)  # [T+1, 4, A]
    inv = torch.empty((T, A, 2), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    reps = 20

    def invert():
        for _ in range(reps):
            G.gd_invert_actions(sim.handle, log.data_ptr(), T, inv.data_ptr(), stream)
    invert()
    ms_inv = _timed(invert) / reps
    nbytes = A * ((T + 1) * 8 + T * 8)
    gbs = nbytes / (ms_inv * 1e-3) / 1e9
    # a device-to-device copy moving the same bytes (half read, half written), for context
    src = torch.empty(nbytes // 8, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)

    def copy():
        for _ in range(reps):
            dst.copy_(src)
    copy()
    ms_copy = _timed(copy) / reps
    del src, dst
    sim.close()
    return {"step_ms": round(ms / T, 5), "step_agent_steps_per_s": round(A * T / (ms / 1e3), 1),
            "invert": {"T": T, "ms_per_launch": round(ms_inv, 5),
                       "agent_steps_per_s": round(A * T / (ms_inv / 1e3), 1),
                       "algorithmic_bytes_per_launch": nbytes, "achieved_GBps": round(gbs, 1),
                       "hbm_frac": round(gbs * 1e9 / HBM_PEAK, 4),
                       "same_bytes_copy_GBps": round(nbytes / (ms_copy * 1e-3) / 1e9, 1)}}


def cpu_baselines_all():
    """The oracle (plain C, OpenMP over worlds) on bounded samples of every workload, on the
    host's cores: the full step for configs 0, 2 (64 of its 1024 worlds) and 4 (32 of 4096
    worlds, LIDAR included), and the differentiable rollout forward and vector-Jacobian
    product for config 3 (all 512 worlds, T = 20)."""
    import numpy as np

    from oracle import oracle as O
    from paper_2408_01584_amd import scenes as S
    O.build(force=False)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"kind": "oracle", "cores": cores, "unit": "agent-steps/s"}
    for c, worlds, steps in ((0, None, 91), (2, 64, 20), (4, 32, 3)):
        sc = S.make_scene(c, worlds=worlds) if worlds else S.make_scene(c)
        acts = S.make_actions(c, steps + 1, sc.num_agents).astype(np.float64)
        sim = O.OracleSim(sc)
        sim.step(acts[0])
        t = time.perf_counter()
        for k in range(1, steps + 1):
            sim.step(acts[k])
        dt = time.perf_counter() - t
        out["config_%d" % c] = {"value": round(sc.num_agents * steps / dt, 1),
                                "sample": "%d worlds x %d steps, %.2f s" % (sc.num_worlds, steps, dt)}
    sc = S.make_scene(3)
    T = 20
    acts = S.make_actions(3, T, sc.num_agents).astype(np.float64)
    sim = O.OracleSim(sc)
    t = time.perf_counter()
    sim.rollout(acts)
    dt_f = time.perf_counter() - t
    t = time.perf_counter()
    sim.rollout_vjp(acts, np.ones((T, sc.num_agents)))
    dt_b = time.perf_counter() - t
    out["config_3"] = {"rollout_fwd": round(sc.num_agents * T / dt_f, 1),
                       "rollout_vjp": round(sc.num_agents * T / dt_b, 1),
                       "sample": "512 worlds, T = 20, %.2f s + %.2f s" % (dt_f, dt_b)}
    return out


def cpu_baseline_decimation(dense, min_area):
    """The oracle's decimation (plain C, OpenMP over polylines) on a bounded sample of the
    dense map: 8 of its 256 worlds."""
    from oracle import oracle as O
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.ingest import polyline_offsets
    O.build(force=False)
    sub = S.make_scene(1, worlds=8, dense=dense)
    spo = polyline_offsets(sub.road_meta)
    t = time.perf_counter()
    O.decimate(spo, sub.road_x, sub.road_y, min_area)
    dt = time.perf_counter() - t
    return {"value": round(sub.num_road / dt, 1), "unit": "points/s", "kind": "oracle",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "sample": "8 of the 256 worlds (%d points), %.2f s" % (sub.num_road, dt)}


def cpu_baseline(cfg_id, steps):
    """The FP64 oracle (plain C, OpenMP over worlds) on a bounded sample of the same
    workload: all worlds for `steps` steps."""
    import numpy as np

    from oracle import oracle as O
    from paper_2408_01584_amd import scenes as S
    O.build(force=False)
    scene = S.make_scene(cfg_id)
    acts = S.make_actions(cfg_id, steps, scene.num_agents).astype(np.float64)
    sim = O.OracleSim(scene)
    sim.step(acts[0])  # warm
    t = time.perf_counter()
    for k in range(1, steps):
        sim.step(acts[k])
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(scene.num_agents * (steps - 1) / dt, 1), "unit": "agent-steps/s",
            "cores": cores, "kind": "oracle",
            "sample": "all %d worlds of the workload for %d steps (FP64 C oracle, OpenMP over "
                      "worlds, %.1f s wall)" % (scene.num_worlds, steps - 1, dt)}


if __name__ == "__main__":
    main()
