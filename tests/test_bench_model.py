"""Host logic of bench.py (no device): the algorithmic byte model of the step and LIDAR
kernels, the roofline fractions and the calibration of the HBM counters."""
import csv
import json

import numpy as np
import pytest

import bench
from paper_2408_01584_amd import scenes as S


def test_step_bytes_headline():
    """256 worlds x 64 agents, K 200, 63 partner slots, 4000 road points per world: per
    agent-step state 32 + static 16 + action 8 + flags 2 + reward 4 + ego 32 + partners
    25 x 63 + road observation 20 x 200 + the world's road 16 x 4000 / 64 = 6669 B."""
    sc = S.make_scene(1, worlds=[0, 1, 2])
    A = sc.num_agents
    per_agent = (32 + 16 + 8 + 2 + 4 + 32) + 25 * 63 + 20 * 200 + 16 * 4000 / 64
    assert per_agent == 6669
    assert bench.step_bytes(sc, 63 * A) == pytest.approx(per_agent * A)


def test_edge_segments_brute_force():
    sc = S.make_scene(0)
    m = np.asarray(sc.road_meta)
    n = 0
    for i in range(len(m) - 1):
        # a segment joins consecutive road-edge points of one polyline
        if (m[i] & 0xFF) == 1 and (m[i + 1] & 0xFF) == 1 and not (m[i] & 0x100):
            n += 1
    assert bench.edge_segments(sc) == n > 0
    p = sc.params
    assert bench.lidar_bytes(sc) == sc.num_agents * (8 * p.lidar_rays + 24) + 16 * n


def test_rooflines():
    r = bench.hbm_roofline("k", 8.0e9, 2.0)  # 8 GB in 2 ms = 4 TB/s
    assert r["frac"] == pytest.approx(0.5) and r["achieved"] == pytest.approx(4000.0)
    assert bench.VALU_PEAK == pytest.approx(78.6432e12)


def test_alu_roofline_from_record(monkeypatch):
    monkeypatch.setattr(bench, "counters_record", lambda k, t: {"valu_insts_per_launch": 1.0e9})
    r = bench.alu_roofline("k", "w", 2.0)  # 64 G lane operations in 2 ms = 32 T/s
    assert r["frac"] == pytest.approx(32e12 / bench.VALU_PEAK, rel=1e-3)
    monkeypatch.setattr(bench, "counters_record", lambda k, t: None)
    assert bench.alu_roofline("k", "w", 2.0)["frac"] is None


def _pmc_folder(path, counter, step_kib, copy_kib):
    path.mkdir()
    with open(path / "p_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d in range(3):
            w.writerow([d, "void gdk::k_step<256, 2>(gdk::SimArgs, gdk::StepCtl)", counter, step_kib])
        w.writerow([9, "__amd_rocclr_copyBuffer", counter, copy_kib])


def test_ingest_counters_calibration(tmp_path, monkeypatch):
    """Each counter is divided by what it reads for the 1 GiB copy over the copy's ideal
    bytes: FETCH_SIZE reading half of the copy counts double."""
    ideal = bench.COPY_ELEMS * 4 / 1024.0
    _pmc_folder(tmp_path / "f", "FETCH_SIZE", 1000.0, 0.5 * ideal)
    _pmc_folder(tmp_path / "w", "WRITE_SIZE", 3000.0, ideal)
    out = tmp_path / "rec.json"
    monkeypatch.setattr(bench, "PMC_FILE", str(out))
    bench.ingest_counters(str(tmp_path / "f"), str(tmp_path / "w"))
    rec = json.load(open(out))
    assert rec["hbm_bytes_per_launch"] == round((1000.0 / 0.5 + 3000.0) * 1024)
    assert rec["counters"]["FETCH_SIZE"]["launches"] == 3
