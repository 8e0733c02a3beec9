"""The C-ABI library loads, exports every entry point that include/gd.h declares, and
validates its arguments on the host (no GPU needed for any call made here)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gd.h")


def declared_entry_points():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gd_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def G():
    from paper_2408_01584_amd import gd
    if not os.path.exists(gd.LIB_PATH):
        from paper_2408_01584_amd import build
        build.build()
    gd.lib()
    return gd


def test_every_declared_symbol_is_exported(G):
    names = declared_entry_points()
    assert len(names) >= 11, names
    out = subprocess.check_output(["nm", "-D", "--defined-only", G.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(G.ENTRY_POINTS)
    for n in names:
        assert hasattr(G.lib(), n)


def test_struct_layout_matches_header(G):
    """ctypes mirrors of gd_config / gd_buffers have the C sizes and offsets."""
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "gd.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(gd_config), offsetof(gd_config, cell_size),
         offsetof(gd_config, obs_cands), offsetof(gd_config, obs_road),
         offsetof(gd_config, dynamics), offsetof(gd_config, lidar_fov), offsetof(gd_config, min_goal_dist),
         sizeof(gd_buffers), offsetof(gd_buffers, lidar_head), offsetof(gd_buffers, agent_class),
         offsetof(gd_buffers, t), offsetof(gd_buffers, workspace_bytes));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        open(src, "w").write(prog)
        exe = os.path.join(d, "l")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, src])
        vals = [int(v) for v in subprocess.check_output([exe], text=True).split()]
    want = [C.sizeof(G.gd_config), G.gd_config.cell_size.offset, G.gd_config.obs_cands.offset,
            G.gd_config.obs_road.offset, G.gd_config.dynamics.offset, G.gd_config.lidar_fov.offset,
            G.gd_config.min_goal_dist.offset, C.sizeof(G.gd_buffers), G.gd_buffers.lidar_head.offset,
            G.gd_buffers.agent_class.offset, G.gd_buffers.t.offset,
            G.gd_buffers.workspace_bytes.offset]
    assert vals == want


def _cfg(G, W=2, **kw):
    c = G.gd_config()
    c.num_worlds = W
    c.top_k = 8
    c.partners = 3
    c.episode_len = 91
    c.dt = 0.1
    c.obs_radius = 50.0
    c.goal_radius = 2.0
    c.v_max = 30.0
    c.lidar_range = 50.0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_host_side_sizes(G):
    ao = np.array([0, 4, 6], np.int32)
    ro = np.array([0, 100, 150], np.int32)
    assert G.gd_partner_slots(_cfg(G), ao) == 6 * 3
    assert G.gd_partner_slots(_cfg(G, partners=-1), ao) == 4 * 3 + 2 * 1
    ws = G.gd_workspace_size(_cfg(G), ao, ro)
    assert ws > 0 and ws % 256 == 0
    ws2 = G.gd_workspace_size(_cfg(G), ao, np.array([0, 200, 300], np.int32))
    assert ws2 > ws


@pytest.mark.parametrize("field,value,status", [
    ("num_worlds", 0, -1), ("top_k", -1, -2), ("top_k", 961, -2), ("partners", -2, -1),
    ("episode_len", 0, -1), ("dt", 0.0, -1), ("obs_radius", -1.0, -1), ("v_max", 0.0, -1),
    ("obs_waves", 3, -1), ("obs_bins", 100, -1), ("lidar_rays", 2000, -2), ("cell_size", -1.0, -1),
    ("obs_road", 3, -1), ("dynamics", 2, -1), ("dynamics", -1, -1), ("lidar_fov", -0.5, -1),
    ("lidar_fov", 1e-6, -1), ("lidar_fov", 7.0, -1), ("min_goal_dist", -1.0, -1),
])
def test_config_validation(G, field, value, status):
    ao = np.array([0, 4, 6], np.int32)
    ro = np.array([0, 100, 150], np.int32)
    c = _cfg(G, **{field: value})
    with pytest.raises(G.GDError) as e:
        G.gd_workspace_size(c, ao, ro)
    assert e.value.status == status
    assert G.gd_last_error() != ""


def test_offsets_validation(G):
    with pytest.raises(G.GDError) as e:
        G.gd_workspace_size(_cfg(G), np.array([0, 4, 3], np.int32), np.array([0, 10, 20], np.int32))
    assert e.value.status == G.GD_E_ARG
    with pytest.raises(G.GDError) as e:
        G.gd_workspace_size(_cfg(G), np.array([0, 2000, 2001], np.int32), np.array([0, 10, 20], np.int32))
    assert e.value.status == G.GD_E_SIZE and "agents" in G.gd_last_error()


def test_create_rejects_null_buffers_before_touching_the_device(G):
    ao = np.array([0, 4, 6], np.int32)
    ro = np.array([0, 100, 150], np.int32)
    b = G.gd_buffers()
    with pytest.raises(G.GDError) as e:
        G.gd_create(_cfg(G), ao, ro, b, 0)
    assert e.value.status == G.GD_E_ARG and "NULL" in G.gd_last_error()
    assert G.lib().gd_destroy(None) == 0


def test_null_handles(G):
    L = G.lib()
    assert L.gd_step(None, None, None) == G.GD_E_ARG
    assert L.gd_obs(None, None) == G.GD_E_ARG
    assert L.gd_reset(None, None, None) == G.GD_E_ARG
    assert L.gd_check(None, None) == G.GD_E_ARG
    assert L.gd_rollout_fwd(None, None, 1, 1, None, None, None, None, None) == G.GD_E_ARG
    assert L.gd_rollout_bwd(None, None, None, 1, 1, None, None, None, None, None, None) == G.GD_E_ARG
    assert L.gd_rollout_obs_features(None, None) == G.GD_E_ARG


def test_decimate_argument_checks(G):
    """Host-side validation of the decimation entry points (no device call is made)."""
    assert G.gd_decimate_workspace_size(0) == 0
    ws = G.gd_decimate_workspace_size(1000)
    assert ws >= 12 * 1000 and ws % 256 == 0
    with pytest.raises(G.GDError) as e:
        G.gd_decimate_workspace_size(-1)
    assert e.value.status == G.GD_E_ARG
    fake = 1 << 20  # never dereferenced: every call below fails before any device work
    cases = [((fake, -1, 10), 0.1, ws, G.GD_E_ARG), ((fake, 2, -5), 0.1, ws, G.GD_E_ARG),
             ((fake, 2, 1000), float("nan"), ws, G.GD_E_ARG), ((fake, 2, 1000), -1.0, ws, G.GD_E_ARG),
             ((fake, 2, 1000), 0.1, ws - 256, G.GD_E_SIZE), ((0, 2, 1000), 0.1, ws, G.GD_E_ARG)]
    for (po, npoly, npts), area, wsb, status in cases:
        with pytest.raises(G.GDError) as e:
            G.gd_decimate(po, npoly, npts, fake, fake, area, fake, fake, fake, wsb, 0)
        assert e.value.status == status, (npoly, npts, area, wsb)
    # nothing to do: returns at once
    G.gd_decimate(0, 0, 0, 0, 0, 0.1, 0, 0, 0, 0, 0)


def test_decimate_noalloc_argument_checks(G):
    """Host-side validation of the allocation-free decimation (no device call is made):
    sizes beyond its limit are refused before anything else."""
    fake = 1 << 20  # never dereferenced: every call below fails before any device work
    lim = G.GD_DECIMATE_NOALLOC_MAX_POINTS
    cases = [((fake, 2, lim + 1), 0.1, G.GD_E_SIZE), ((fake, -1, 10), 0.1, G.GD_E_ARG),
             ((fake, 2, -5), 0.1, G.GD_E_ARG), ((fake, 2, 1000), float("inf"), G.GD_E_ARG),
             ((fake, 2, 1000), -1.0, G.GD_E_ARG), ((0, 2, 1000), 0.1, G.GD_E_ARG)]
    for (po, npoly, npts), area, status in cases:
        with pytest.raises(G.GDError) as e:
            G.gd_decimate_noalloc(po, npoly, npts, fake, fake, area, fake, fake, 0)
        assert e.value.status == status, (npoly, npts, area)
        if status == G.GD_E_SIZE:
            assert "exceeds" in str(e.value)
    G.gd_decimate_noalloc(0, 0, 0, 0, 0, 0.1, 0, 0, 0)
