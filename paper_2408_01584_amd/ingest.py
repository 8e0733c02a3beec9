"""Ingest-time road decimation (Sec. 3.1): thin a scene's road polylines with the
library's Visvalingam-Whyatt kernel (``gd_decimate``) and return a scene holding the kept
points.  The kernel decides which points survive and computes their new directions; this
module only moves arrays (upload, gather of the kept points, new CSR offsets)."""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import gd as G


def polyline_offsets(road_meta: np.ndarray) -> np.ndarray:
    """CSR offsets of the polylines: a polyline ends at each point marked GD_META_LAST."""
    last = np.flatnonzero(np.asarray(road_meta) & G.GD_META_LAST)
    return np.concatenate([[0], last + 1]).astype(np.int32)


def decimate_road(x: torch.Tensor, y: torch.Tensor, poly_off: torch.Tensor, min_area: float):
    """keep [n] uint8 and dir [n] float32 for device points x, y (float32) and device
    polyline offsets poly_off (int32), on the current stream."""
    n = int(x.numel())
    assert x.dtype == y.dtype == torch.float32 and poly_off.dtype == torch.int32
    assert x.is_contiguous() and y.is_contiguous() and poly_off.is_contiguous() and y.numel() == n
    keep = torch.empty(n, dtype=torch.uint8, device=x.device)
    dirs = torch.empty(n, dtype=torch.float32, device=x.device)
    wsb = G.gd_decimate_workspace_size(n)
    ws = torch.empty(wsb + 256, dtype=torch.uint8, device=x.device)
    wptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    G.gd_decimate(poly_off.data_ptr(), int(poly_off.numel()) - 1, n, x.data_ptr(), y.data_ptr(),
                  float(min_area), keep.data_ptr(), dirs.data_ptr(), wptr, wsb,
                  torch.cuda.current_stream().cuda_stream)
    return keep, dirs


def decimate_scene(scene, min_area: float, device="cuda"):
    """A copy of ``scene`` whose road keeps only the points that survive decimation with
    threshold ``min_area`` (m^2), their directions recomputed by the kernel.  Returns
    (scene, keep mask as a numpy bool array)."""
    po = polyline_offsets(scene.road_meta)
    ro = np.asarray(scene.road_off)
    if not np.isin(ro[1:][np.diff(ro) > 0], po).all():
        raise ValueError("every world's road must end with a GD_META_LAST point")
    dev = torch.device(device)
    x = torch.as_tensor(np.ascontiguousarray(scene.road_x, np.float32), device=dev)
    y = torch.as_tensor(np.ascontiguousarray(scene.road_y, np.float32), device=dev)
    keep, dirs = decimate_road(x, y, torch.as_tensor(po, device=dev), min_area)
    k = keep.cpu().numpy().astype(bool)
    d = dirs.cpu().numpy()
    ck = np.concatenate([[0], np.cumsum(k, dtype=np.int64)])
    road_off = ck[ro].astype(np.int32)
    out = dataclasses.replace(scene, road_off=road_off, road_x=np.ascontiguousarray(scene.road_x[k]),
                              road_y=np.ascontiguousarray(scene.road_y[k]),
                              road_dir=np.ascontiguousarray(d[k]),
                              road_meta=np.ascontiguousarray(scene.road_meta[k]),
                              extra=dict(scene.extra))
    return out, k
