"""Helpers shared by the tests: hand-built one-world scenes."""
import numpy as np


def tiny_world(agents, edges=(), lanes=(), goals=None, speeds=None, params=None, extra_road=None):
    """One world from boxes (x, y, yaw, L, W) and edge / lane polylines [(x, y), ...]."""
    from paper_2408_01584_amd import scenes as S

    pts, metas, dirs = [], [], []
    for typ, poly in [(S.EDGE, s) for s in edges] + [(S.LANE, s) for s in lanes]:
        poly = [tuple(p) for p in poly]
        for k, p in enumerate(poly):
            pts.append(p)
            metas.append(typ | (S.META_LAST if k == len(poly) - 1 else 0))
            q = poly[k + 1] if k + 1 < len(poly) else None
            r = poly[k - 1] if k > 0 else None
            if q is not None:
                dirs.append(np.arctan2(q[1] - p[1], q[0] - p[0]))
            elif r is not None:
                dirs.append(np.arctan2(p[1] - r[1], p[0] - r[0]))
            else:
                dirs.append(0.0)
    if extra_road is not None:
        for (x, y, d, m) in extra_road:
            pts.append((x, y)); dirs.append(d); metas.append(m)
    pts = np.array(pts, dtype=np.float64).reshape(-1, 2)
    n = len(agents)
    goals = goals if goals is not None else [(1e3, 1e3)] * n
    speeds = speeds if speeds is not None else [0.0] * n
    part = dict(x=[a[0] for a in agents], y=[a[1] for a in agents], yaw=[a[2] for a in agents],
                speed=list(speeds), length=[a[3] for a in agents], width=[a[4] for a in agents],
                goal_x=[g[0] for g in goals], goal_y=[g[1] for g in goals], road_x=pts[:, 0],
                road_y=pts[:, 1], road_dir=np.array(dirs), road_meta=np.array(metas, np.int32))
    params = params if params is not None else S.SimParams(top_k=8, partners=max(n - 1, 0))
    return S.assemble(0, [part], params)


def wrap(a):
    return (np.asarray(a) + np.pi) % (2 * np.pi) - np.pi


def key32(px, py, qx, qy):
    """binary32 squared distance with the fixed operation order (numpy float32 arithmetic
    is IEEE single precision without contraction)."""
    px, py = np.float32(px), np.float32(py)
    dx = (np.asarray(qx, np.float32) - px).astype(np.float32)
    dy = (np.asarray(qy, np.float32) - py).astype(np.float32)
    return (dx * dx).astype(np.float32) + (dy * dy).astype(np.float32)


def key64(px, py, qx, qy):
    """FP64 squared distance (the definition the oracle's decisions use by default)."""
    dx = np.asarray(qx, np.float64) - np.float64(px)
    dy = np.asarray(qy, np.float64) - np.float64(py)
    return dx * dx + dy * dy
