"""The allocation-free decimation (gd_decimate_noalloc, workspace in the library's static
device array) against gd_decimate with a caller workspace: keep masks and directions
identical bit for bit, on two calls in a row, the second with a smaller input.  Both
inputs hold polylines longer than the 4096 points staged in LDS, so the kernel works in
the static array."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _polylines(lens, seed):
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for n in lens:
        s = np.arange(n) * 0.1
        xs.append(s + rng.normal(0, 0.003, n))
        ys.append(0.5 * np.sin(s / 7.0) + rng.normal(0, 0.003, n))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return off, np.concatenate(xs).astype(np.float32), np.concatenate(ys).astype(np.float32)


def _both(G, off, x, y, min_area):
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(a, device=dev)
    po, tx, ty = t(off), t(x), t(y)
    n, npoly = int(x.size), int(off.size) - 1
    stream = torch.cuda.current_stream(dev).cuda_stream
    wsb = G.gd_decimate_workspace_size(n)
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=dev)
    keep_a = torch.full((n,), 7, dtype=torch.uint8, device=dev)
    dir_a = torch.full((n,), 9.0, dtype=torch.float32, device=dev)
    keep_b, dir_b = keep_a.clone(), dir_a.clone()
    G.gd_decimate(po.data_ptr(), npoly, n, tx.data_ptr(), ty.data_ptr(), min_area, keep_a.data_ptr(),
                  dir_a.data_ptr(), ws.data_ptr(), wsb, stream)
    G.gd_decimate_noalloc(po.data_ptr(), npoly, n, tx.data_ptr(), ty.data_ptr(), min_area,
                          keep_b.data_ptr(), dir_b.data_ptr(), stream)
    torch.cuda.synchronize()
    return keep_a.cpu().numpy(), dir_a.cpu().numpy(), keep_b.cpu().numpy(), dir_b.cpu().numpy()


def test_noalloc_decimation_matches_workspace_variant(gpu):
    from paper_2408_01584_amd import gd as G
    calls = [([9000, 5, 0, 4097, 1, 2, 300, 12000, 64], 11, 0.001),   # 25 469 points
             ([4500, 3, 7000, 0, 65], 12, 0.01)]                       # smaller, second call
    sizes = []
    for lens, seed, min_area in calls:
        off, x, y = _polylines(lens, seed)
        sys_msg = "noalloc decimation: %d polylines, %d points, min_area %g" % (len(lens), x.size, min_area)
        print(sys_msg, flush=True)
        ka, da, kb, db = _both(G, off, x, y, min_area)
        assert np.array_equal(ka, kb), "keep differs at %s" % np.flatnonzero(ka != kb)[:5]
        assert np.array_equal(da.view(np.uint32), db.view(np.uint32)), "dir differs"
        assert set(np.unique(ka)) <= {0, 1} and 0 < int(ka.sum()) < x.size
        sizes.append(x.size)
    assert sizes[1] < sizes[0]


def test_noalloc_decimation_rejects_oversize(gpu):
    from paper_2408_01584_amd import gd as G
    with pytest.raises(G.GDError) as e:
        G.gd_decimate_noalloc(1 << 20, 1, G.GD_DECIMATE_NOALLOC_MAX_POINTS + 1, 1 << 20, 1 << 20, 0.1,
                              1 << 20, 1 << 20, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == G.GD_E_SIZE
