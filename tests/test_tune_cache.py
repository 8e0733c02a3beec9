"""Host logic of the tuned-shape cache (no device): the key is the workload signature and
the device's architecture and compute-unit count; a graph-mode simulator without a record
of its own takes the direct-launch shape."""
import dataclasses
import json

from paper_2408_01584_amd import scenes as S
from paper_2408_01584_amd import tune


def test_cached_shape_lookup(tmp_path, monkeypatch):
    sc = S.make_scene(0)
    dev = "gfx950:sramecc+:xnack-:256"
    shape = {"obs_waves": 8, "obs_bins": 256, "obs_cands": 512, "cell_size": 15.0, "obs_road": 1}
    cache = tmp_path / "shapes.json"
    cache.write_text(json.dumps({tune.signature(sc, sc.params, False) + "@" + dev:
                                 {"shape": shape, "ms_per_step": 0.01, "candidates": 1}}))
    monkeypatch.setattr(tune, "CACHE", str(cache))
    monkeypatch.setattr(tune, "_device_name", lambda: dev)
    assert tune.cached_shape(sc) == shape
    assert tune.cached_shape(sc, graph=True) == shape  # no graph record: the direct shape
    # another device, or another workload, has no record
    monkeypatch.setattr(tune, "_device_name", lambda: "gfx942:304")
    assert tune.cached_shape(sc) is None
    monkeypatch.setattr(tune, "_device_name", lambda: dev)
    assert tune.cached_shape(sc, dataclasses.replace(sc.params, top_k=sc.params.top_k + 1)) is None


def test_signature_separates_graph_mode():
    sc = S.make_scene(0)
    assert tune.signature(sc, sc.params, False) != tune.signature(sc, sc.params, True)
