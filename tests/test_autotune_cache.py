"""The autotuner's cache (CPU only): keys separate what the library's work
plan separates, and entries survive a write and a reload."""
import json

from paper_1412_8754_amd import autotune


def test_key_separates_shapes(monkeypatch, tmp_path):
    pts = [(0.1, 0.002, 64, 64), (0.2, 0.03, 64, 64), (0.0, 0.001, 32, 16)]
    k = autotune.shape_key(pts, 128, 16, 3, 0, "gfx950")
    assert k == autotune.shape_key(list(reversed(pts)), 128, 16, 3, 0, "gfx950")
    assert k != autotune.shape_key(pts, 128, 16, 3, 1, "gfx950")
    assert k != autotune.shape_key(pts, 64, 16, 3, 0, "gfx950")
    assert k != autotune.shape_key(pts[:2], 128, 16, 3, 0, "gfx950")
    # the temperature class picks the sweep kernel
    hot = [(0.1, 0.006, 64, 64)] + pts[1:]
    assert k != autotune.shape_key(hot, 128, 16, 3, 0, "gfx950")
    assert k != autotune.shape_key(pts, 128, 16, 3, 0, "gfx942")


def test_cache_round_trip(monkeypatch, tmp_path):
    f = tmp_path / "tune.json"
    monkeypatch.setenv("OMEGA_TUNE_CACHE", str(f))
    pts = [(0.1, 0.002, 256, 256)]
    assert autotune.lookup(pts, 64, 8, 3, 0, arch="gfx950") is None
    key = autotune.shape_key(pts, 64, 8, 3, 0, "gfx950")
    autotune.save_entry(key, {"sweep_blocks_per_cu": 2, "sweep_queues": 16, "ms": 1.0})
    assert autotune.lookup(pts, 64, 8, 3, 0, arch="gfx950") == {
        "sweep_blocks_per_cu": 2, "sweep_queues": 16}
    assert json.load(open(f))[key]["ms"] == 1.0
