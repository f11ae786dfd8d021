"""Host logic of the autotuner's cache (no GPU): the serving tuner keeps the fastest configuration and
records every tuning axis, and the cached lookups give back what was recorded."""
import json

from paper_1305_4376_amd import autotune


def test_serving_tuner_records_every_axis(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "_device_key", lambda kernel, blocks: f"gfx950/256/{kernel}/2^{blocks.bit_length() - 1}")
    path = str(tmp_path / "tuning.json")
    speeds = {None: 700.0, (128, 12, 2048, 2): 650.0, (256, 4, 1800, 2): 720.0}
    res = autotune.tune_serving(lambda sh: speeds[sh], list(speeds), 1 << 24, path=path)
    assert res["shape"] == (256, 4, 1800, 2)
    entry = json.load(open(path))["gfx950/256/serve/2^24"]
    assert set(entry) == set(autotune.FIELDS) | {"gbs"}
    assert autotune.cached_serving(1 << 24, path) == (256, 4, 1800, 2)
    speeds[None] = 900.0
    autotune.tune_serving(lambda sh: speeds[sh], list(speeds), 1 << 24, path=path)
    assert autotune.cached_serving(1 << 24, path) is None   # the default won
    assert autotune.cached_serving(1 << 20, path) is None   # nothing recorded for that step size


def test_batch_cache_lookup(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "_device_key", lambda kernel, blocks: f"gfx950/256/{kernel}/2^{blocks.bit_length() - 1}")
    path = str(tmp_path / "tuning.json")
    autotune.save_cache({"gfx950/256/batch/2^25": {"threads": 128, "groups_per_cu": 12, "wave_remainder": 2048,
                                                    "tiles_per_draw": 2, "seconds": 0.0004}}, path)
    assert autotune.cached_tuning(45_000_000, path=path) == (128, 12, 2048, 2)
    assert autotune.cached_tuning(1000, path=path) is None
