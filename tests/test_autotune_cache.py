"""Host logic of the autotuner's cache (no GPU needed)."""
import numpy as np

from paper_1705_07497_amd import autotune


def test_cache_key_distinguishes_geometry_and_mask():
    m1 = np.ones(10, np.uint8)
    m2 = m1.copy()
    m2[3] = 0
    keys = {autotune.cache_key("gfx950", 64, 10, 91, m, k) for m in (m1, m2) for k in (0, 2)}
    keys.add(autotune.cache_key("gfx950", 65, 10, 91, m1, 0))
    keys.add(autotune.cache_key("gfx942", 64, 10, 91, m1, 0))
    assert len(keys) == 6


def test_cache_store_and_load_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    e1 = {"tuning": dict(autotune.DEFAULT, fwd_waves=2), "batch": 4, "timings_s": {}}
    autotune.store("k1", e1, path)
    autotune.store("k2", {"tuning": autotune.DEFAULT, "batch": 1, "timings_s": {}}, path)
    data = autotune.load_cache(path)
    assert data["k1"] == e1 and set(data) == {"k1", "k2"}
    (tmp_path / "bad.json").write_text("not json")
    assert autotune.load_cache(str(tmp_path / "bad.json")) == {}
