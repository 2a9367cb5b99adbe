"""Host logic of the autotuner's cache file (no GPU needed)."""
import numpy as np

from paper_1705_07497_amd import autotune


def test_geometry_key_distinguishes_geometry_mask_kind_and_arch():
    m1 = np.ones(10, np.uint8)
    m2 = m1.copy()
    m2[3] = 0
    keys = {autotune.geometry_key("gfx950", 64, 10, 91, m, k) for m in (m1, m2) for k in (0, 2)}
    keys.add(autotune.geometry_key("gfx950", 65, 10, 91, m1, 0))
    keys.add(autotune.geometry_key("gfx942", 64, 10, 91, m1, 0))
    keys.add(autotune.geometry_key("gfx950", 64, 10, 91, m1, 0, compact=True))
    assert len(keys) == 7
    assert autotune.geometry_key("gfx950", 64, 10, 91, m1, 0) == \
        autotune.geometry_key("gfx950", 64, 10, 91, m1, 0, compact=False)


def test_bundle_cache_roundtrip_last_line_wins_and_foreign_lines_ignored(tmp_path):
    path = str(tmp_path / "sub" / "tune.txt")
    assert autotune.load_bundles(path) == {}
    autotune.store_bundle("k1", 32, path=path)
    autotune.store_bundle("k2", 16, path=path)
    autotune.store_bundle("k1", 64, 4, path=path)
    autotune.store_bundle("k4", 32, 2, path=path)
    with open(path, "a") as fh:   # the library's launch lines and junk share the file
        fh.write("sparsect-tune gfx950|n64|a10|b91|m0|k0|bw16|B1 2 1 4 8\n")
        fh.write("sparsect-bundle k3 48\n")      # not a valid width
        fh.write("sparsect-bundle k5 16 2\n")    # 8 bins per angle: not a layout
        fh.write("sparsect-bundle k6 32\n")      # a line without the angle count: one angle
        fh.write("garbage\n")
    assert autotune.load_bundles(path) == {"k1": (64, 4), "k2": (16, 1), "k4": (32, 2), "k6": (32, 1)}
