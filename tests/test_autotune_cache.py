"""Host-side behaviour of the autotuner's cache (no GPU needed)."""
import json

from paper_2609_03613_amd import autotune


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "c.json")
    assert autotune.load_cache(path) == {}
    autotune.save_cache(path, {"k": {"tile_size": 16, "num_bins": 64}})
    assert autotune.load_cache(path) == {"k": {"tile_size": 16, "num_bins": 64}}


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "c.json"
    path.write_text("{not json")
    assert autotune.load_cache(str(path)) == {}
    path.write_text(json.dumps([1, 2, 3]))
    assert autotune.load_cache(str(path)) == {}


def test_candidates_cover_tile_sizes_and_bins():
    assert set(ts for ts, _ in autotune.CANDIDATES) == {8, 16, 32}
    assert all(k & (k - 1) == 0 for _, k in autotune.CANDIDATES)
