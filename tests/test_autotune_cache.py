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


def test_bin_weights_fallback(tmp_path):
    import numpy as np
    from paper_2609_03613_amd import bins
    assert bins.load_weights(str(tmp_path / "missing.npz")) is None
    p = str(tmp_path / "w.npz")
    bins.save_weights(p, np.zeros(10))
    assert bins.load_weights(p) is None  # wrong size
    w = bins.init_weights()
    w[3] = np.inf
    bins.save_weights(p, w)
    assert bins.load_weights(p) is None  # not finite
    w = bins.init_weights()
    bins.save_weights(p, w, note="x")
    assert np.array_equal(bins.load_weights(p), w)
    (tmp_path / "bad.npz").write_bytes(b"not a zip")
    assert bins.load_weights(str(tmp_path / "bad.npz")) is None


def test_committed_bin_weights_are_valid():
    import numpy as np
    from paper_2609_03613_amd import bins
    w = bins.load_weights()
    assert w is not None and w.shape == (5768,) and np.all(np.isfinite(w))
    with np.load(bins.WEIGHTS_PATH, allow_pickle=False) as z:
        assert float(z["c_seg"]) >= 0 and np.all(np.asarray(z["c_bucket"]) >= 0)
