"""CPU checks of the autotuner's cache bookkeeping (no device work)."""
import json

from paper_2607_17978_amd import autotune


def test_tile_key_buckets_atom_counts():
    assert autotune.tile_key((192, 192, 192), 6, 32768) == "tiles/192x192x192/p6/n2^15"
    assert autotune.tile_key((192, 192, 192), 6, 30000) == autotune.tile_key((192, 192, 192), 6, 32768)
    assert autotune.tile_key((320, 320, 320), 8, 131072) == "tiles/320x320x320/p8/n2^17"


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "autotune.json"
    monkeypatch.setenv("QEQ_AUTOTUNE_CACHE", str(path))
    assert autotune.cache_path() == str(path)
    assert autotune.cached_tiles((96, 96, 96), 6, 4096) is None
    autotune._store_cache(str(path), autotune.tile_key((96, 96, 96), 6, 4096), {"tiles": [16, 8, 4], "ms": 1.0})
    autotune._store_cache(str(path), autotune.tile_key((48, 48, 48), 6, 512), {"tiles": [0, 0, 0], "ms": 0.5})
    assert autotune.cached_tiles((96, 96, 96), 6, 4096) == (16, 8, 4)
    assert autotune.cached_tiles((48, 48, 48), 6, 512) == (0, 0, 0)
    d = json.loads(path.read_text())
    assert len(d) == 2
    # a damaged file reads as empty instead of failing the solve set-up
    path.write_text("{not json")
    assert autotune.cached_tiles((96, 96, 96), 6, 4096) is None
