"""Autotuner bookkeeping that needs no GPU: size buckets and the JSON cache."""
import json

from paper_2302_14812_amd import autotune


def test_keys_bucket_by_powers_of_two():
    assert autotune.single_key(10000, 4096, 16384, "mixed") == "single/mixed/p13/s12/c14"
    assert autotune.single_key(9000, 4000, 16000, "mixed") == autotune.single_key(
        10000, 4096, 16384, "mixed")
    assert autotune.batch_key(64, 4.5e13, 1e4) != autotune.batch_key(8, 4.5e13, 1e4)


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = str(tmp_path / "sub" / "tune.json")
    monkeypatch.setenv("RADIO_TUNE_CACHE", path)
    assert autotune.cache_path() == path
    assert autotune.load_cache() == {}
    cache = {"single/mixed/p13/s12/c14": {"target_blocks": 3072, "ms": 5000.0}}
    autotune.save_cache(cache)
    assert autotune.load_cache() == cache
    with open(path, "w") as f:
        f.write("{not json")
    assert autotune.load_cache() == {}
