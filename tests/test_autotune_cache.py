"""Autotuner bookkeeping that needs no GPU: size buckets and the JSON cache."""
import json

from paper_2302_14812_amd import autotune


def test_keys_bucket_by_powers_of_two():
    assert autotune.single_key(10000, 4096, 16384, "mixed") == "single/mixed/p13/s7/c14"
    assert autotune.single_key(9000, 4000, 16000, "mixed") == autotune.single_key(
        10000, 4096, 16384, "mixed")
    assert autotune.batch_key(64, 4.5e13, 1e4) != autotune.batch_key(8, 4.5e13, 1e4)
    # long chunks share one step bucket
    assert autotune.single_key(200000, 200, 65536, "mixed") == autotune.single_key(
        200000, 1000, 65536, "mixed")
    assert autotune.single_key(200000, 16, 65536, "mixed") != autotune.single_key(
        200000, 1000, 65536, "mixed")


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = str(tmp_path / "sub" / "tune.json")
    monkeypatch.setenv("RADIO_TUNE_CACHE", path)
    assert autotune.cache_path() == path
    assert autotune.load_cache(shipped=False) == {}
    cache = {"single/mixed/p13/s7/c14": {"target_blocks": 3072, "shape": 0, "ms": 5000.0}}
    autotune.save_cache(cache)
    assert autotune.load_cache(shipped=False) == cache
    # the user's entries win over the shipped ones
    merged = autotune.load_cache()
    assert merged["single/mixed/p13/s7/c14"] == cache["single/mixed/p13/s7/c14"]
    with open(path, "w") as f:
        f.write("{not json")
    assert autotune.load_cache(shipped=False) == {}


def test_shipped_cache_entries():
    """The shipped cache, where present, holds a shape and a launch split per entry."""
    import paper_2302_14812_amd as radio
    shipped = autotune.load_cache(path="/nonexistent/none.json")
    for key, rec in shipped.items():
        assert key.startswith(("single/", "batch/", "runtime/"))
        assert rec["shape"] in radio.SHAPES
        assert ("target_blocks" in rec) if key.startswith("single/") else (
            "items_per_workgroup" in rec)


def test_runtime_keys():
    """Run-time blocks have their own bucket: a one-pair batch of a 16-step block
    is not the 64-set batch, nor a single deposit of the whole run."""
    k = autotune.runtime_key(10000, 16, 16384, "mixed")
    assert k == "runtime/mixed/p13/s4/c14"
    assert k != autotune.single_key(10000, 16, 16384, "mixed")
    assert autotune.runtime_key(10000, 16, 16384, "fp64") != k
