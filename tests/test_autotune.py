"""Autotune table keys: workload class (scene size bucket, texture resolution,
texel type, camera set, direction) and the nearest-size fallback."""
from paper_2608_17682_amd import autotune


def test_key_is_the_workload_class():
    k = autotune.workload_key(100_000, 8, 0, [0, 0], "fwd")
    assert k == "n131072|r8|f32|pinhole|fwd"
    k5 = autotune.workload_key(4_000_000, 8, 1, [3, 0, 2, 1, 0], "bwd")
    assert k5 == "n4194304|r8|f16|fisheye+pinhole+rolling_shutter+thin_lens|bwd"
    assert autotune.size_bucket(1) == 1 and autotune.size_bucket(1025) == 2048


def test_lookup_exact_then_nearest_size_then_none():
    t = {"n131072|r8|f32|pinhole|fwd": {"lanes_per_ray": 1, "tile_w": 8, "tile_h": 8,
                                        "block": 128, "schedule": 1, "ms": 1.0},
         "n2097152|r8|f32|pinhole|fwd": {"lanes_per_ray": 2, "tile_w": 8, "tile_h": 4,
                                         "block": 256, "schedule": 2, "ms": 1.0}}
    e = autotune.lookup_key("n131072|r8|f32|pinhole|fwd", t)
    assert e == {"lanes_per_ray": 1, "tile_w": 8, "tile_h": 8, "block": 128, "schedule": 1}
    # 1M sites: nearest tuned size is 2M (log scale)
    assert autotune.lookup_key("n1048576|r8|f32|pinhole|fwd", t)["lanes_per_ray"] == 2
    assert autotune.lookup_key("n262144|r8|f32|pinhole|fwd", t)["lanes_per_ray"] == 1
    # other texel type, camera set or direction: no entry
    assert autotune.lookup_key("n131072|r8|f16|pinhole|fwd", t) is None
    assert autotune.lookup_key("n131072|r8|f32|fisheye|fwd", t) is None
    assert autotune.lookup_key("n131072|r8|f32|pinhole|bwd", t) is None


def test_committed_table_entries_are_valid_launches():
    t = autotune._load()
    assert t
    for k, e in t.items():
        assert k.count("|") == 4 and k.split("|")[-1] in ("fwd", "bwd")
        assert e["tile_w"] * e["tile_h"] * e["lanes_per_ray"] == 64
        assert e["block"] in (64, 128, 256) and e["schedule"] in (1, 2, 3)
