"""Host logic of the autotuner's per-architecture cache (no GPU)."""
import json

from paper_2403_17261_amd import scenes, tuning


def test_signature_names_the_world_shape():
    sc = scenes.config1(0)
    sig = tuning.signature(sc)
    assert sig == "scenes=1 partitions=2 bodies~64 capsules=0 joints=no"
    big = scenes.config5(0)
    assert "bodies~100000" in tuning.signature(big) and "partitions=64" in tuning.signature(big)


def test_cache_file_per_architecture(tmp_path):
    assert tuning.load("gfx950", str(tmp_path)) == {}
    path = tuning.cache_path("gfx950", str(tmp_path))
    assert path.endswith("autotune_gfx950.json")
    entry = {"scenes=1 partitions=2 bodies~64 capsules=0 joints=no": {"pgs_block": 512, "pgs_lds_reps": 2400,
                                                                       "persistent": 1}}
    with open(path, "w") as f:
        json.dump(entry, f)
    assert tuning.load("gfx950", str(tmp_path)) == entry
    assert tuning.load("gfx942", str(tmp_path)) == {}
