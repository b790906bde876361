"""Host-side logic of the autotuner (no GPU)."""
from paper_1608_01362_amd import autotune, cagra


def test_candidates_cover_every_memory_level():
    c = autotune.candidate_segment_sizes(1 << 25, cagra.F32)
    assert 32768 in c and (1 << 20) in c and (1 << 24) in c and (1 << 25) in c
    assert max(x for x in c if x <= 32768) == cagra.STAGE_BYTES // 4
    cb = autotune.candidate_segment_sizes(1 << 25, cagra.BF16)
    assert 65536 in cb
    small = autotune.candidate_segment_sizes(1000, cagra.F32)
    assert max(small) == 1000 and all(x <= 32768 for x in small)


def test_merge_capacity_rule_matches_header():
    assert autotune.fused_merge_fits(16384, 4055)
    assert not autotune.fused_merge_fits(16384, 4096)
    assert autotune.fused_merge_fits(8192, 1024)


def test_byte_model_monotone_in_q():
    a = autotune.byte_model(1 << 20, 1 << 24, 1 << 22, 32, 8192, 4)
    b = autotune.byte_model(1 << 20, 1 << 24, 1 << 23, 32, 8192, 4)
    assert b - a == 10 * (1 << 22)


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "c.json")
    autotune.save_cache(p, {"k": {"N": 1, "B": 2, "tile_edges": 64, "staged": True}})
    assert autotune.load_cache(p)["k"]["B"] == 2
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}
