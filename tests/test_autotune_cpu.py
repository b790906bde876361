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


def test_pool_keeps_staged_candidates_when_cache_gathers_move_fewer_bytes():
    """A one-segment pull moves fewer HBM bytes than LDS-sized segments but pays
    for its random reads in requests; the pool must still time staged sizes."""
    C = autotune.Choice
    cands = [C(1 << 25, 8192, 262144, False, 17_000_000, 5_030_000_000),
             C(1 << 24, 8192, 262144, False, 28_000_000, 5_140_000_000),
             C(32768, 8192, 262144, True, 575_000_000, 8_540_000_000),
             C(32768, 4096, 262144, True, 575_000_000, 8_560_000_000),
             C(8192, 8192, 262144, True, 900_000_000, 14_000_000_000)]
    pool = autotune.select_pool(cands, 1.6, 4)
    assert [c.staged for c in pool] == [True, True, False]
    assert pool[0].N == 32768 and pool[-1].N == 1 << 25
    assert all(c.N != 8192 for c in pool)  # 1.64x the best staged bytes: pruned
    only_unstaged = autotune.select_pool(cands[:2], 1.6, 4)
    assert [c.N for c in only_unstaged] == [1 << 25, 1 << 24]


def test_batched_and_multi_candidates():
    c = autotune.ppr_candidates(1 << 22)
    assert {n for n, _, _ in c} == {1 << 16, 1 << 18, 1 << 20, 1 << 21, 1 << 22}
    assert all(b <= 512 for _, b, _ in c)  # the batched merge keeps B x 64 floats in LDS
    assert autotune.size_class(1 << 13) == 0 and autotune.size_class(1 << 14) == 1
    assert autotune.size_class(1 << 17) == 1 and autotune.size_class(1 << 18) == 2
    assert all(n <= cagra.EDGE16_MAX_N for n, _, _ in autotune.multi_candidates())
