"""Autotuner cache and key bucketing (host only)."""
import json

from paper_2401_01607_amd import autotune as A


def test_pow2_buckets():
    assert [A._pow2(v) for v in (1, 2, 3, 4, 5, 1024, 1025, 65536)] == [1, 2, 4, 4, 8, 1024, 2048, 65536]


def test_cache_round_trip_and_memory_only(tmp_path):
    p = tmp_path / "sub" / "tune.json"
    c = A.TuneCache(str(p))
    assert c.get("k") is None
    c.put("k", {"tile": [16, 4], "ms": {"16,4": 0.7}})
    assert json.loads(p.read_text())["k"]["tile"] == [16, 4]
    assert A.TuneCache(str(p)).get("k") == {"tile": [16, 4], "ms": {"16,4": 0.7}}
    m = A.TuneCache(None)
    m.put("k", 1)
    assert m.get("k") == 1


def test_cache_ignores_a_corrupt_file(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    assert A.TuneCache(str(p)).get("k") is None


def test_candidates_are_the_library_tiles():
    assert set(r for r, _ in A.STREAM_CANDIDATES) == {4, 8, 12, 14, 16}
    assert set(w for _, w in A.STREAM_CANDIDATES) == {1, 2, 4}
    assert set(A.POOL_CANDIDATES) == {4, 8, 12, 16}
