"""Host logic of the autotuner: candidate selection, de-duplication, size
buckets and the JSON cache (no device work)."""
import math

from paper_1604_04815_amd.autotune import Cache, Candidate, Entry, cache_key, distinct_by_grid, pick_best, size_bucket


def test_pick_best_prefers_fastest_then_smaller_grid():
    cands = [Candidate(256, 8, 5, 1280, 0.41), Candidate(512, 8, 2, 512, 0.41), Candidate(1024, 4, 1, 256, 0.50),
             Candidate(256, 2, 8, 2048, float("inf"))]
    b = pick_best(cands)
    assert (b.block_threads, b.grid) == (512, 512)
    assert pick_best([Candidate(256, 8, 1, 256, 0.3), Candidate(256, 4, 1, 256, 0.2)]).vectors_per_lane == 4


def test_pick_best_rejects_nothing_run():
    try:
        pick_best([Candidate(256, 8, 1, 256)])
    except ValueError:
        return
    raise AssertionError("expected ValueError")


def test_distinct_by_grid():
    c = [Candidate(256, 8, 5, 1280), Candidate(256, 8, 6, 1280), Candidate(256, 8, 4, 1024)]
    assert [x.groups_per_cu for x in distinct_by_grid(c)] == [5, 4]


def test_size_bucket():
    assert size_bucket(1) == 0 and size_bucket(2 ** 20) == 20 and size_bucket(2 ** 20 + 5) == 20
    assert size_bucket(0) == 0


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    c = Cache(path)
    e = Entry("MI355X", "int32", "add", False, "plain", 28, 256, 8, 5, 0.40, 5300.0, tried=30)
    c.put(e)
    c.save()
    d = Cache(path)
    got = d.get("MI355X", "int32", "add", False, "plain", 2 ** 28 + 17)
    assert got is not None and (got.block_threads, got.vectors_per_lane, got.groups_per_cu) == (256, 8, 5)
    assert d.get("MI355X", "int32", "add", True, "plain", 2 ** 28) is None
    assert e.key() == cache_key("MI355X", "int32", "add", False, "plain", 28)
    assert math.isclose(got.gbs, 5300.0)
