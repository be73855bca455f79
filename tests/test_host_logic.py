"""Host-side logic of the systems layers, on the CPU: the serving loop's
latency percentiles and HBM budget, and the tuner's workload classes, cache
and candidate knobs (every candidate must name knobs that DecomposeJob
takes, so that a tuned job runs)."""
import inspect
import json

import pytest

import paper_1506_03265_amd as cd
from paper_1506_03265_amd import serve, tune


def test_percentile_nearest_rank():
    xs = [5.0, 1.0, 4.0, 2.0, 3.0]
    assert serve.percentile(xs, 0) == 1.0
    assert serve.percentile(xs, 50) == 3.0
    assert serve.percentile(xs, 100) == 5.0
    assert serve.percentile(list(range(101)), 99) == 99
    assert serve.percentile([], 50) == 0.0


def test_budget_admits_within_total_and_always_one_request():
    b = serve._Budget(100)
    assert b.fits(1000)              # alone, even a request larger than the budget runs
    b.take(60)
    assert b.fits(40) and not b.fits(41)
    b.take(40)
    assert not b.fits(1)
    b.give(60)
    assert b.used == 40 and b.fits(60) and not b.fits(61)
    b.give(40)
    assert b.used == 0 and b.fits(10 ** 12)


class _G:
    def __init__(self, n, m):
        self.n, self.m = n, m


def test_workload_class_buckets_by_powers_of_two():
    assert tune.workload_class([_G(1000, 8000)]) == "g1-n2^9-m2^12"
    assert tune.workload_class([_G(1000, 8000), _G(24, 100)]) == "g2-n2^10-m2^12"   # 1024 nodes, 8100 arcs
    assert tune.workload_class([_G(1, 0)]) == "g1-n2^0-m2^0"


def test_tune_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "cache.json"
    monkeypatch.setenv("CLDIAM_TUNE_CACHE", str(path))
    assert tune._load() == {}
    tune._save({"g1-n2^9-m2^12": {"driver": 1, "local_rounds": 8}})
    assert json.loads(path.read_text()) == {"g1-n2^9-m2^12": {"driver": 1, "local_rounds": 8}}
    assert tune._load()["g1-n2^9-m2^12"]["local_rounds"] == 8
    path.write_text("not json")
    assert tune._load() == {}


def test_candidates_name_decompose_job_knobs():
    knobs = set(inspect.signature(cd.DecomposeJob.__init__).parameters) - {"self", "graphs", "params"}
    assert len(tune.CANDIDATES) >= 20
    for c in tune.CANDIDATES:
        assert set(c) <= knobs, c
    modes = {c.get("pull_mode") for c in tune.CANDIDATES}
    assert {cd.PULL_NEVER, cd.PULL_ALWAYS} <= modes
    # no two candidates are the same schedule
    assert len({json.dumps(c, sort_keys=True) for c in tune.CANDIDATES}) == len(tune.CANDIDATES)
