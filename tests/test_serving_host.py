"""Host logic of the serving loop (no GPU): batch formation, fairness and
ordering, HBM-budget admission and LRU eviction, latency statistics."""

import pytest
import torch

from paper_1803_04128_amd.serving import (AdmissionError, PinnedError,
                                          PlanCache, Request,
                                          Scheduler, summarize)
from synthetic import serving_requests, SERVING_SHAPES


def _req(rid, plan, nvec, t=0.0):
    return Request(rid, plan, torch.zeros(nvec, 4), t)


def test_batches_take_the_oldest_plan_in_order_up_to_capacity():
    s = Scheduler(max_batch=8)
    for rid, (plan, nv) in enumerate([("a", 3), ("b", 2), ("a", 4), ("a", 2),
                                      ("b", 8), ("a", 1)]):
        s.add(_req(rid, plan, nv, t=rid))
    name, b = s.next_batch()
    # a: 3 + 4 fit, 2 does not: the batch ends there (order kept)
    assert name == "a" and [r.rid for r in b] == [0, 2]
    name, b = s.next_batch()
    assert name == "b" and [r.rid for r in b] == [1]
    name, b = s.next_batch()
    assert name == "a" and [r.rid for r in b] == [3, 5]
    name, b = s.next_batch()
    assert name == "b" and [r.rid for r in b] == [4]
    assert s.next_batch() is None


def test_every_request_is_batched_once_and_per_plan_order_holds():
    s = Scheduler(max_batch=32)
    reqs = [_req(i, f"p{k}", nv, t)
            for i, (t, k, nv) in enumerate(serving_requests(500, 4))]
    for r in reqs:
        s.add(r)
    seen, last = [], {}
    while True:
        nb = s.next_batch()
        if nb is None:
            break
        name, batch = nb
        assert batch and sum(r.nvec for r in batch) <= 32
        assert all(r.plan == name for r in batch)
        for r in batch:
            assert last.get(name, -1) < r.rid
            last[name] = r.rid
        seen += [r.rid for r in batch]
    assert sorted(seen) == list(range(500))


def test_oversized_request_is_rejected():
    s = Scheduler(max_batch=4)
    with pytest.raises(ValueError):
        s.add(_req(0, "a", 5))


class _Fake:
    def __init__(self, name, size, log):
        self.name, self.footprint, self.log = name, size, log

    def close(self):
        self.log.append(self.name)


def test_cache_evicts_least_recently_used_and_refuses_oversized():
    closed = []
    sizes = {"a": 40, "b": 30, "c": 50, "huge": 101}
    cache = PlanCache(100, lambda n: _Fake(n, sizes[n], closed),
                      lambda n: sizes[n])
    cache.get("a")
    cache.get("b")
    cache.get("a")                        # a is now the most recent
    cache.get("c")                        # 120 > 100: evict b (LRU)
    assert closed == ["b"] and cache.names() == ["a", "c"]
    assert cache.resident_bytes == 90
    with pytest.raises(AdmissionError):
        cache.get("huge")                 # refused before it is built
    assert closed == ["b"] and cache.names() == ["a", "c"]
    assert cache.builds == 3
    # pinned plans are never evicted
    with pytest.raises(AdmissionError):
        cache.get("b", pinned={"a", "c"})
    assert cache.names() == ["a", "c"]
    cache.get("b", pinned={"c"})          # evicts a only
    assert cache.names() == ["c", "b"] and cache.evictions == 2
    cache.clear()
    assert cache.resident_bytes == 0


def test_summary_statistics():
    reqs = []
    for i in range(100):
        r = _req(i, "a", 2, t=i * 0.01)
        r.done = r.arrival + (i + 1) * 1e-3
        reqs.append(r)
    bad = _req(100, "a", 1)
    bad.error = "refused"
    s = summarize(reqs + [bad], lambda name: 1000)
    assert s["served"] == 100 and s["failed"] == 1
    assert abs(s["p50_ms"] - 50.5) < 1e-9
    assert abs(s["p99_ms"] - 99.01) < 1e-9
    span = 0.99 + 0.1
    assert abs(s["throughput"] - 100 * 2 * 1000 / span) < 1e-6


def test_request_stream_is_seeded_and_weighted():
    a = serving_requests(2000, 4, rate=100.0)
    b = serving_requests(2000, 4, rate=100.0)
    assert a == b
    t = [x[0] for x in a]
    assert all(t[i] < t[i + 1] for i in range(len(t) - 1))
    assert 15 < t[-1] < 25                 # about 2000 / 100 s
    kinds = [x[1] for x in a]
    assert set(kinds) == set(range(len(SERVING_SHAPES)))
    assert kinds.count(0) > kinds.count(26)  # N = 2^12 vs 2^20: 16 vs 1
    # the mix: every 1D depth 12..20 (odd ones too), 2D n = 64..512, r in
    # {1, 2, 4} for both, 1..32 vectors per request
    shapes = [SERVING_SHAPES[k][0] for k in set(kinds)]
    assert {n for d, n, *_ in shapes if d == 1} == {1 << k
                                                     for k in range(12, 21)}
    assert {n for d, n, *_ in shapes if d == 2} == {64, 128, 256, 512}
    for dim in (1, 2):
        assert {s[4] for s in shapes if s[0] == dim} == {1, 2, 4}
    assert {x[2] for x in a} == set(range(1, 33))


def test_busy_plans_are_skipped_without_losing_order():
    s = Scheduler(max_batch=8)
    for rid, plan in enumerate(["a", "b", "a", "c", "b"]):
        s.add(_req(rid, plan, 1, t=rid))
    name, b = s.next_batch(busy={"a"})
    assert name == "b" and [r.rid for r in b] == [1, 4]
    assert s.next_batch(busy={"a", "c"}) is None
    name, b = s.next_batch(busy={"c"})
    assert name == "a" and [r.rid for r in b] == [0, 2]
    name, b = s.next_batch()
    assert name == "c" and [r.rid for r in b] == [3]


def test_overlap_fraction():
    from paper_1803_04128_amd.serving import overlap_fraction
    assert overlap_fraction([]) == 0.0
    assert overlap_fraction([(0, 1, "a", 0), (2, 3, "b", 1)]) == 0.0
    # [0,2] and [1,3]: busy 3, two at once during [1,2]
    assert abs(overlap_fraction([(0, 2, "a", 0), (1, 3, "b", 1)]) - 1 / 3) < 1e-12


class _Device:
    """Counts the bytes fake plans hold, as device memory would."""

    def __init__(self):
        self.held = self.peak = 0
        self.built = []

    def build(self, name, size, fail=False):
        if fail:
            raise RuntimeError("[-2] hipMalloc failed")
        self.built.append(name)
        self.held += size
        self.peak = max(self.peak, self.held)
        dev = self

        class _P:
            footprint = size

            def close(self):
                dev.held -= size
        return _P()


def test_admission_never_exceeds_the_budget_and_builds_once():
    dev = _Device()
    sizes = {"a": 40, "b": 30, "c": 50, "d": 60, "e": 100}
    cache = PlanCache(100, lambda n: dev.build(n, sizes[n]),
                      lambda n: sizes[n])
    for name in "abcadbeca":
        cache.get(name)
        assert dev.held == cache.resident_bytes <= 100
    assert dev.peak <= 100
    # one build per admission: a plan is rebuilt only after its eviction
    assert dev.built.count("a") == 3 and cache.builds == len(dev.built)
    # no room next to pinned plans: refused before building anything
    n_built = len(dev.built)
    cache.clear()
    cache.get("c")
    with pytest.raises(PinnedError):
        cache.get("d", pinned={"c"})
    assert len(dev.built) == n_built + 1 and dev.held == 50


def test_failed_build_is_an_admission_error_of_that_plan():
    dev = _Device()
    sizes = {"a": 40, "bad": 30}
    cache = PlanCache(100, lambda n: dev.build(n, sizes[n], fail=n == "bad"),
                      lambda n: sizes[n])
    cache.get("a")
    with pytest.raises(AdmissionError, match="build failed"):
        cache.get("bad")
    assert cache.names() == ["a"] and dev.held == 40
