"""Serving scheduler on the host (fake backend, virtual clock): admission by
free slots and HBM budget, continuous batching, completion and latency
accounting."""
import numpy as np
import pytest

from serving_fake import FakeBackend
from paper_2609_08800_amd.serving import Request, ServingEngine, SlotAllocator, percentile, \
    poisson_arrivals


class B:  # minimal packed-batch stand-in: only the world count matters to the fake backend
    def __init__(self, n):
        self.n_worlds = n


def run(reqs, capacity=16, budget=1e12, tick=0.01):
    be = FakeBackend(capacity, tick_seconds=tick)
    eng = ServingEngine(be, budget, clock=be.clock)
    out = eng.run(reqs)
    return be, eng, out


def test_slot_allocator_first_fit_and_merge():
    a = SlotAllocator(10)
    assert a.alloc(4) == 0 and a.alloc(4) == 4 and a.alloc(4) == -1
    a.release(0, 4)
    assert a.alloc(3) == 0
    a.release(4, 4)
    a.release(0, 3)
    assert a.free == [(0, 10)]


def test_every_request_completes_all_iterations():
    reqs = [Request(i, B(2 + i), T=3 + i, iters=4, arrival=0.005 * i) for i in range(5)]
    be, eng, out = run(reqs)
    assert len(out["requests"]) == 5
    for r in out["requests"]:
        assert len(r.iter_latency) == 4 and len(r.losses) == 4
        assert r.finished_at >= r.admitted_at >= r.arrival
        # an iteration is T forward ticks and T backward ticks
        assert min(r.iter_latency) >= 2 * r.T * 0.01 - 1e-12


def test_admission_waits_for_free_slots():
    reqs = [Request(i, B(6), T=2, iters=1, arrival=0.0) for i in range(3)]
    be, eng, out = run(reqs, capacity=12)
    admitted = sorted((r.admitted_at, r.rid) for r in out["requests"])
    assert admitted[0][0] == admitted[1][0] == 0.0
    assert admitted[2][0] > 0.0   # the third waits until a range of 6 slots frees up
    assert max(n_f + n_b for _, n_f, n_b, _ in eng.ticks) <= 12


def test_admission_respects_hbm_budget():
    reqs = [Request(i, B(2), T=4, iters=1, arrival=0.0) for i in range(3)]
    per = 1.0 * 2 * 5
    be, eng, out = run(reqs, capacity=64, budget=per * 1.5)
    # only one request fits the budget at a time: their lifetimes do not overlap
    spans = sorted((r.admitted_at, r.finished_at) for r in out["requests"])
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0
    with pytest.raises(ValueError):
        run([Request(9, B(2), T=4, iters=1)], budget=per * 0.5)


def test_continuous_batching_admits_while_others_run():
    early = Request(0, B(4), T=20, iters=2, arrival=0.0)
    late = Request(1, B(4), T=5, iters=1, arrival=0.1)
    be, eng, out = run([early, late], capacity=16)
    # the late request joins ticks in which the early one is still in flight
    shared = [rids for _, _, _, rids in eng.ticks if rids == (0, 1)]
    assert shared
    assert late.admitted_at < early.finished_at
    assert late.finished_at < early.finished_at   # a short request overtakes a long one in flight
    # some tick mixes a forward phase and a backward phase
    assert any(f and b for f, b in be.log)


def test_results_do_not_depend_on_the_mix():
    alone = Request(7, B(3), T=6, iters=3)
    _, _, o1 = run([alone])
    mixed = Request(7, B(3), T=6, iters=3, arrival=0.02)
    others = [Request(i, B(2), T=4 + i, iters=2, arrival=0.01 * i) for i in range(4)]
    _, _, o2 = run([mixed] + others)
    assert np.array_equal(alone.knots, mixed.knots)
    assert all(np.array_equal(a, b) for a, b in zip(alone.losses, mixed.losses))


def test_percentiles_and_arrivals():
    assert percentile([1, 2, 3, 4], 50) == 2.5
    a = poisson_arrivals(100.0, 2.0, seed=1)
    assert all(0 < x < 2.0 for x in a) and a == sorted(a)
    assert 120 < len(a) < 280
    _, _, out = run([Request(i, B(1), T=2, iters=2, arrival=t) for i, t in enumerate(a[:20])])
    assert out["iter_latency_p50_s"] <= out["iter_latency_p99_s"]


def test_deadline_reports_unfinished_and_frees_memory():
    reqs = [Request(i, B(4), T=50, iters=10, arrival=0.0) for i in range(3)]
    be = FakeBackend(8, tick_seconds=0.01)
    eng = ServingEngine(be, 1e12, clock=be.clock)
    out = eng.run(reqs, deadline=2.0)
    assert len(out["unfinished"]) == 3 - len(out["requests"])
    assert out["unfinished"] and eng.used == 0.0 and eng.slots.n_free == 8
    assert out["iterations"] >= 1


def test_lazy_request_worlds_are_built_once_and_only_when_read():
    """The benchmark's deferred request worlds: the world count is known without building
    them, the engine itself reads nothing else (only a backend's admission builds them),
    and the worlds built are those of the same seed, built once."""
    import bench
    import scenes
    lazy = [bench._LazyRequestWorlds(100 + i, 2) for i in range(6)]
    reqs = [Request(i, w, T=3, iters=1, arrival=0.0) for i, w in enumerate(lazy)]
    be = FakeBackend(4, tick_seconds=0.01)
    eng = ServingEngine(be, 1e12, clock=be.clock)
    out = eng.run(reqs)                     # the fake backend reads only the world count
    assert len(out["requests"]) == 6 and all(w._b is None for w in lazy)
    eager = scenes.terrain_request_batch(101, 2)
    assert lazy[1].n_worlds == 2 and lazy[1]._b is None
    assert np.array_equal(lazy[1].q0, eager.q0) and np.array_equal(lazy[1].hmap_heights, eager.hmap_heights)
    built = lazy[1]._b
    _ = lazy[1].u0
    assert lazy[1]._b is built


def test_request_larger_than_the_pool_is_rejected_not_waited_for():
    """A request with more worlds than the pool holds can never be admitted: once
    nothing runs (so nothing will free slots), the engine says so instead of spinning,
    after serving what came before it."""
    reqs = [Request(0, B(4), T=2, iters=1, arrival=0.0), Request(1, B(20), T=2, iters=1, arrival=0.0)]
    be = FakeBackend(16, tick_seconds=0.01)
    eng = ServingEngine(be, 1e12, clock=be.clock)
    with pytest.raises(ValueError, match="can never be admitted"):
        eng.run(reqs)
    assert reqs[0].it == 1  # the admissible request ahead of it was served


@pytest.mark.parametrize("n,T,iters", [(0, 3, 1), (2, 0, 1), (2, 3, 0)])
def test_degenerate_requests_are_rejected(n, T, iters):
    """A request without worlds, steps or iterations is an argument error, raised before
    anything is admitted."""
    be = FakeBackend(16, tick_seconds=0.01)
    eng = ServingEngine(be, 1e12, clock=be.clock)
    with pytest.raises(ValueError, match="at least one world"):
        eng.run([Request(0, B(2), T=2, iters=1), Request(1, B(n), T=T, iters=iters)])
    assert eng.ticks == [] and eng.used == 0.0
