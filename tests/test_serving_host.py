"""Host logic of the serving loop (no GPU): batch formation, one request in flight per
simulation, arrival order, HBM-budget admission with least-recently-used eviction, the
Poisson arrival stream and the latency summary."""
import math

import numpy as np

from paper_2401_08586_amd.serving import Request, Scheduler, percentile, poisson_arrivals, summarize


def test_batch_takes_each_idle_sim_once_in_arrival_order():
    s = Scheduler(sizes=[10, 20, 30, 40], nbytes=[1, 1, 1, 1])
    for t, sim in enumerate([2, 0, 2, 1, 3, 0]):
        s.push(Request(sim, float(t)))
    s.start([3])  # sim 3 busy
    b = s.next_batch()
    assert [r.sim for r in b] == [2, 0, 1]
    assert [r.arrival for r in b] == [0.0, 1.0, 3.0]
    # the rest stays queued in arrival order
    assert [(r.sim, r.arrival) for r in s.queue] == [(2, 2.0), (3, 4.0), (0, 5.0)]


def test_batch_particle_budget():
    s = Scheduler(sizes=[600, 500, 300, 5000], nbytes=[1] * 4, max_batch_particles=1000)
    for sim in (0, 1, 2, 3):
        s.push(Request(sim, 0.0))
    b = s.next_batch()
    assert [r.sim for r in b] == [0, 2]  # 600 + 300; 500 would pass the budget
    s.start([0, 2])
    b = s.next_batch()
    assert [r.sim for r in b] == [1]  # 5000 alone would fit only as a first request
    s.start([1])
    b = s.next_batch()
    assert [r.sim for r in b] == [3]  # a request above the budget still runs, alone


def test_batch_shares_one_group():
    s = Scheduler(sizes=[1] * 5, nbytes=[1] * 5, groups=[2, 3, 2, 3, 2])
    for sim in (1, 0, 3, 2, 4):
        s.push(Request(sim, 0.0))
    assert [r.sim for r in s.next_batch()] == [1, 3]      # the first request's group (3D)
    assert [r.sim for r in s.next_batch()] == [0, 2, 4]   # then the 2D ones


def test_admission_evicts_least_recently_used_idle_sims():
    s = Scheduler(sizes=[1] * 5, nbytes=[40, 30, 20, 50, 10], budget_bytes=100)
    assert s.admit([0, 1]) == ([0, 1], [])
    assert s.admit([2]) == ([2], [])            # 90 bytes resident
    s.start([2])
    need, evict = s.admit([3])                  # 50 more: evicting the LRU idle sim 0 suffices
    assert need == [3] and evict == [0]
    assert s.resident_bytes() == 100
    s.finish([2])
    need, evict = s.admit([4, 1])               # 10 more; 1 is in the batch, 2 is LRU and idle
    assert need == [4] and evict == [2]
    assert s.resident_bytes() == 90
    assert list(s.resident) == [3, 4, 1]
    assert s.evictions == 2 and s.admissions == 5


def test_admission_never_evicts_busy_or_batch_sims_and_admits_oversized_batches():
    s = Scheduler(sizes=[1] * 3, nbytes=[60, 60, 150], budget_bytes=100)
    s.admit([0])
    s.start([0])
    need, evict = s.admit([2])                  # 150 > budget; 0 is busy: kept
    assert need == [2] and evict == []
    s.finish([0])
    need, evict = s.admit([1])                  # 0 idle and LRU, 2 idle: both go
    assert evict == [0, 2]
    assert s.admit([1]) == ([], [])


def test_poisson_arrivals():
    a = poisson_arrivals(1000.0, 20000, nsims=64, seed=3)
    t = np.array([x for x, _ in a])
    assert np.all(np.diff(t) >= 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1e-3) < 3e-5          # mean gap 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.03  # exponential: cv = 1
    sims = np.array([s for _, s in a])
    assert sims.min() == 0 and sims.max() == 63
    assert a == poisson_arrivals(1000.0, 20000, nsims=64, seed=3)


def test_summary():
    reqs = []
    for i in range(100):
        r = Request(i % 4, arrival=i * 1e-3)
        r.done_ms = i + 1.0 + (i % 10)   # latency 1..10 ms
        r.issued = r.arrival + 1e-3 * (i % 10) / 2  # half of it queued
        r.device_ms = 1.0 + (i % 10) / 2
        r.nnz = 1000
        r.batch = i // 2
        reqs.append(r)
    out = summarize(reqs, warmup=0)
    assert out["requests"] == 100
    assert math.isclose(out["queue_p50_ms"], percentile([(i % 10) / 2 for i in range(100)], 50))
    assert math.isclose(out["device_p99_ms"], percentile([1 + (i % 10) / 2 for i in range(100)], 99))
    # the tail (latency 10 ms) queued 4.5 ms and ran 5.5 ms
    assert math.isclose(out["tail_queue_ms"], 4.5) and math.isclose(out["tail_device_ms"], 5.5)
    assert math.isclose(out["p50_ms"], percentile([1 + (i % 10) for i in range(100)], 50))
    assert out["p99_ms"] == percentile([1 + (i % 10) for i in range(100)], 99)
    assert out["mean_batch"] == 2.0
    assert math.isclose(out["gpairs_per_s"], 100 * 1000 / ((99 + 1 + 9) * 1e-3) / 1e9)
    assert summarize(reqs, warmup=100) == {}
