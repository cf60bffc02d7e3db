"""Admission core of the serving form (host only): slot ranges, HBM budget, FIFO order."""
import numpy as np
import pytest

from paper_2601_22074_amd.serve import Scheduler, SlotPool
from workloads.requests import Request, mean_request_work, poisson_requests


def test_slot_pool_first_fit_and_coalescing():
    p = SlotPool(100)
    a = p.alloc(30)
    b = p.alloc(30)
    c = p.alloc(30)
    assert (a, b, c) == (0, 30, 60)
    assert p.alloc(11) is None
    p.release(b, 30)
    assert p.alloc(31) is None             # the hole is 30 wide
    p.release(a, 30)
    assert p.free == [(0, 60), (90, 10)]   # merged with its right neighbour
    p.release(c, 30)
    assert p.free == [(0, 100)]
    with pytest.raises(AssertionError):
        p.release(10, 5)


def test_slot_pool_random_against_bitmap():
    rng = np.random.default_rng(3)
    cap = 257
    p = SlotPool(cap)
    used = np.zeros(cap, bool)
    held = []
    for _ in range(3000):
        if held and rng.random() < 0.45:
            s, n = held.pop(int(rng.integers(len(held))))
            p.release(s, n)
            used[s:s + n] = False
        else:
            n = int(rng.integers(1, 40))
            s = p.alloc(n)
            # first fit: the lowest start of a free run of n slots
            runs = [i for i in range(cap - n + 1) if not used[i:i + n].any()]
            assert s == (runs[0] if runs else None)
            if s is not None:
                used[s:s + n] = True
                held.append((s, n))
        assert p.free_slots() == cap - used.sum()


def _sched(budget, cap=1000):
    return Scheduler({"a": cap, "b": cap}, {"a": 100, "b": 1000}, budget)


def test_budget_blocks_and_fifo():
    s = _sched(budget=50_000)
    r = [Request(0, "b", 30, 10, 1), Request(1, "a", 10, 10, 2), Request(2, "b", 30, 10, 3)]
    for x in r:
        s.submit(x)
    got = s.admit()
    assert [x.rid for x, _ in got] == [0, 1]      # 30 000 + 1 000 bytes; the third needs 30 000 more
    assert s.used == 31_000 and len(s.queue) == 1
    assert s.admit() == []
    s.release(got[0][0], got[0][1])
    got2 = s.admit()
    assert [x.rid for x, _ in got2] == [2] and s.used == 31_000
    assert s.peak <= s.budget


def test_head_of_line_blocks_later_requests():
    s = _sched(budget=10_000)
    s.submit(Request(0, "b", 8, 1, 0))
    s.submit(Request(1, "b", 8, 1, 0))
    s.submit(Request(2, "a", 1, 1, 0))            # small, but behind a blocked request
    got = s.admit()
    assert [x.rid for x, _ in got] == [0]
    assert [x.rid for x in s.queue] == [1, 2]


def test_pool_fragmentation_blocks_until_release():
    s = Scheduler({"a": 10}, {"a": 1}, 10 ** 9)
    for i, n in enumerate([4, 2, 4]):
        s.submit(Request(i, "a", n, 1, 0))
    got = s.admit()
    assert [st for _, st in got] == [0, 4, 6]
    s.release(got[0][0], 0)
    s.release(got[2][0], 6)
    s.submit(Request(3, "a", 5, 1, 0))            # 8 slots free, but no 5 in a row
    assert s.admit() == []
    s.release(got[1][0], 4)
    assert s.admit()[0][1] == 0


def test_never_fitting_request_is_rejected():
    s = _sched(budget=1000)
    with pytest.raises(ValueError):
        s.submit(Request(0, "b", 2, 1, 0))
    with pytest.raises(ValueError):
        _sched(budget=10 ** 9, cap=4).submit(Request(0, "a", 5, 1, 0))


def test_poisson_request_stream():
    rs = poisson_requests(200.0, 60.0, seed=1)
    n = np.array([r.n for r in rs])
    h = np.array([r.horizon for r in rs])
    t = np.array([r.arrival for r in rs])
    assert abs(len(rs) - 12000) < 4 * np.sqrt(12000)
    assert np.all(np.diff(t) > 0) and t[-1] < 60
    assert n.min() >= 16 and n.max() <= 4096 and h.min() >= 50 and h.max() <= 500
    # log-uniform world counts: log n is uniform, so its mean is the midpoint
    assert abs(np.log(n).mean() - (np.log(16) + np.log(4097)) / 2) < 0.05
    assert abs(h.mean() - 275) < 3
    assert {r.name for r in rs} == {"chain3", "quadruped", "humanoid", "arm_box"}
    assert abs(mean_request_work() / (n * h).mean() - 1) < 0.05
    assert poisson_requests(200.0, 1.0, seed=1)[:5] == rs[:5]


def test_admission_bounded_by_device_free_memory():
    """With a free-memory probe, a request waits while the device reports less free memory
    (less the reserve) than its worlds need, even when the budget has room; it is admitted
    once the device frees memory, in FIFO order."""
    free = {"bytes": 10_000}
    s = Scheduler({"a": 100}, {"a": 100}, budget=1 << 30, free_probe=lambda: free["bytes"], reserve=1_000)
    s.submit(Request(0, "a", 50, 10, 0))     # needs 5000 <= 10000 - 1000
    s.submit(Request(1, "a", 40, 10, 1))     # needs 4000
    got = s.admit()
    assert [r.rid for r, _ in got] == [0, 1]
    free["bytes"] = 4_000                     # the device filled up
    s.submit(Request(2, "a", 5, 10, 2))       # needs 500 > 4000 - 1000? no: 500 <= 3000
    s.submit(Request(3, "a", 40, 10, 3))      # needs 4000 > 3000: waits (and blocks the queue)
    got = s.admit()
    assert [r.rid for r, _ in got] == [2]
    assert s.admit() == [] and s.blocked_by_device >= 1
    for r, st in [(Request(0, "a", 50, 10, 0), 0), (Request(1, "a", 40, 10, 1), 50)]:
        s.release(r, st)
    free["bytes"] = 20_000
    got = s.admit()
    assert [r.rid for r, _ in got] == [3]
