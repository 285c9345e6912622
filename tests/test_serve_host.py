"""Host-side pieces of the request loop (no GPU): the HBM budget blocks and
wakes admissions, the batched loop's intake takes requests of the grid sides
below their limit in arrival order, and the request stream is seeded and
reproducible."""
import threading
import time

import numpy as np
import pytest


def test_budget_blocks_until_release():
    from paper_2608_29082_amd.serve import _Budget
    b = _Budget(100)
    b.acquire(70)
    got = []

    def worker():
        b.acquire(50)
        got.append(time.perf_counter())

    t = threading.Thread(target=worker)
    t.start()
    time.sleep(0.05)
    assert not got
    t_rel = time.perf_counter()
    b.release(70)
    t.join(2)
    assert got and got[0] >= t_rel
    with pytest.raises(MemoryError):
        b.acquire(1000)


def test_request_stream_reproducible():
    from paper_2608_29082_amd.serve import make_stream
    a = make_stream(20, 5.0, seed=2)
    b = make_stream(20, 5.0, seed=2)
    assert [r.side for r in a] == [r.side for r in b]
    assert all(np.array_equal(x.f, y.f) and np.array_equal(x.blocks, y.blocks) for x, y in zip(a, b))
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    assert set(r.side for r in make_stream(200, 0.0, seed=1)) == {65, 129, 257, 513, 1025}


def _req(rid, side):
    from paper_2608_29082_amd.serve import Request
    return Request(rid, side, np.ones((16, 16)))


def test_intake_skips_a_side_at_its_limit():
    """FIFO within a side; a side whose set-up hierarchies are all waiting for
    slots (at the limit) does not hold up the other sides' requests behind it."""
    from paper_2608_29082_amd.serve import Intake
    it = Intake(limit=1)
    for rid, side in enumerate([513, 513, 65, 513, 65]):
        it.put(_req(rid, side), 0.0)
    it.close()
    order = [it.take()[0].rid]          # 513 (rid 0): 513 now at its limit
    order.append(it.take()[0].rid)      # the oldest request of a side below its limit: 65 (rid 2)
    it.release(65)
    order.append(it.take()[0].rid)      # 65 again (rid 4); 513 still at its limit
    it.release(513)
    order.append(it.take()[0].rid)      # 513 (rid 1), then (rid 3) after the next release
    it.release(513)
    order.append(it.take()[0].rid)
    assert order == [0, 2, 4, 1, 3]
    it.release(65)
    it.release(513)
    assert it.take() is None             # closed and empty


def test_intake_wakes_a_waiting_worker_on_release():
    from paper_2608_29082_amd.serve import Intake
    it = Intake(limit=1)
    it.put(_req(0, 129), 0.0)
    it.put(_req(1, 129), 0.0)
    assert it.take()[0].rid == 0
    got = []
    t = threading.Thread(target=lambda: got.append(it.take()))
    t.start()
    time.sleep(0.05)
    assert not got                       # 129 at its limit: the worker waits
    it.release(129)
    t.join(2)
    assert got and got[0][0].rid == 1
    it.close()
    it.release(129)
    assert it.take() is None
