"""Host-side pieces of the request loop (no GPU): the HBM budget blocks and
wakes admissions, and the request stream is seeded and reproducible."""
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
