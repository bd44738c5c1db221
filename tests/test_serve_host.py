"""Host logic of the served stream (CPU): how a free slot's batch is formed
(paper_1811_01277_amd.serve.take_batch) — the batch cap, the work bound, the
memory budget and the idle-device rule — and the latency statistics."""
from paper_1811_01277_amd.serve import take_batch, latency_stats


class Req:
    def __init__(self, rid, flops, size, arrival=0.0, ready=0.0, start=0.0, done=1.0):
        self.rid, self._flops, self.size = rid, flops, size
        self.arrival, self.t_ready, self.t_start, self.t_done = arrival, ready, start, done

    def flops(self):
        return self._flops


def ids(rs):
    return [r.rid for r in rs]


def size(r):
    return r.size


def test_cap_and_order():
    ready = [Req(i, 1.0, 10) for i in range(5)]
    batch, nbytes, rest = take_batch(ready, 3, 0, 1000, 1e9, size)
    assert ids(batch) == [0, 1, 2] and nbytes == 30 and ids(rest) == [3, 4]


def test_work_bound_first_request_always_goes():
    big, small = Req(0, 100.0, 1), Req(1, 5.0, 1)
    batch, _, rest = take_batch([big, small], 8, 0, 1000, 50.0, size)
    assert ids(batch) == [0] and ids(rest) == [1]          # big alone past the bound
    batch, _, rest = take_batch([small, Req(2, 40.0, 1), Req(3, 20.0, 1), Req(4, 5.0, 1)],
                                8, 0, 1000, 50.0, size)
    # 5 + 40 fits, + 20 does not, + 5 does (later small requests still join)
    assert ids(batch) == [1, 2, 4] and ids(rest) == [3]


def test_memory_budget_and_idle_device():
    ready = [Req(0, 1.0, 600), Req(1, 1.0, 300), Req(2, 1.0, 100)]
    # busy device: only what fits next to the 500 bytes in flight
    batch, nbytes, rest = take_batch(ready, 8, 500, 1000, 1e9, size)
    assert ids(batch) == [1, 2] and nbytes == 400 and ids(rest) == [0]
    # idle device: the oldest request goes even above the budget, alone
    batch, nbytes, rest = take_batch(ready, 8, 0, 200, 1e9, size)
    assert ids(batch) == [0] and nbytes == 600 and ids(rest) == [1, 2]
    # nothing fits on a busy device
    batch, nbytes, rest = take_batch(ready, 8, 950, 1000, 1e9, size)
    assert batch == [] and nbytes == 0 and ids(rest) == [0, 1, 2]


def test_latency_stats():
    rs = [Req(i, 2e9, 1, arrival=0.1 * i, ready=0.1 * i, start=0.1 * i, done=0.1 * i + 0.01 * (i + 1))
          for i in range(10)]
    st = latency_stats(rs)
    assert st["solves"] == 10
    assert abs(st["span_s"] - 1.0) < 1e-9                  # 0 .. 0.9 + 0.10
    assert abs(st["max_ms"] - 100.0) < 1e-6
    assert abs(st["service_ms"] - 55.0) < 1e-6
    assert abs(st["gflops"] - 20.0) < 1e-6
