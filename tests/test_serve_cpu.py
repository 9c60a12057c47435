"""The serving loop's admission and batching logic on the CPU: a simulated
clock and a fake executor whose batches take a + b * size seconds.  This is a
test double of the GPU executor, not a second product path."""
import numpy as np
import pytest

serve_mod = pytest.importorskip("paper_2005_12489_amd.serve")


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-6          # every look at the clock costs a microsecond
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeExecutor:
    def __init__(self, clock, lanes=2, a=200e-6, b=2e-6):
        self.clock, self.a, self.b = clock, a, b
        self.busy = [None] * lanes
        self.launched = []

    def idle_lane(self):
        for k, x in enumerate(self.busy):
            if x is None:
                return k
        return None

    def launch(self, lane, ids):
        assert self.busy[lane] is None
        self.busy[lane] = (list(ids), self.clock.t + self.a + self.b * len(ids))
        self.launched.append(list(ids))

    def poll(self):
        out = []
        for k, x in enumerate(self.busy):
            if x is not None and x[1] <= self.clock.t:
                out.append((np.asarray(x[0]), x[1]))
                self.busy[k] = None
        return out


def _run(rate, n, max_batch=4096, mem_budget=1 << 30, max_inflight=16384, lanes=2, seed=0):
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1.0 / rate, n))
    clk = SimClock()
    sch = serve_mod.Scheduler(max_batch=max_batch, mem_budget=mem_budget, max_inflight=max_inflight)
    ex = FakeExecutor(clk, lanes=lanes)
    st = serve_mod.serve(arr, sch, ex, clock=clk, sleep=clk.sleep)
    return st, ex, sch, arr


def test_every_request_served_once_in_fifo_batches():
    st, ex, sch, arr = _run(20000.0, 5000)
    ids = np.concatenate([np.asarray(b) for b in ex.launched])
    assert np.array_equal(ids, np.arange(5000))            # FIFO, each exactly once
    assert np.all(np.isfinite(st["latency_s"])) and np.all(st["latency_s"] > 0)
    assert sch.inflight == 0 and sch.mem_used == 0
    assert st["batches"] == len(ex.launched) and st["mean_batch"] > 1


def test_batch_size_slots_and_memory_limits_hold():
    per = serve_mod.Scheduler().request_bytes
    st, ex, sch, _ = _run(200000.0, 6000, max_batch=300, mem_budget=700 * per, max_inflight=10000)
    assert max(len(b) for b in ex.launched) <= 300
    assert sch.peak_mem <= 700 * per
    st, ex, sch, _ = _run(200000.0, 6000, max_batch=4096, max_inflight=450)
    assert sch.peak_inflight <= 450


def test_batching_beats_one_launch_per_request_under_load():
    batched, *_ = _run(50000.0, 8000)
    single, *_ = _run(50000.0, 8000, max_batch=1)
    assert batched["p99_ms"] < single["p99_ms"] / 10
    assert batched["tiles_per_s"] > 5 * single["tiles_per_s"]


def test_light_load_latency_is_one_launch():
    st, ex, *_ = _run(100.0, 200)
    # at 100 req/s nearly every request is launched alone and waits ~a + b
    assert st["p50_ms"] < 0.3
