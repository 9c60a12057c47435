"""Continuous-batching tile server over resident indexes.

The paper serves tiles through a web server that turns requests into tasks
(Sec. 4.1), a FIFO task pool with a result pool (Sec. 4.2) and an engine
whose idle processes take the next task as soon as they are free (Sec. 4.3).
Here the same roles map onto one GPU:

* ``Scheduler`` -- the task pool.  Arrived requests wait in FIFO order and
  are admitted while in-flight slots and device memory allow; each admitted
  request holds ``request_bytes`` of device memory (its tile frontier --
  the candidate buffer of its pixel blocks -- its bookkeeping and its 8 KiB
  mask) until its result is back on the host.
* ``GpuExecutor`` -- the engine.  One graph-captured ``hv_batcher`` per HIP
  stream; whenever a stream is idle, everything admitted so far is launched
  on it as one batch (continuous batching), so batches on different streams
  overlap on the device.  Finished masks are copied to pinned host memory
  (the result pool) before a request counts as complete.
* ``serve`` -- the loop: open-loop arrivals at their scheduled times,
  completions polled through HIP events, latency = completion - arrival.

The scheduler takes its clock from the caller, so its admission and batching
logic runs on the CPU against a simulated clock and a fake executor.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

MASK_BYTES = 8192


def workspace_bytes_per_request() -> int:
    """Device workspace one request occupies in a batch: request record (24 B),
    frontier (256 x 4 B), frontier size, level and region bits (16 B),
    work-list and empty-list entries (2 x 4 B), completion counter (4 B) and
    stamp (8 B)."""
    return 24 + 256 * 4 + 16 + 4 + 4 + 4 + 8


@dataclass
class Scheduler:
    """FIFO admission and batching; pure host logic with an injected clock."""
    max_batch: int = 4096                 # requests per launch
    max_inflight: int = 16384             # admitted and not yet complete
    mem_budget: int = 1 << 30             # device bytes for admitted requests
    request_bytes: int = MASK_BYTES + workspace_bytes_per_request()
    queue: collections.deque = field(default_factory=collections.deque)
    inflight: int = 0
    mem_used: int = 0
    peak_mem: int = 0
    peak_inflight: int = 0

    def arrive(self, rid: int) -> None:
        self.queue.append(rid)

    def admissible(self) -> int:
        """How many queued requests could be admitted now."""
        by_slots = self.max_inflight - self.inflight
        by_mem = (self.mem_budget - self.mem_used) // self.request_bytes
        return max(0, min(len(self.queue), by_slots, by_mem, self.max_batch))

    def take_batch(self) -> list:
        """Admit and return the next batch (FIFO), or [] if nothing fits."""
        k = self.admissible()
        batch = [self.queue.popleft() for _ in range(k)]
        self.inflight += k
        self.mem_used += k * self.request_bytes
        self.peak_mem = max(self.peak_mem, self.mem_used)
        self.peak_inflight = max(self.peak_inflight, self.inflight)
        return batch

    def complete(self, n: int) -> None:
        self.inflight -= n
        self.mem_used -= n * self.request_bytes
        assert self.inflight >= 0 and self.mem_used >= 0


class GpuExecutor:
    """Batches on several HIP streams, each with its own graph-captured batcher."""

    def __init__(self, reqs: np.ndarray, streams: int = 2, max_batch: int = 4096, max_indexes: int = 8,
                 max_levels: int = 10, launch=None, keep_masks: bool = False):
        import torch

        from . import hv
        self.hv, self.torch = hv, torch
        self.reqs = reqs
        self.keep_masks = keep_masks
        self.masks = np.zeros((len(reqs), MASK_BYTES), dtype=np.uint8) if keep_masks else None
        self.lanes = []
        for _ in range(streams):
            s = torch.cuda.Stream()          # default priority
            with torch.cuda.stream(s):
                b = hv.hv_batcher_create(max_batch, max_indexes=max_indexes, max_levels=max_levels, launch=launch)
            self.lanes.append({
                "stream": s, "batcher": b, "busy": None,
                "out": torch.empty((max_batch, MASK_BYTES), dtype=torch.uint8, device="cuda"),
                "host": torch.empty((max_batch, MASK_BYTES), dtype=torch.uint8, pin_memory=True),
                "event": torch.cuda.Event(),
            })

    def idle_lane(self):
        for k, ln in enumerate(self.lanes):
            if ln["busy"] is None:
                return k
        return None

    def launch(self, lane: int, ids: list) -> None:
        ln = self.lanes[lane]
        ids = np.asarray(ids, dtype=np.int64)
        with self.torch.cuda.stream(ln["stream"]):
            self.hv.hv_batcher_run(ln["batcher"], self.reqs[ids], ln["out"])
            ln["host"][:len(ids)].copy_(ln["out"][:len(ids)], non_blocking=True)
            ln["event"].record(ln["stream"])
        ln["busy"] = ids

    def poll(self):
        """Returns [(ids, completion_time)] for batches finished since the last poll."""
        done = []
        for ln in self.lanes:
            if ln["busy"] is not None and ln["event"].query():
                t = time.perf_counter()
                ids = ln["busy"]
                if self.keep_masks:
                    self.masks[ids] = ln["host"][:len(ids)].numpy()
                ln["busy"] = None
                done.append((ids, t))
        return done

    def close(self):
        self.torch.cuda.synchronize()
        for ln in self.lanes:
            self.hv.hv_batcher_free(ln["batcher"])
        self.lanes = []


def serve(arrivals: np.ndarray, scheduler: Scheduler, executor, clock=time.perf_counter,
          sleep=time.sleep, max_batch: int | None = None) -> dict:
    """Serves requests 0..n-1 arriving at ``arrivals`` seconds (sorted) after
    the start.  Returns per-request latency (s) and throughput figures."""
    n = len(arrivals)
    if max_batch is not None:
        scheduler.max_batch = max_batch
    t0 = clock()
    done_at = np.full(n, np.nan)
    nxt = 0
    finished = 0
    batches = 0
    sizes = []
    while finished < n:
        now = clock() - t0
        while nxt < n and arrivals[nxt] <= now:
            scheduler.arrive(nxt)
            nxt += 1
        for ids, t in executor.poll():
            done_at[ids] = t - t0
            scheduler.complete(len(ids))
            finished += len(ids)
        lane = executor.idle_lane()
        while lane is not None and scheduler.queue:
            batch = scheduler.take_batch()
            if not batch:
                break
            executor.launch(lane, batch)
            batches += 1
            sizes.append(len(batch))
            lane = executor.idle_lane()
        if finished < n and nxt < n and not scheduler.queue and executor.idle_lane() is not None:
            gap = arrivals[nxt] - (clock() - t0)
            if gap > 2e-4:
                sleep(gap - 1e-4)
    makespan = np.nanmax(done_at) if n else 0.0
    lat = done_at - arrivals
    return {
        "requests": n, "batches": batches,
        "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
        "tiles_per_s": n / makespan if makespan > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if n else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if n else None,
        "max_ms": float(np.max(lat) * 1e3) if n else None,
        "peak_inflight": scheduler.peak_inflight, "peak_mem_bytes": scheduler.peak_mem,
        "latency_s": lat,
    }
