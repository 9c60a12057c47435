"""Continuous-batching tile server over resident indexes.

The paper serves tiles through a web server that turns requests into tasks
(Sec. 4.1), a FIFO task pool with a result pool (Sec. 4.2) and an engine
whose idle processes take the next task as soon as they are free (Sec. 4.3).
Here the same roles map onto one GPU:

* ``Scheduler`` -- the task pool.  Arrived requests wait in FIFO order and
  are admitted while in-flight slots and device memory allow; each admitted
  request holds the device bytes the library reports for it
  (hv_estimate_bytes: its tile frontier -- the candidate buffer its regions
  start from -- its bookkeeping and its 8 KiB mask) until its result is back
  on the host.
* ``GpuExecutor`` -- the engine.  One graph-captured ``hv_batcher`` per HIP
  stream; whenever a stream is idle, everything admitted so far is launched
  on it as one batch (continuous batching), so batches on different streams
  overlap on the device.  Finished masks are copied to pinned host memory
  (the result pool) before a request counts as complete.
* ``serve`` -- the loop: open-loop arrivals at their scheduled times,
  completions polled through HIP events, latency = completion - arrival.
* ``RequestParser`` and ``ResultCache`` -- the paper's task parsing (Sec.
  4.1) and result pool (Sec. 4.2): a request with a wrong expression, a tile
  outside its dataset's bounds, a result still in the pool or a request
  identical to one already queued or running makes no new task.

The scheduler takes its clock from the caller, so its admission and batching
logic runs on the CPU against a simulated clock and a fake executor.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

MASK_BYTES = 8192
MAX_ZOOM = 22
MAX_RADIUS = 64.0

# what parsing makes of a request (Sec. 4.1)
TASK, EMPTY, REJECT = 0, 1, 2


class RequestParser:
    """Parse Tasks (Sec. 4.1) for requests (dataset, z, x, y, r).

    REJECT: a wrong request expression -- unknown dataset, zoom outside
    [0, 22], x or y outside [0, 2^z), r not in (0, 64].  EMPTY: the tile's
    pixel centres grown by r miss the dataset's bounding box (or the dataset
    is empty), so every pixel is unlit; it is answered with a zero mask and
    makes no task.  TASK: anything else.

    ``roots``: per dataset the index's root box (minX, minY, maxX, maxY) in
    normalised Mercator, or None for an empty index.  The test grows the
    tile by slightly more than the kernels do, so it never empties a tile
    they would light."""

    def __init__(self, roots):
        self.roots = [None if b is None else tuple(float(v) for v in b) for b in roots]

    def classify(self, dataset: int, z: int, x: int, y: int, r: float) -> int:
        if not 0 <= dataset < len(self.roots):
            return REJECT
        if not (0 <= z <= MAX_ZOOM) or not (0 <= x < (1 << z) and 0 <= y < (1 << z)):
            return REJECT
        if not (r > 0.0 and r <= MAX_RADIUS):       # also rejects NaN
            return REJECT
        root = self.roots[dataset]
        if root is None:
            return EMPTY
        inv = 1.0 / (256.0 * (1 << z))
        m = r + 1e-4
        x0, x1 = (256.0 * x + 0.5 - m) * inv, (256.0 * x + 255.5 + m) * inv
        y0, y1 = (256.0 * y + 0.5 - m) * inv, (256.0 * y + 255.5 + m) * inv
        if root[0] > x1 or root[2] < x0 or root[1] > y1 or root[3] < y0:
            return EMPTY
        return TASK


class ResultCache:
    """Result Pool (Sec. 4.2): finished masks keyed by the request
    expression (dataset, z, x, y, r).

    An entry older than ``ttl_s`` no longer answers requests.  Expired
    entries are cleaned only when the cached bytes exceed ``cap_bytes``, as
    the paper cleans expired results once memory reaches its limit; if that
    is not enough, the oldest entries go too, so the cap always holds."""

    def __init__(self, cap_bytes: int = 1 << 30, ttl_s: float = 60.0):
        self.cap_bytes, self.ttl_s = int(cap_bytes), float(ttl_s)
        self._d = collections.OrderedDict()      # key -> (time stored, mask), oldest first
        self.bytes = 0
        self.hits = self.misses = self.expired_cleaned = self.evicted = 0

    def __len__(self):
        return len(self._d)

    def get(self, key, now: float):
        e = self._d.get(key)
        if e is None or now - e[0] > self.ttl_s:
            self.misses += 1
            return None
        self.hits += 1
        return e[1]

    def put(self, key, mask: np.ndarray, now: float) -> None:
        old = self._d.pop(key, None)
        if old is not None:
            self.bytes -= old[1].nbytes
        self._d[key] = (now, mask)
        self.bytes += mask.nbytes
        if self.bytes > self.cap_bytes:
            self._clean(now)

    def _clean(self, now: float) -> None:
        # entries are in the order they were stored, so the expired ones lead
        while self._d:
            k, (t, m) = next(iter(self._d.items()))
            if now - t <= self.ttl_s:
                break
            del self._d[k]
            self.bytes -= m.nbytes
            self.expired_cleaned += 1
        while self.bytes > self.cap_bytes and self._d:
            _, (_, m) = self._d.popitem(last=False)
            self.bytes -= m.nbytes
            self.evicted += 1


def request_bytes(index: int, tile, r_px: float) -> int:
    """Device bytes one request holds while it is in a batch, as the library
    itself counts them (hv_estimate_bytes: its records in the batch
    workspace -- the tile frontier its regions start from among them -- and
    its mask)."""
    from . import hv
    return hv.hv_estimate_bytes(int(index), tile, r_px)


@dataclass
class Scheduler:
    """FIFO admission and batching; pure host logic with an injected clock.

    A queued request is admitted when an in-flight slot is free and its
    device bytes fit in what is left of ``mem_budget``; admission stops at
    the first request that does not fit (FIFO).  ``request_bytes`` gives a
    request's bytes: a number for all of them, or a function of the request
    id; None takes the executor's (``serve`` fills it in)."""
    max_batch: int = 4096                 # requests per launch
    max_inflight: int = 16384             # admitted and not yet complete
    mem_budget: int = 1 << 30             # device bytes for admitted requests
    request_bytes: object = None
    queue: collections.deque = field(default_factory=collections.deque)
    inflight: int = 0
    mem_used: int = 0
    peak_mem: int = 0
    peak_inflight: int = 0
    _held: dict = field(default_factory=dict)

    def _bytes(self, rid: int) -> int:
        rb = self.request_bytes
        if rb is None:
            raise ValueError("Scheduler.request_bytes is not set")
        return int(rb(rid)) if callable(rb) else int(rb)

    def arrive(self, rid: int) -> None:
        self.queue.append(rid)

    def admissible(self) -> int:
        """How many queued requests (from the head) could be admitted now."""
        room = min(len(self.queue), self.max_inflight - self.inflight, self.max_batch)
        free = self.mem_budget - self.mem_used
        k = 0
        while k < room:
            b = self._bytes(self.queue[k])
            if b > free:
                break
            free -= b
            k += 1
        return max(0, k)

    def take_batch(self) -> list:
        """Admit and return the next batch (FIFO), or [] if nothing fits."""
        k = self.admissible()
        batch = [self.queue.popleft() for _ in range(k)]
        for rid in batch:
            b = self._bytes(rid)
            self._held[rid] = b
            self.mem_used += b
        self.inflight += k
        self.peak_mem = max(self.peak_mem, self.mem_used)
        self.peak_inflight = max(self.peak_inflight, self.inflight)
        return batch

    def complete(self, ids) -> None:
        """Releases the slots and bytes of completed requests."""
        for rid in ids:
            self.mem_used -= self._held.pop(int(rid))
        self.inflight -= len(ids)
        assert self.inflight >= 0 and self.mem_used >= 0


class GpuExecutor:
    """Batches on several HIP streams, each with its own graph-captured batcher."""

    def __init__(self, reqs: np.ndarray, streams: int = 2, max_batch: int = 4096, max_indexes: int = 8,
                 max_levels: int = 10, launch=None, keep_masks: bool = False, return_masks: bool = False,
                 mem_budget: int | None = None):
        """reqs: the hv_request array of every request that may be served.
        mem_budget: the device bytes the scheduler admits against; a lane
        then holds no more requests than that budget admits at once."""
        import torch

        from . import hv
        self.hv, self.torch = hv, torch
        self.reqs = reqs
        # the library's own count of the device bytes each request holds in a batch
        self.bytes = np.array([hv.hv_estimate_bytes(int(q["index"]), (q["z"], q["x"], q["y"]), float(q["r_px"]))
                               for q in reqs], dtype=np.int64)
        if mem_budget is not None and len(reqs):
            max_batch = max(1, min(max_batch, int(mem_budget // int(self.bytes.min()))))
        self.max_batch = max_batch
        # device memory the executor holds: per lane a batcher (two workspaces)
        # and the masks of one batch
        ws = hv.hv_estimate_batch_bytes(max_batch, max_indexes) - max_batch * MASK_BYTES
        self.device_bytes = streams * (2 * ws + max_batch * MASK_BYTES)
        self.keep_masks = keep_masks
        self.return_masks = return_masks
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

    def request_bytes(self, rid: int) -> int:
        return int(self.bytes[rid])

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
        """Returns [(ids, completion_time, masks)] for batches finished since
        the last poll; masks (len(ids), 8192) when return_masks, else None."""
        done = []
        for ln in self.lanes:
            if ln["busy"] is not None and ln["event"].query():
                t = time.perf_counter()
                ids = ln["busy"]
                rows = ln["host"][:len(ids)].numpy()
                if self.keep_masks:
                    self.masks[ids] = rows
                ln["busy"] = None
                done.append((ids, t, rows.copy() if self.return_masks else None))
        return done

    def close(self):
        self.torch.cuda.synchronize()
        for ln in self.lanes:
            self.hv.hv_batcher_free(ln["batcher"])
        self.lanes = []


def serve(arrivals: np.ndarray, scheduler: Scheduler, executor, clock=time.perf_counter,
          sleep=time.sleep, max_batch: int | None = None, requests: dict | None = None,
          parser: RequestParser | None = None, cache: ResultCache | None = None) -> dict:
    """Serves requests 0..n-1 arriving at ``arrivals`` seconds (sorted) after
    the start.  Returns per-request latency (s) and throughput figures.

    With ``requests`` (arrays "dataset", "tiles" (n, 3) and "r"), arriving
    requests are parsed first: rejected ones complete at once with status
    REJECT, empty ones at once with a zero mask, a hit in ``cache`` at once
    with the cached mask, and a request equal to one already queued or
    running waits for that one instead of making a task.  The executor must
    then return masks from ``poll`` when a cache is given."""
    n = len(arrivals)
    if max_batch is not None:
        scheduler.max_batch = max_batch
    if scheduler.request_bytes is None:
        scheduler.request_bytes = executor.request_bytes
    keep = getattr(executor, "masks", None)
    keyed = requests is not None
    if keyed:
        ds = np.asarray(requests["dataset"])
        tl = np.asarray(requests["tiles"])
        rr = np.asarray(requests["r"], dtype=np.float64)
    status = np.full(n, TASK, dtype=np.int8)
    waiting = {}                 # request key -> ids served by the task in flight
    counts = {"tasks": 0, "rejected": 0, "empty": 0, "cache_hits": 0, "joined": 0}
    zero = np.zeros(MASK_BYTES, dtype=np.uint8)
    t0 = clock()
    done_at = np.full(n, np.nan)
    nxt = 0
    finished = 0
    batches = 0
    sizes = []

    def key_of(i):
        return (int(ds[i]), int(tl[i, 0]), int(tl[i, 1]), int(tl[i, 2]), float(rr[i]))

    while finished < n:
        now = clock() - t0
        while nxt < n and arrivals[nxt] <= now:
            i = nxt
            nxt += 1
            if not keyed:
                scheduler.arrive(i)
                counts["tasks"] += 1
                continue
            kind = parser.classify(*key_of(i)) if parser else TASK
            if kind != TASK:
                status[i] = kind
                done_at[i] = now
                finished += 1
                counts["rejected" if kind == REJECT else "empty"] += 1
                if kind == EMPTY and keep is not None:
                    keep[i] = zero
                continue
            k = key_of(i)
            hit = cache.get(k, now) if cache is not None else None
            if hit is not None:
                done_at[i] = now
                finished += 1
                counts["cache_hits"] += 1
                if keep is not None:
                    keep[i] = hit
                continue
            if k in waiting:
                waiting[k].append(i)
                counts["joined"] += 1
                continue
            waiting[k] = [i]
            scheduler.arrive(i)
            counts["tasks"] += 1
        for res in executor.poll():
            ids, t = res[0], res[1]
            rows = res[2] if len(res) > 2 else None
            done_at[ids] = t - t0
            scheduler.complete(ids)
            finished += len(ids)
            if rows is not None and keep is not None:
                keep[ids] = rows
            if keyed:
                for j, i in enumerate(ids):
                    k = key_of(i)
                    for w in waiting.pop(k, ())[1:]:
                        done_at[w] = t - t0
                        finished += 1
                        if keep is not None:
                            keep[w] = keep[i]
                    if cache is not None:
                        cache.put(k, rows[j], t - t0)
        lane = executor.idle_lane()
        while lane is not None and scheduler.queue:
            batch = scheduler.take_batch()
            if not batch:
                break
            executor.launch(lane, batch)
            batches += 1
            sizes.append(len(batch))
            lane = executor.idle_lane()
        # Sleep until the next arrival only when nothing is queued or in
        # flight; while a batch runs the loop keeps polling, so that its
        # completion is seen at once rather than at the next arrival.
        if finished < n and nxt < n and not scheduler.queue and scheduler.inflight == 0:
            gap = arrivals[nxt] - (clock() - t0)
            if gap > 2e-4:
                sleep(gap - 1e-4)
    makespan = np.nanmax(done_at) if n else 0.0
    lat = done_at - arrivals
    return {
        "requests": n, "batches": batches, **counts, "status": status,
        "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
        "tiles_per_s": n / makespan if makespan > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if n else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if n else None,
        "max_ms": float(np.max(lat) * 1e3) if n else None,
        "peak_inflight": scheduler.peak_inflight, "peak_mem_bytes": scheduler.peak_mem,
        "latency_s": lat,
    }
