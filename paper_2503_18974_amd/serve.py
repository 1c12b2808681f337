"""Serving loop: open-loop arrivals, admission by an HBM budget, continuous batching.

Requests (a packed binary matrix, and whether the caller also wants the int32 side map)
arrive on their own schedule.  The loop:

  * queues every request whose arrival time has passed (the client never waits for the
    server: open loop, so a server that falls behind shows up as growing latency);
  * admits queued requests in arrival order while the device arena (the HBM budget) can hold
    their packed bits, plus their map when one is wanted; a request that does not fit waits
    until earlier ones complete and free their memory;
  * launches everything admitted as one batched call on the next free stream slot
    (ms_max_square_batched, then ms_square_map_from_max for the requests that want a map), so
    requests that arrive while others run on the GPU join the next launch and their work
    overlaps on the device;
  * polls the slots' completion events, hands each result to the caller, and frees the
    request's memory.

Failures stay with the requests they concern: a request that is malformed or larger than the
whole budget is rejected at admission; a batch whose launch or result collection fails fails
only its own requests (their memory is freed and the loop goes on); a device error seen while
polling (the stream can no longer report) fails every request in flight and every request not
yet served, and ends the run.  A request can be cancelled at any time: before launch it is
dropped, in flight its result is discarded when the batch completes.

Latency is measured from a request's arrival time to the moment the loop sees its result;
p50/p99 come from those.  The executor is an interface so the scheduling logic is tested on
the CPU with a simulated device (tests/test_serve.py); GpuExecutor drives the library.
"""
from __future__ import annotations

import bisect
import collections
import ctypes
import gc
import time
from dataclasses import dataclass, field

import numpy as np

ALIGN = 256


def _round_up(x: int, a: int = ALIGN) -> int:
    return (int(x) + a - 1) // a * a


@dataclass
class Request:
    """One detection request.  `bits` is the packed matrix on the host (uint64 or int64,
    (m, ld_words)); `arrival` is seconds after the start of the run."""
    rid: int
    m: int
    n: int
    bits: object
    arrival: float
    want_map: bool = False
    # filled in by the server
    admitted: float | None = None
    launched: float | None = None
    done: float | None = None
    result: tuple | None = None
    error: str | None = None
    cancelled: bool = False

    def cancel(self) -> None:
        """Ask the server to drop this request (before launch) or discard its result."""
        self.cancelled = True

    def invalid(self) -> str | None:
        """Why the request cannot be served, or None."""
        if int(self.m) < 0 or int(self.n) < 0:
            return "negative dimensions"
        shape = getattr(self.bits, "shape", None)
        if self.cells and shape is not None:
            if len(shape) != 2 or int(shape[0]) != int(self.m) or int(shape[1]) < self.ld_words:
                return "packed bits of shape %s do not hold %d rows of %d words" % (
                    tuple(shape), int(self.m), self.ld_words)
        return None

    @property
    def cells(self) -> int:
        return int(self.m) * int(self.n)

    @property
    def ld_words(self) -> int:
        return max(1, (int(self.n) + 63) // 64)

    @property
    def bits_bytes(self) -> int:
        return _round_up(int(self.m) * self.ld_words * 8)

    @property
    def map_bytes(self) -> int:
        return _round_up(int(self.m) * int(self.n) * 4) if self.want_map else 0

    @property
    def device_bytes(self) -> int:
        return self.bits_bytes + self.map_bytes

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


class Arena:
    """First-fit allocator over [0, capacity) in ALIGN-byte units, with coalescing on free.
    Offsets only: the executor maps them onto one device buffer."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity) // ALIGN * ALIGN
        self.free_starts = [0]              # sorted
        self.free_len = {0: self.capacity}
        self.used = {}
        self.in_use = 0
        self.peak = 0

    def alloc(self, nbytes: int):
        size = _round_up(max(int(nbytes), 1))
        for i, s in enumerate(self.free_starts):
            ln = self.free_len[s]
            if ln >= size:
                del self.free_len[s]
                self.free_starts.pop(i)
                if ln > size:
                    rest = s + size
                    self.free_len[rest] = ln - size
                    bisect.insort(self.free_starts, rest)
                self.used[s] = size
                self.in_use += size
                self.peak = max(self.peak, self.in_use)
                return s
        return None

    def free(self, off: int) -> None:
        size = self.used.pop(off)
        self.in_use -= size
        i = bisect.bisect_left(self.free_starts, off)
        # merge with the following block
        if i < len(self.free_starts) and self.free_starts[i] == off + size:
            nxt = self.free_starts.pop(i)
            size += self.free_len.pop(nxt)
        # merge with the preceding block
        if i > 0:
            prv = self.free_starts[i - 1]
            if prv + self.free_len[prv] == off:
                self.free_len[prv] += size
                return
        self.free_len[off] = size
        self.free_starts.insert(i, off)

    def largest_free(self) -> int:
        return max(self.free_len.values(), default=0)


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait(self, until: float) -> None:
        """Idle until `until` (seconds) at most: waits under a millisecond spin (a sleep can
        overshoot by much more than that), longer ones sleep to half a millisecond before."""
        dt = until - self.now()
        if dt > 1e-3:
            time.sleep(dt - 5e-4)


@dataclass
class Stats:
    requests: int = 0
    completed: int = 0
    rejected: int = 0
    failed: int = 0
    cancelled: int = 0
    batches: int = 0
    cells: int = 0
    max_queue: int = 0
    peak_bytes: int = 0
    latencies: list = field(default_factory=list)
    queue_waits: list = field(default_factory=list)    # arrival -> admitted
    launch_waits: list = field(default_factory=list)   # admitted -> launched
    device_times: list = field(default_factory=list)   # launched -> result seen
    first_arrival: float = 0.0
    last_done: float = 0.0
    batch_sizes: list = field(default_factory=list)

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        span = max(self.last_done - self.first_arrival, 1e-9)

        def p99(v):
            return float(np.percentile(np.array(v), 99) * 1e3) if v else 0.0

        return {
            "p99_queue_ms": p99(self.queue_waits), "p99_launch_wait_ms": p99(self.launch_waits),
            "p99_device_ms": p99(self.device_times),
            "requests": self.requests, "completed": self.completed, "rejected": self.rejected,
            "failed": self.failed, "cancelled": self.cancelled,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
            "gcells_s": self.cells / span / 1e9,
            "req_s": self.completed / span,
            "batches": self.batches,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "max_queue": self.max_queue, "peak_bytes": self.peak_bytes,
        }


class Server:
    """The scheduling loop.  executor: launch(batch, offsets) -> handle, done(handle) -> bool,
    finish(handle) -> [(side, row, col)], release(handle); slots: concurrent launches."""

    def __init__(self, executor, budget_bytes: int, slots: int = 4, max_batch: int = 512,
                 clock=None, on_complete=None):
        self.ex = executor
        self.arena = Arena(budget_bytes)
        self.slots = int(slots)
        self.max_batch = int(max_batch)
        self.clock = clock or WallClock()
        self.on_complete = on_complete

    def run(self, requests) -> Stats:
        """Serve `requests` (arrival times relative to the start of this call); the collector
        is paused meanwhile so that its pauses do not land in the latencies."""
        was_enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests)
        finally:
            if was_enabled:
                gc.enable()

    def _run(self, requests) -> Stats:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        st = Stats(requests=len(reqs))
        st.first_arrival = reqs[0].arrival if reqs else 0.0
        queue = collections.deque()   # arrived, not admitted (FIFO)
        pending = []        # admitted (memory held), not launched: [(req, bits_off, map_off)]
        inflight = []       # [(handle, [(req, bits_off, map_off)])]
        nxt = 0
        clk = self.clock

        def release_memory(items):
            for _, boff, moff in items:
                self.arena.free(boff)
                if moff is not None:
                    self.arena.free(moff)

        def fail(items, why):
            for r, _, _ in items:
                r.error = why
                st.failed += 1
            release_memory(items)

        while nxt < len(reqs) or queue or pending or inflight:
            now = clk.now()
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
            st.max_queue = max(st.max_queue, len(queue))
            # completions, in any order
            still = []
            device_error = None
            for k, (h, items) in enumerate(inflight):
                try:
                    finished = self.ex.done(h)
                except Exception as e:  # the device can no longer report: see below
                    device_error = "device error: %s" % e
                    still.extend(inflight[k:])
                    break
                if not finished:
                    still.append((h, items))
                    continue
                try:
                    res = self.ex.finish(h)
                except Exception as e:  # this batch's results are unusable
                    fail(items, "batch failed: %s" % e)
                    self.ex.release(h)
                    continue
                t = clk.now()
                for (r, boff, moff), rv in zip(items, res):
                    if r.cancelled:
                        r.error = "cancelled"
                        st.cancelled += 1
                        continue
                    r.done = t
                    r.result = tuple(int(v) for v in rv)
                    if self.on_complete:
                        self.on_complete(r, self.ex.map_view(h, r, moff))
                    st.completed += 1
                    st.cells += r.cells
                    st.latencies.append(r.done - r.arrival)
                    st.queue_waits.append(r.admitted - r.arrival)
                    st.launch_waits.append(r.launched - r.admitted)
                    st.device_times.append(r.done - r.launched)
                    st.last_done = max(st.last_done, t)
                release_memory(items)
                self.ex.release(h)
            if device_error is not None:
                # every request not yet served fails with the error, and nothing more is
                # launched: the batches still in flight, the admitted ones, the queue and the
                # arrivals to come
                for _, items in still:
                    fail(items, device_error)
                fail(pending, device_error)
                for r in list(queue) + reqs[nxt:]:
                    r.error = device_error
                    st.failed += 1
                return st
            inflight = still
            # admission: arrival order, while the budget holds the next request
            while queue and len(pending) < self.max_batch:
                r = queue[0]
                if r.cancelled:
                    queue.popleft()
                    r.error = "cancelled"
                    st.cancelled += 1
                    continue
                why = r.invalid()
                if why is None and r.device_bytes > self.arena.capacity:
                    why = "larger than the HBM budget"
                if why is not None:
                    queue.popleft()
                    r.error = why
                    st.rejected += 1
                    continue
                boff = self.arena.alloc(r.bits_bytes)
                if boff is None:
                    break
                moff = None
                if r.want_map:
                    moff = self.arena.alloc(r.map_bytes)
                    if moff is None:
                        self.arena.free(boff)
                        break
                queue.popleft()
                r.admitted = clk.now()
                pending.append((r, boff, moff))
            st.peak_bytes = max(st.peak_bytes, self.arena.in_use)
            # requests cancelled while admitted are dropped before launch
            if any(r.cancelled for r, _, _ in pending):
                gone = [x for x in pending if x[0].cancelled]
                pending = [x for x in pending if not x[0].cancelled]
                for r, _, _ in gone:
                    r.error = "cancelled"
                    st.cancelled += 1
                release_memory(gone)
            # launch everything admitted on a free slot
            if pending and len(inflight) < self.slots:
                t = clk.now()
                for r, _, _ in pending:
                    r.launched = t
                try:
                    h = self.ex.launch(pending)
                except Exception as e:  # only this batch fails; its memory returns
                    fail(pending, "launch failed: %s" % e)
                    pending = []
                    continue
                inflight.append((h, pending))
                st.batches += 1
                st.batch_sizes.append(len(pending))
                pending = []
                continue
            # nothing to do right now: wait for the next arrival (or poll the device)
            if nxt < len(reqs) and not inflight and not pending:
                clk.wait(reqs[nxt].arrival)
            elif inflight:
                clk.wait(min(reqs[nxt].arrival if nxt < len(reqs) else float("inf"),
                             clk.now() + 2e-5))
        return st


class GpuExecutor:
    """Runs batches through the library on `slots` streams of one device.  One ms_ctx per
    slot (contexts keep a small scratch that concurrent calls must not share).  The device
    arena is one allocation of `budget_bytes`; request bits are copied into it from pinned
    host memory, and maps are written into it."""

    def __init__(self, budget_bytes: int, slots: int = 4, max_batch: int = 512,
                 max_n: int = 8192, device: int = 0, plain: bool = False):
        """plain: one ms_max_square launch pair per request instead of the batched call (the
        one-launch-per-matrix baseline)."""
        import torch
        self.plain = bool(plain)
        from . import Context, lib, _Matrix, ms_batched_workspace_size
        self.torch = torch
        self.L = lib()
        self.dev = torch.device("cuda", device)
        self.arena = torch.empty(int(budget_bytes) // ALIGN * ALIGN, dtype=torch.uint8,
                                 device=self.dev)
        self.base = self.arena.data_ptr()
        self.slots = []
        self.max_batch = int(max_batch)
        msz = ctypes.sizeof(_Matrix)
        self._Matrix = _Matrix
        # the workspace bound: every matrix as large as the widest allowed
        probe = (_Matrix * self.max_batch)()
        for i in range(self.max_batch):
            probe[i] = _Matrix(1, max_n, max_n, (max_n + 63) // 64)
        ws_bytes = ms_batched_workspace_size(None, probe, self.max_batch)
        from . import ms_set_batched_graphs, GRAPHS_OFF
        for _ in range(int(slots)):
            ctx = Context(device)
            # a slot's buffers are reused by batches of the same shapes now and then: no graph
            # capture (or eviction, which waits for the device) inside a request's latency
            ms_set_batched_graphs(ctx.handle, GRAPHS_OFF)
            self.slots.append({
                "ctx": ctx,
                "stream": torch.cuda.Stream(device=self.dev),
                "d_mats": torch.empty(self.max_batch * msz, dtype=torch.uint8, device=self.dev),
                "h_mats": (_Matrix * self.max_batch)(),
                "h_mats_pinned": torch.empty(self.max_batch * msz, dtype=torch.uint8,
                                             pin_memory=True),
                "d_out": torch.empty((self.max_batch, 3), dtype=torch.int64, device=self.dev),
                "h_out": torch.empty((self.max_batch, 3), dtype=torch.int64, pin_memory=True),
                "ws": torch.empty(ws_bytes, dtype=torch.uint8, device=self.dev),
                "ws_bytes": ws_bytes,
                "event": torch.cuda.Event(),
                "busy": False,
            })
        # Size every slot context's scratch for the largest admissible request now (one search
        # over an all-zeros max_n x max_n matrix): a context grows its scratch on demand, and
        # growing waits for the whole device, which would land in some request's latency.
        zero = torch.zeros((int(max_n), (int(max_n) + 63) // 64), dtype=torch.int64,
                           device=self.dev)
        res = torch.empty(3, dtype=torch.int64, device=self.dev)
        for slot in self.slots:
            rc = self.L.ms_max_square(slot["ctx"].handle, zero.data_ptr(), int(max_n), int(max_n),
                                      zero.stride(0), res.data_ptr(), slot["stream"].cuda_stream)
            if rc:
                raise RuntimeError("ms_max_square failed while sizing a slot: %d" % rc)
        torch.cuda.synchronize(self.dev)
        del zero, res

    def host_bits(self, bits):
        """Pinned host copy of a packed matrix (int64 view), for asynchronous uploads."""
        t = self.torch.from_numpy(np.ascontiguousarray(bits).view(np.int64))
        return t.pin_memory()

    def launch(self, batch):
        """Enqueue a batch on a free slot.  On failure the slot's stream is drained (so no copy
        into the batch's arena memory is still pending when the server frees it), the slot is
        freed, and the error is raised for the server to fail this batch alone."""
        slot = next(s for s in self.slots if not s["busy"])
        slot["busy"] = True
        try:
            if len(batch) > self.max_batch:
                raise ValueError("batch larger than the executor's max_batch")
            return self._enqueue(slot, batch)
        except Exception:
            slot["stream"].synchronize()
            slot["busy"] = False
            raise

    def _enqueue(self, slot, batch):
        torch = self.torch
        st = slot["stream"]
        sp = st.cuda_stream
        h = slot["h_mats"]
        with torch.cuda.stream(st):
            for i, (r, boff, moff) in enumerate(batch):
                nb = int(r.m) * r.ld_words * 8
                src = r.bits if isinstance(r.bits, torch.Tensor) else self.host_bits(r.bits)
                if nb:
                    self.arena[boff:boff + nb].copy_(src.view(-1).view(torch.uint8)[:nb],
                                                     non_blocking=True)
                h[i] = self._Matrix(self.base + boff, r.m, r.n, r.ld_words)
            count = len(batch)
            raw = ctypes.string_at(ctypes.addressof(h), ctypes.sizeof(self._Matrix) * count)
            slot["h_mats_pinned"][:len(raw)].copy_(torch.frombuffer(bytearray(raw),
                                                                     dtype=torch.uint8))
            slot["d_mats"][:len(raw)].copy_(slot["h_mats_pinned"][:len(raw)], non_blocking=True)
            ctx = slot["ctx"].handle
            if self.plain:
                for i, (r, boff, moff) in enumerate(batch):
                    rc = self.L.ms_max_square(ctx, self.base + boff, r.m, r.n, r.ld_words,
                                              slot["d_out"][i].data_ptr(), sp)
                    if rc:
                        raise RuntimeError("ms_max_square failed: %d" % rc)
            else:
                rc = self.L.ms_max_square_batched(ctx, h, slot["d_mats"].data_ptr(), count,
                                                  slot["d_out"].data_ptr(), slot["ws"].data_ptr(),
                                                  slot["ws_bytes"], sp)
                if rc:
                    raise RuntimeError("ms_max_square_batched failed: %d" % rc)
            for i, (r, boff, moff) in enumerate(batch):
                if moff is not None and r.cells:
                    rc = self.L.ms_square_map_from_max(ctx, self.base + boff, r.m, r.n, r.ld_words,
                                                       slot["d_out"][i].data_ptr(),
                                                       self.base + moff, r.n, sp)
                    if rc:
                        raise RuntimeError("ms_square_map_from_max failed: %d" % rc)
            slot["h_out"][:count].copy_(slot["d_out"][:count], non_blocking=True)
            slot["event"].record(st)
        slot["count"] = count
        return slot

    def done(self, slot) -> bool:
        return slot["event"].query()

    def finish(self, slot):
        rows = slot["h_out"][:slot["count"]].tolist()
        if any(r[0] < 0 for r in rows):
            raise RuntimeError("batched call reported an inconsistent batch")
        return rows

    def map_view(self, slot, r, moff):
        """The request's dp map as an int32 (m, n) device view; valid until its memory is
        freed right after the completion callback returns."""
        if moff is None:
            return None
        nb = int(r.m) * int(r.n) * 4
        return self.arena[moff:moff + nb].view(self.torch.int32).view(int(r.m), int(r.n))

    def release(self, slot):
        slot["busy"] = False

    def close(self):
        self.torch.cuda.synchronize(self.dev)
        for s in self.slots:
            s["ctx"].close()


def poisson_arrivals(count: int, rate: float, seed) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson client: exponential gaps of mean
    1 / rate from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=int(count)))


def make_requests(pool, count: int, rate: float, map_fraction: float = 0.1, seed=None):
    """count requests cycling through `pool` ([(bits, m, n), ...]), Poisson arrivals at
    `rate`, each wanting its map with probability map_fraction."""
    seed = [30000, int(rate)] if seed is None else seed
    arr = poisson_arrivals(count, rate, seed)
    rng = np.random.default_rng([30002, int(rate)])
    want = rng.random(count) < map_fraction
    out = []
    for k in range(count):
        bits, m, n = pool[k % len(pool)]
        out.append(Request(rid=k, m=m, n=n, bits=bits, arrival=float(arr[k]),
                           want_map=bool(want[k])))
    return out
