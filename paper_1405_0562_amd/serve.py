"""Serving form: continuous batching of match requests over resident tables.

Requests (table index, bytes) arrive at any time.  ``Server.step()`` is the
scheduler loop body:

1. completion: batches whose device event has fired publish their results
   and give their memory back;
2. admission: waiting requests are admitted in arrival order while the
   device memory pool can hold their bytes and a batch slot is free
   (memory-admitted continuous batching: requests that arrive while earlier
   batches run join the next batch, which overlaps with them on the device);
3. launch: admitted requests form one batch (one job per request) launched on
   the next stream; requests of at least ``big_bytes``, and requests for a
   table the batch kernel does not take (``backend.batchable``: no stride-1
   walk image, e.g. a large or on-the-fly D-SFA), go alone through the
   single-stream matcher instead, which splits them over the whole GPU.

The backend owns device work; ``GpuBackend`` drives libsfa.so, the CPU
``FakeBackend`` (tests) simulates completion times with a caller's clock so
that admission, ordering and latency bookkeeping can be checked without a GPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    table: int
    data: np.ndarray
    arrival: float
    admitted: float = -1.0
    done: float = -1.0
    result: tuple | None = None

    @property
    def nbytes(self) -> int:
        return int(self.data.size)


class PoolAllocator:
    """First-fit allocator over [0, capacity) with 256-byte granularity."""

    def __init__(self, capacity: int, align: int = 256):
        self.capacity = capacity
        self.align = align
        self.free = [(0, capacity)]          # sorted (offset, size)
        self.used = 0

    def _round(self, n: int) -> int:
        return max(self.align, (n + self.align - 1) // self.align * self.align)

    def alloc(self, n: int) -> int | None:
        n = self._round(n)
        for i, (off, size) in enumerate(self.free):
            if size >= n:
                if size == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, size - n)
                self.used += n
                return off
        return None

    def release(self, off: int, n: int) -> None:
        n = self._round(n)
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged


@dataclass
class Launch:
    requests: list
    offset: int
    nbytes: int
    handle: object = None
    big: bool = False


class Server:
    """Continuous-batching scheduler (backend-agnostic)."""

    def __init__(self, backend, pool_bytes: int = 1 << 30, max_batch_requests: int = 4096,
                 max_inflight: int = 4, big_bytes: int = 8 << 20, clock=time.perf_counter):
        self.backend = backend
        self.pool = PoolAllocator(pool_bytes)
        self.max_batch = max_batch_requests
        self.max_inflight = max_inflight
        self.big_bytes = big_bytes
        self.clock = clock
        self.waiting: collections.deque = collections.deque()
        self.inflight: list[Launch] = []
        self.finished: list[Request] = []
        self.rejected: list[Request] = []
        self.n_launches = 0
        self._rid = 0

    # -- client side ------------------------------------------------------
    def submit(self, table: int, data: np.ndarray, arrival: float | None = None) -> Request:
        r = Request(self._rid, int(table), np.ascontiguousarray(data, dtype=np.uint8),
                    self.clock() if arrival is None else arrival)
        self._rid += 1
        if r.nbytes > self.pool.capacity:
            r.done = r.arrival
            self.rejected.append(r)
        else:
            self.waiting.append(r)
        return r

    @property
    def idle(self) -> bool:
        return not self.waiting and not self.inflight

    # -- scheduler --------------------------------------------------------
    def _complete(self) -> int:
        n = 0
        still = []
        for L in self.inflight:
            if self.backend.done(L.handle):
                now = self.clock()
                results = self.backend.results(L.handle)
                for r, res in zip(L.requests, results):
                    r.result = (int(res[0]), int(res[1]))
                    r.done = now
                    self.finished.append(r)
                self.pool.release(L.offset, L.nbytes)
                n += 1
            else:
                still.append(L)
        self.inflight = still
        return n

    def _admit_and_launch(self) -> int:
        launched = 0
        while self.waiting and len(self.inflight) < self.max_inflight:
            head = self.waiting[0]
            if head.nbytes >= self.big_bytes or not self._batchable(head):
                off = self.pool.alloc(head.nbytes)
                if off is None:
                    break
                self.waiting.popleft()
                head.admitted = self.clock()
                L = Launch([head], off, head.nbytes, big=True)
                L.handle = self.backend.launch_single(head, off)
            else:
                batch, total = [], 0
                for r in self.waiting:
                    if r.nbytes >= self.big_bytes or len(batch) >= self.max_batch or not self._batchable(r):
                        break
                    batch.append(r)
                    total += r.nbytes
                # shrink until the pool can hold the batch
                off = self.pool.alloc(total)
                while off is None and len(batch) > 1:
                    total -= batch.pop().nbytes
                    off = self.pool.alloc(total)
                if off is None:
                    break
                now = self.clock()
                for _ in batch:
                    r = self.waiting.popleft()
                    r.admitted = now
                L = Launch(batch, off, total)
                L.handle = self.backend.launch_batch(batch, off)
            self.inflight.append(L)
            self.n_launches += 1
            launched += 1
        return launched

    def _batchable(self, r: Request) -> bool:
        fn = getattr(self.backend, "batchable", None)
        return True if fn is None else bool(fn(r.table))

    def step(self) -> tuple[int, int]:
        """One scheduler pass: (batches completed, batches launched)."""
        done = self._complete()
        launched = self._admit_and_launch()
        return done, launched

    def drain(self, poll_sleep: float = 0.0) -> None:
        while not self.idle:
            self.step()
            if poll_sleep:
                time.sleep(poll_sleep)

    # -- reporting --------------------------------------------------------
    def latency_stats(self) -> dict:
        lat = np.array([r.done - r.arrival for r in self.finished], dtype=np.float64)
        nbytes = sum(r.nbytes for r in self.finished)
        if lat.size == 0:
            return {"n": 0}
        t0 = min(r.arrival for r in self.finished)
        t1 = max(r.done for r in self.finished)
        return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "bytes": int(nbytes), "makespan_s": float(t1 - t0),
                "gbs": float(nbytes / max(1e-9, t1 - t0) / 1e9), "launches": self.n_launches,
                "rejected": len(self.rejected)}


class GpuBackend:
    """Device side of the server: pinned staging, device pool, batch and single launches."""

    def __init__(self, tables, pool_bytes: int = 1 << 30, n_streams: int = 3, piece_bytes: int = 4096,
                 units_per_lane: int = 2, device=None, max_batch_requests: int = 4096, result_slots: int = 64,
                 ws_bytes: int = 32 << 20, warmup: bool = True, warmup_max_bytes: int = 64 << 20,
                 direct_bytes: int = 1 << 20):
        import torch
        from .batch import Batch, BatchOptions
        self.torch = torch
        self.Batch, self.BatchOptions = Batch, BatchOptions
        self.tables = list(tables)
        self.device = self.tables[0].device if device is None else device
        # the batch plan takes the tables with a stride-1 walk image; requests
        # for the others are matched alone
        self._batch_ids = {}
        for i, t in enumerate(self.tables):
            if t.info["strides"] & 2 and not t.info["partial"]:
                self._batch_ids[i] = len(self._batch_ids)
        self.batch_tables = [t for i, t in enumerate(self.tables) if i in self._batch_ids]
        self.dev_pool = torch.empty(pool_bytes, dtype=torch.uint8, device=self.device)
        self.host_pool = torch.empty(pool_bytes, dtype=torch.uint8, pin_memory=True)
        self.host_np = self.host_pool.numpy()
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.next_stream = 0
        self.options = BatchOptions(piece_bytes, units_per_lane)
        self.piece_bytes, self.units_per_lane = piece_bytes, units_per_lane
        # pinned result slots, reused round robin (more slots than batches in flight)
        self.result_slots = [torch.empty((max_batch_requests, 2), dtype=torch.int32, pin_memory=True)
                             for _ in range(result_slots)]
        self.next_slot = 0
        # batch workspace and output per stream: launches on one stream run
        # in order, so they share them, and serving allocates nothing
        self.max_batch_requests = max_batch_requests
        self.warmup_max_bytes = warmup_max_bytes
        self.direct_bytes = direct_bytes
        self.stream_ws = [torch.empty(ws_bytes, dtype=torch.uint8, device=self.device) for _ in self.streams]
        self.stream_out = [torch.empty((max_batch_requests, 2), dtype=torch.int32, device=self.device)
                           for _ in self.streams]
        if warmup:
            self.warmup()

    def warmup(self) -> None:
        """Run the launch paths before serving: every table alone at sizes
        from 4 KiB to the largest request the pool holds (the matcher picks
        different kernels and workspaces by size) and a batch over all tables
        on every stream.  First launches load kernel code, set kernel
        attributes and grow the allocator's cache, which would otherwise land
        on the first requests served."""
        cap = min(self.dev_pool.numel(), self.warmup_max_bytes)
        sizes = [4096, 1 << 20]
        while sizes[-1] * 8 <= cap:
            sizes.append(sizes[-1] * 8)
        blanks = [np.zeros(n, dtype=np.uint8) for n in sizes]
        for t in range(len(self.tables)):
            for x in blanks:
                self.launch_single(Request(-1, t, x, 0.0), 0)[0].synchronize()
        small = np.zeros(4096, dtype=np.uint8)
        for _ in self.streams:
            reqs = [Request(-1, t, small, 0.0) for t in self._batch_ids]
            if len(reqs) >= 2:
                self.launch_batch(reqs, 0)[0].synchronize()
        self.torch.cuda.synchronize(self.device)

    def _stream(self):
        i = self.next_stream % len(self.streams)
        self.next_stream += 1
        return i, self.streams[i]

    def _stage(self, requests, off, stream):
        """Copies the requests' bytes to dev_pool[off:] on `stream`: small
        ones through the pinned pool (one host copy, then one asynchronous
        transfer for all of them), requests of at least ``direct_bytes``
        straight from their own memory (one transfer, no host copy)."""
        cur = off
        run = off   # start of the pending run of small requests in the pinned pool
        with self.torch.cuda.stream(stream):
            for r in requests:
                if r.nbytes >= self.direct_bytes:
                    if cur > run:
                        self.dev_pool[run:cur].copy_(self.host_pool[run:cur], non_blocking=True)
                    self.dev_pool[cur:cur + r.nbytes].copy_(self.torch.from_numpy(r.data), non_blocking=True)
                    cur += r.nbytes
                    run = cur
                else:
                    self.host_np[cur:cur + r.nbytes] = r.data
                    cur += r.nbytes
            if cur > run:
                self.dev_pool[run:cur].copy_(self.host_pool[run:cur], non_blocking=True)
        return cur - off

    def _slot(self, n):
        buf = self.result_slots[self.next_slot % len(self.result_slots)]
        self.next_slot += 1
        return buf[:n]

    def batchable(self, table: int) -> bool:
        return table in self._batch_ids

    def _options(self, total: int):
        """Piece length for a batch of `total` bytes: a lane walks a piece one
        byte after another, so a small batch is cut finer (about 16K pieces
        per batch, 256 B to piece_bytes) and ends sooner."""
        piece = 256
        while piece < self.piece_bytes and piece * 2 * 16384 <= total:
            piece *= 2
        return self.BatchOptions(piece, self.units_per_lane)

    def launch_batch(self, requests, off):
        torch = self.torch
        if len(requests) == 1:
            return self.launch_single(requests[0], off)
        i, s = self._stream()
        total = self._stage(requests, off, s)
        lens = np.array([r.nbytes for r in requests], dtype=np.int64)
        doc_off = np.zeros(len(requests) + 1, dtype=np.int64)
        np.cumsum(lens, out=doc_off[1:])
        jobs = np.stack([np.arange(len(requests)), [self._batch_ids[r.table] for r in requests]],
                        axis=1).astype(np.uint32)
        with torch.cuda.stream(s):
            b = self.Batch(self.batch_tables, doc_off, jobs, self._options(total), stream=s, ws=self.stream_ws[i],
                           out=self.stream_out[i])
            if b.ws is not self.stream_ws[i]:
                self.stream_ws[i] = b.ws   # grown once for a larger plan, kept for the next ones
            data = self.dev_pool[off:off + max(total, 1)]
            out = b.run(data, stream=s)
            host_out = self._slot(len(requests))
            host_out.copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, host_out, b)

    def launch_single(self, request, off):
        torch = self.torch
        from .matcher import match
        _, s = self._stream()
        self._stage([request], off, s)
        with torch.cuda.stream(s):
            data = self.dev_pool[off:off + request.nbytes]
            out = match(self.tables[request.table], data, stream=s)
            host_out = self._slot(1)
            host_out.copy_(out.view(1, 2), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, host_out, out)

    def done(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        return handle[1].numpy().tolist()


# The server keeps at most max_inflight launches in flight; result slots are
# reused round robin, so GpuBackend needs result_slots > max_inflight.


class PlainBackend:
    """The plain path: one request at a time through sfa_match on one stream."""

    def __init__(self, tables, device=None):
        import torch
        self.torch = torch
        self.tables = list(tables)
        self.device = self.tables[0].device if device is None else device

    def run_one(self, request) -> tuple:
        from .matcher import match
        x = self.torch.from_numpy(request.data).to(self.device, non_blocking=False)
        return tuple(match(self.tables[request.table], x).tolist())


class FakeBackend:
    """CPU stand-in for tests: results from a callable, completion after a
    simulated service time measured on the caller's clock."""

    def __init__(self, clock, result_fn, service_time=lambda nbytes: 1e-3 + nbytes / 1e9, unbatchable=()):
        self.clock = clock
        self.result_fn = result_fn
        self.service_time = service_time
        self.launches = []
        self.unbatchable = set(unbatchable)

    def batchable(self, table: int) -> bool:
        return table not in self.unbatchable

    def _launch(self, requests, big):
        t_done = self.clock() + self.service_time(sum(r.nbytes for r in requests))
        h = {"t": t_done, "req": list(requests), "big": big}
        self.launches.append(h)
        return h

    def launch_batch(self, requests, off):
        return self._launch(requests, False)

    def launch_single(self, request, off):
        return self._launch([request], True)

    def done(self, handle) -> bool:
        return self.clock() >= handle["t"]

    def results(self, handle):
        return [self.result_fn(r) for r in handle["req"]]


def run_open_loop(server: Server, arrivals, clock=time.perf_counter, spin: float = 0.0):
    """Submit (arrival_s, table, data) triples at their times (relative to
    now) while stepping the scheduler; returns when all are finished."""
    t0 = clock()
    arrivals = sorted(arrivals, key=lambda a: a[0])
    i = 0
    reqs = []
    while i < len(arrivals) or not server.idle:
        now = clock() - t0
        while i < len(arrivals) and arrivals[i][0] <= now:
            a = arrivals[i]
            reqs.append(server.submit(a[1], a[2], arrival=t0 + a[0]))
            i += 1
        server.step()
        if spin:
            time.sleep(spin)
    return reqs
