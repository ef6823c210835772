"""Serving scheduler on the CPU: a fake backend with a manual clock.

Checks admission by memory and slots, FIFO admission order, routing of big
requests to the single-stream path, continuous batching (requests arriving
while batches are in flight join later batches that overlap them), pool
accounting, rejection of requests larger than the pool and the latency
bookkeeping.  Results come from the oracle, so each request's answer is also
checked against its own computation.
"""
import numpy as np
import pytest

from paper_1405_0562_amd.serve import FakeBackend, PoolAllocator, Server
import workloads as W
from oracle.automata import compile_regex
from oracle import scan as oscan


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


REGEXES = [W.REGEX_C1, W.REGEX_C2, ".*abc.*"]
DFAS = [compile_regex(rx) for rx in REGEXES]


def oracle_result(r):
    d = DFAS[r.table]
    q = oscan.scan(d, r.data)
    return (q, int(d.accept[q]))


def make_server(clock, pool=1 << 20, **kw):
    backend = FakeBackend(clock, oracle_result, service_time=lambda nb: 0.010 + nb / 1e8)
    return Server(backend, pool_bytes=pool, clock=clock, **kw), backend


def test_pool_allocator_first_fit_and_merge():
    p = PoolAllocator(4096)
    a = p.alloc(1000)
    b = p.alloc(1000)
    c = p.alloc(2000)
    assert (a, b) == (0, 1024) and c == 2048 and p.alloc(1) is None
    p.release(b, 1000)
    assert p.alloc(1024) == 1024
    p.release(a, 1000)
    p.release(1024, 1024)
    p.release(c, 2000)
    assert p.free == [(0, 4096)] and p.used == 0


def test_admission_respects_memory_slots_and_order():
    clock = Clock()
    srv, be = make_server(clock, pool=64 * 1024, max_inflight=2, max_batch_requests=8)
    rng = np.random.default_rng(0)
    reqs = [srv.submit(i % 3, rng.integers(97, 100, size=5000).astype(np.uint8)) for i in range(40)]
    peak = 0
    while not srv.idle:
        srv.step()
        assert len(srv.inflight) <= 2
        assert srv.pool.used <= srv.pool.capacity
        peak = max(peak, srv.pool.used)
        for L in srv.inflight:
            assert len(L.requests) <= 8
        clock.t += 0.003
    admitted = [r.rid for r in sorted(reqs, key=lambda r: (r.admitted, r.rid))]
    assert admitted == list(range(40))                       # FIFO admission
    assert all(r.result == oracle_result(r) for r in reqs)
    assert peak > 0 and srv.pool.used == 0


def test_big_requests_go_alone_and_small_ones_batch():
    clock = Clock()
    srv, be = make_server(clock, pool=1 << 22, big_bytes=100_000)
    srv.submit(0, np.zeros(10, np.uint8))
    srv.submit(1, np.full(200_000, ord("a"), np.uint8))
    srv.submit(2, np.zeros(20, np.uint8))
    srv.submit(2, np.zeros(30, np.uint8))
    srv.step()
    kinds = [(h["big"], len(h["req"])) for h in be.launches]
    assert kinds == [(False, 1), (True, 1), (False, 2)]
    while not srv.idle:
        clock.t += 0.01
        srv.step()
    assert all(r.result == oracle_result(r) for r in srv.finished)


def test_unbatchable_tables_go_alone():
    # a table the batch kernel does not take (no stride-1 image, or an
    # on-the-fly D-SFA) is matched alone, in arrival order with the rest
    clock = Clock()
    backend = FakeBackend(clock, oracle_result, service_time=lambda nb: 0.010 + nb / 1e8, unbatchable={1})
    srv = Server(backend, pool_bytes=1 << 22, max_inflight=8, clock=clock)
    for t in (0, 2, 1, 0, 2):
        srv.submit(t, np.zeros(16, np.uint8))
    srv.step()
    kinds = [(h["big"], [r.table for r in h["req"]]) for h in backend.launches]
    assert kinds == [(False, [0, 2]), (True, [1]), (False, [0, 2])]
    while not srv.idle:
        clock.t += 0.01
        srv.step()
    assert all(r.result == oracle_result(r) for r in srv.finished)


def test_continuous_batching_overlaps_arrivals():
    clock = Clock()
    srv, be = make_server(clock, pool=1 << 22, max_inflight=4)
    arrivals = [(0.001 * i, i % 3, np.full(1000 + i, ord("a") + i % 3, np.uint8)) for i in range(50)]
    # drive time by hand: submit arrivals as the clock passes them
    i = 0
    while i < len(arrivals) or not srv.idle:
        while i < len(arrivals) and arrivals[i][0] <= clock.t:
            srv.submit(arrivals[i][1], arrivals[i][2], arrival=arrivals[i][0])
            i += 1
        srv.step()
        clock.t += 0.0005
    assert len(srv.finished) == 50
    assert srv.n_launches > 3                                  # arrivals spread over several batches
    overlapped = any(a["t"] > b["t"] - 0.010 and a is not b for a in be.launches for b in be.launches)
    assert overlapped
    st = srv.latency_stats()
    assert st["n"] == 50 and 0 < st["p50_ms"] <= st["p99_ms"]
    assert all(r.done >= r.arrival for r in srv.finished)
    assert all(r.result == oracle_result(r) for r in srv.finished)


def test_too_large_requests_are_rejected():
    clock = Clock()
    srv, _ = make_server(clock, pool=4096)
    r = srv.submit(0, np.zeros(10_000, np.uint8))
    assert r in srv.rejected and srv.idle
    assert srv.latency_stats()["n"] == 0


def test_same_result_alone_and_in_the_mix():
    clock = Clock()
    rng = np.random.default_rng(3)
    datas = [rng.choice(np.frombuffer(b"abc0", np.uint8), size=rng.integers(0, 3000)) for _ in range(30)]
    alone = []
    for i, d in enumerate(datas):
        srv, _ = make_server(clock)
        srv.submit(i % 3, d)
        while not srv.idle:
            clock.t += 0.01
            srv.step()
        alone.append(srv.finished[0].result)
    srv, _ = make_server(clock, max_batch_requests=7)
    reqs = [srv.submit(i % 3, d) for i, d in enumerate(datas)]
    while not srv.idle:
        clock.t += 0.01
        srv.step()
    assert [r.result for r in reqs] == alone
