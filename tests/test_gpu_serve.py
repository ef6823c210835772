"""GPU serving: continuous batching over 16 resident tables.

Every request's result in the served mix must equal the oracle and the same
request matched alone through the plain single-stream path.
"""
import functools

import numpy as np
import pytest

import workloads as W
from oracle.automata import compile_regex
from oracle import scan as oscan

pytestmark = pytest.mark.gpu

sfa = pytest.importorskip("paper_1405_0562_amd")
from paper_1405_0562_amd.serve import GpuBackend, PlainBackend, Server, run_open_loop  # noqa: E402


@functools.lru_cache(maxsize=None)
def oracle_dfa(rx):
    d = compile_regex(rx)
    return d, oscan.table_u32(d)


def test_served_results_equal_alone_and_oracle():
    regexes = W.c5_regexes(0)
    tables = [sfa.load(sfa.compile(rx)) for rx in regexes]
    reqs = W.c5_requests(1, n_req=150, qps=20000.0, max_len=1 << 20)
    # two requests above the big-request threshold go through the single-stream path
    big = W.uniform_over(W.rng_for(2, 7), W.ALPHABET_C4, 3 << 20)
    arrivals = [(r.arrival_s, r.table, r.data) for r in reqs] + [(0.001, 3, big), (0.002, 5, big[: (2 << 20) + 7])]
    backend = GpuBackend(tables, pool_bytes=64 << 20, n_streams=3)
    srv = Server(backend, pool_bytes=64 << 20, max_inflight=3, big_bytes=1 << 20)
    print("[gpu-case] serve", len(arrivals), "requests", flush=True)
    served = run_open_loop(srv, arrivals)
    assert len(srv.finished) == len(arrivals) and not srv.rejected
    assert any(len(L) for L in [srv.finished])
    plain = PlainBackend(tables)
    for r in served:
        d, tab = oracle_dfa(regexes[r.table])
        q = oscan.scan(d, r.data, table=tab)
        assert r.result == (q, int(d.accept[q])), r.rid
        assert r.result == plain.run_one(r), r.rid
    st = srv.latency_stats()
    assert st["n"] == len(arrivals) and st["p99_ms"] >= st["p50_ms"] > 0
    assert srv.n_launches < len(arrivals)            # requests were batched


def test_tables_without_batch_image_are_served_alone():
    """A large keyword D-SFA (global-table walk, no stride-1 image) and an
    on-the-fly D-SFA served beside batchable tables: their requests go
    through the single-stream matcher, every result equals the oracle."""
    regexes = W.c5_regexes(0)[:6]
    kws = W.c3_keywords(0)
    big_rx = W.c3_regex(kws)
    lazy_rx = W.c3_regex(W.c3_keywords(1, count=60))
    sample = W.c3_input(3, 1 << 18, kws, rate=1e-4)
    tables = [sfa.load(sfa.compile(rx)) for rx in regexes]
    tables.append(sfa.load(sfa.compile(big_rx), profile_sample=sample))
    tables.append(sfa.load(sfa.compile(lazy_rx, sfa_cap=0).build_lazy(sample), profile_sample=sample))
    all_rx = regexes + [big_rx, lazy_rx]
    backend = GpuBackend(tables, pool_bytes=64 << 20, n_streams=3)
    assert not backend.batchable(6) and not backend.batchable(7) and backend.batchable(0)
    rng = np.random.default_rng(4)
    arrivals = []
    for i in range(120):
        t = int(rng.integers(0, len(tables)))
        n = int(rng.integers(0, 40_000))
        data = (W.c3_input(100 + i, n, kws, rate=1e-3) if t >= 6 else
                W.uniform_over(W.rng_for(100 + i, 7), W.ALPHABET_C4, n))
        arrivals.append((0.0002 * i, t, data))
    srv = Server(backend, pool_bytes=64 << 20, max_inflight=3, big_bytes=1 << 20)
    print("[gpu-case] serve with unbatchable tables", len(arrivals), "requests", flush=True)
    served = run_open_loop(srv, arrivals)
    assert len(srv.finished) == len(arrivals) and not srv.rejected
    for r in served:
        d, tab = oracle_dfa(all_rx[r.table])
        q = oscan.scan(d, r.data, table=tab)
        assert r.result == (q, int(d.accept[q])), (r.rid, r.table)
