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
