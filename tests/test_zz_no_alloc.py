"""sfa_match_noalloc (the entry point with the library's own workspace)
against sfa_match with a caller workspace, through the C ABI: two calls in
a row on each table, the second with a smaller input, each result also
equal to the oracle's; and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle.automata import compile_regex
from oracle import scan as oscan

pytestmark = pytest.mark.gpu

sfa = pytest.importorskip("paper_1405_0562_amd")


def oracle_result(rx, data):
    d = compile_regex(rx)
    q = oscan.scan(d, data)
    return [q, int(d.accept[q])]


def both(t, x, n_chunks=0):
    """(sfa_match with its own workspace, sfa_match_noalloc), each synchronised."""
    L = sfa.lib()
    n = x.numel()
    need = ctypes.c_size_t()
    assert L.sfa_match_workspace_bytes(t.handle, n, n_chunks, ctypes.byref(need)) == 0
    ws = torch.zeros(max(need.value, 4096), dtype=torch.uint8, device="cuda")
    a = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    b = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.sfa_match(t.handle, x.data_ptr() if n else None, n, n_chunks, ws.data_ptr(), ws.numel(),
                       a.data_ptr(), s) == 0
    st = L.sfa_match_noalloc(t.handle, x.data_ptr() if n else None, n, n_chunks, b.data_ptr(), s)
    assert st == 0, L.sfa_last_error()
    torch.cuda.synchronize()
    return a.tolist(), b.tolist()


def c3_small(seed, n):
    kws = W.c3_keywords(seed)
    return W.c3_regex(kws), W.c3_input(seed, n, kws, rate=3e-6)


CASES = [
    ("c2", lambda n: (W.REGEX_C2, W.c2_input(1, n)), (1 << 24) + 5, 300_001, 4096),
    ("c1", lambda n: (W.REGEX_C1, W.c1_input(2, n)), 1_048_570, 65_536, 256),
    ("c3", lambda n: c3_small(3, n), (1 << 24) + 3, 1_000_003, 0),
]


@pytest.mark.parametrize("name,make,n_big,n_small,n_chunks", CASES)
def test_noalloc_matches_caller_workspace(name, make, n_big, n_small, n_chunks):
    print("[gpu-case] noalloc", name, n_big, n_small, n_chunks, flush=True)
    rx, big = make(n_big)
    t = sfa.load(sfa.compile(rx))
    xb = torch.from_numpy(big).cuda()
    want = oracle_result(rx, big)
    a, b = both(t, xb, n_chunks)
    assert a == b == want
    # second call, smaller input, from an unaligned base
    small = big[7:7 + n_small]
    xs = torch.from_numpy(small.copy()).cuda()
    want2 = oracle_result(rx, small)
    a2, b2 = both(t, xs, 0)
    assert a2 == b2 == want2
    a3, b3 = both(t, xb[7:7 + n_small], n_chunks)
    assert a3 == b3 == want2


def test_noalloc_rejects_plans_over_its_workspace():
    rx, data = c3_small(4, 1 << 16)
    t = sfa.load(sfa.compile(rx))
    x = torch.from_numpy(data).cuda()
    L = sfa.lib()
    out = torch.empty(2, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    # 2^24 chunks over a 136-state DFA need about 9 MB of block mappings
    assert L.sfa_match_noalloc(t.handle, x.data_ptr(), x.numel(), 1 << 24, out.data_ptr(), s) == 1
    assert b"workspace" in L.sfa_last_error()
    # the library's workspace still works afterwards
    assert L.sfa_match_noalloc(t.handle, x.data_ptr(), x.numel(), 0, out.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert out.tolist() == oracle_result(rx, data)
