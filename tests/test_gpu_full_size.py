"""GPU parity at the full sizes of the 4 GiB single-stream workloads.

The keyword workload (20 seeded 8-letter keywords, 4 GiB of text over a-z
and space) and the (a|b)*a(a|b){4} workload at 2^32 + 13 bytes from an
unaligned base, each in the launch configuration the benchmark times
(library-chosen chunks), compared bit for bit with the oracle's Algorithm 2
in C over the same bytes.  These inputs put byte offsets past 2^32 and use
the grid composition with 131,072 chunks.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.automata import compile_regex
from oracle import scan as oscan

pytestmark = pytest.mark.gpu

sfa = pytest.importorskip("paper_1405_0562_amd")

N4G = 1 << 32


def say(*a):
    print("[gpu-case]", *a, flush=True)


def oracle_result(rx, data):
    d = compile_regex(rx)
    q = oscan.scan(d, data, table=oscan.table_u32(d))
    return [q, int(d.accept[q])]


def to_device(data: np.ndarray, offset: int = 0) -> torch.Tensor:
    buf = torch.empty(data.size + offset + 16, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + data.size]
    view.copy_(torch.from_numpy(data))
    return view


@pytest.mark.parametrize("seed,rate", [(0, 1e-6), (1, 0.0)])
def test_c3_keywords_4gib(seed, rate):
    kws = W.c3_keywords(seed)
    rx = W.c3_regex(kws)
    say("c3 4GiB seed", seed, "rate", rate, "generating")
    data = W.c3_input(seed, N4G, kws, rate=rate)
    want = oracle_result(rx, data)
    if rate:
        assert want[1] == 1        # about 4,300 planted keywords
    c = sfa.compile(rx)
    assert c.info.n_sfa > 0 and not c.info.sfa_over_cap
    x = to_device(data)
    del data
    # the benchmark's table: hot rows chosen from a profile of an independent
    # sample of the same text distribution
    prof = W.c3_input(seed + 1000, 1 << 20, kws, rate=rate)
    for t in (sfa.load(c, profile_sample=prof), sfa.load(c)):
        assert t.info["table_in_lds"] == 0 and 0 < t.info["hot_rows"] < c.info.n_sfa
        say("c3 4GiB seed", seed, "hot rows", t.info["hot_rows"])
        got = sfa.match(t, x).tolist()
        assert got == want, (seed, got, want)
    torch.cuda.synchronize()


def test_c2_regex_past_4gib_unaligned():
    n = N4G + 13
    say("c2 regex n=2^32+13 offset 3, generating")
    data = W.c2_input(5, n)
    want = oracle_result(W.REGEX_C2, data)
    assert want[1] == int(data[-5] == ord("a"))      # closed form
    x = to_device(data, offset=3)
    del data
    t = sfa.load(sfa.compile(W.REGEX_C2))
    assert t.info["table_in_lds"] == 1
    for n_chunks in (0, 65536, 1 << 20):
        say("c2 regex n=2^32+13 chunks", n_chunks)
        assert sfa.match(t, x, n_chunks=n_chunks).tolist() == want, n_chunks
    torch.cuda.synchronize()
