"""GPU parity of N-SFA matching against the oracle.

An N-SFA compilation (position automaton, Algorithm 4 over correspondences)
is loaded and matched like a D-SFA; the result state names the final set of
NFA states S_fin = U_{q in I} f_fin(q).  Every case compares S_fin and the
accept bit with the oracle's NFA run (the plain definition), bit for bit,
through the LDS walk (product table and mapping composition), the global
walk, the speculative kernel and the batched form.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import nsfa as ON

pytestmark = pytest.mark.gpu

sfa = pytest.importorskip("paper_1405_0562_amd")


def say(*a):
    print("[gpu-case]", *a, flush=True)


def oracle_set(rx, data):
    a = ON.glushkov(rx)
    s = ON.nfa_run(a, bytes(data))
    return s, bool(s & a.final)


def text_for(rx, seed, n):
    rng = np.random.default_rng(seed)
    if rx == W.REGEX_C1:
        return W.c1_input(seed, n=n - n % 2)
    if rx == W.REGEX_C2:
        return W.c2_input(seed, n=n)
    data = W.uniform_over(W.rng_for(seed, 3), W.ALPHABET_C4, n)
    if rx.startswith(".*") and rx.endswith(".*") and n > len(rx):
        kw = rx[2:-2].encode()
        for p in rng.integers(0, max(1, n - len(kw)), size=3):
            data[p:p + len(kw)] = np.frombuffer(kw, np.uint8)
    return data


NSFA_RX = [W.REGEX_C1, W.REGEX_C2, "(ab)*", ".*abc.*"] + W.c4_regexes(0)[:4]


@pytest.mark.parametrize("rx", NSFA_RX)
def test_nsfa_all_paths(rx):
    c = sfa.compile_nsfa(rx)
    assert c.info.n_sfa > 0
    t_lds = sfa.load(c)
    t_glob = sfa.load(c, force_global=True)
    t_map = sfa.load(c, product=False)
    for seed, n in ((1, 150_017), (2, 4099), (3, 0)):
        data = text_for(rx, seed, n)
        want = oracle_set(rx, data)
        x = torch.from_numpy(data).cuda() if n else torch.empty(0, dtype=torch.uint8, device="cuda")
        for t in (t_lds, t_glob, t_map):
            for n_chunks in (0, 3, 777, 65536):
                say(rx[:30], "n", n, "chunks", n_chunks, t.info)
                q, acc = sfa.match(t, x, n_chunks=n_chunks).tolist()
                assert (c.nsfa_set(q), bool(acc)) == want, (rx, n, n_chunks, t.info)
        q, acc = sfa.match_speculative(t_lds, x, n_chunks=1000).tolist()
        assert (c.nsfa_set(q), bool(acc)) == want


def test_nsfa_modes_reported():
    small = sfa.load(sfa.compile_nsfa(W.REGEX_C2))          # 64 states: product table
    big = sfa.load(sfa.compile_nsfa(W.c4_regexes(0)[0]))    # 442 states: mapping composition
    assert small.info["product_table"] == 1
    assert big.info["product_table"] == 0 and big.info["n_sfa"] > 128


def test_nsfa_over_cap_speculative():
    rx = W.c4_regexes(0)[0]
    c = sfa.compile_nsfa(rx, nsfa_cap=50)
    assert c.info.n_sfa == 0
    t = sfa.load(c)
    data = text_for(rx, 7, 300_000)
    q, acc = sfa.match_speculative(t, torch.from_numpy(data).cuda(), n_chunks=256).tolist()
    assert (c.nsfa_set(q), bool(acc)) == oracle_set(rx, data)


def test_nsfa_batch():
    regexes = W.c4_regexes(1)[:4]
    comps = [sfa.compile_nsfa(rx) for rx in regexes]
    tables = [sfa.load(c) for c in comps]
    rng = np.random.default_rng(3)
    lens = rng.integers(0, 20_000, size=40)
    off = np.zeros(41, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    data = W.uniform_over(W.rng_for(4, 7), W.ALPHABET_C4, int(off[-1]))
    jobs = np.array([(d, t) for d in range(40) for t in range(4)], dtype=np.uint32)
    b = sfa.Batch(tables, off, jobs)
    got = b.run(torch.from_numpy(data).cuda()).cpu().numpy()
    for i, (d, t) in enumerate(jobs):
        want = oracle_set(regexes[t], data[off[d]:off[d + 1]])
        assert (comps[t].nsfa_set(int(got[i, 0])), bool(got[i, 1])) == want, (d, t)
