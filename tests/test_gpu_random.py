"""GPU parity on random regexes through every matcher.

Seeded random regexes over small alphabets (tests/regexgen.py), each matched
on a seeded text over its alphabet (with stray bytes) by the D-SFA walk (LDS
image or global table, whichever the loader picks, and the global table
forced), the speculative kernel, an on-the-fly D-SFA built from a short
sample, and one batch over all regexes and several documents; every result
must equal the oracle's Algorithm 2 run bit for bit.
"""
import functools
import random

import numpy as np
import pytest
import torch

from regexgen import random_regex
from oracle.automata import compile_regex
from oracle import scan as oscan

pytestmark = pytest.mark.gpu

sfa = pytest.importorskip("paper_1405_0562_amd")


def say(*a):
    print("[gpu-case]", *a, flush=True)


@functools.lru_cache(maxsize=None)
def oracle_dfa(rx):
    d = compile_regex(rx)
    return d, oscan.table_u32(d)


def oracle_result(rx, data):
    d, tab = oracle_dfa(rx)
    q = oscan.scan(d, data, table=tab)
    return [q, int(d.accept[q])]


def regexes(seed, count, alphabet):
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        rx = random_regex(rng, alphabet, depth=3)
        try:
            small = compile_regex(rx).n <= 300
        except OverflowError:   # the subset construction blows up: not a test case here
            small = False
        if small:
            out.append(rx)
    return out


def text(seed, n, alphabet):
    rng = np.random.default_rng(seed)
    alpha = np.frombuffer(alphabet.encode(), np.uint8)
    out = rng.choice(alpha, size=n).astype(np.uint8)
    stray = rng.random(n) < 0.001
    out[stray] = rng.integers(0, 256, size=int(stray.sum()), dtype=np.uint8)
    return out


def to_device(data):
    x = torch.empty(max(1, data.size), dtype=torch.uint8, device="cuda")
    if data.size:
        x[: data.size].copy_(torch.from_numpy(np.ascontiguousarray(data)))
    return x[: data.size]


@pytest.mark.parametrize("alphabet,seed", [("ab", 1), ("abc", 2), ("abcd", 3)])
def test_random_regexes_every_matcher(alphabet, seed):
    for i, rx in enumerate(regexes(seed, 12, alphabet)):
        data = text(seed * 100 + i, (1 << 18) + 37 * i, alphabet)
        want = oracle_result(rx, data)
        x = to_device(data)
        comp = sfa.compile(rx)
        say(alphabet, i, rx, "n_sfa=%d" % comp.info.n_sfa)
        for force_global in (False, True):
            t = sfa.load(comp, force_global=force_global)
            for n_chunks in (0, 1, 977):
                assert sfa.match(t, x, n_chunks=n_chunks).tolist() == want, (rx, force_global, n_chunks)
            assert sfa.match_speculative(t, x, n_chunks=300).tolist() == want, rx
        lazy = sfa.compile(rx, sfa_cap=0).build_lazy(data[:4096], start_every=64, walk_bytes=256, max_states=64)
        tl = sfa.load(lazy, profile_sample=data[:4096])
        for n_chunks in (0, 333):
            assert sfa.match(tl, x, n_chunks=n_chunks).tolist() == want, (rx, "lazy", n_chunks)


def test_random_regexes_in_one_batch():
    # regexes whose tables the batch kernel takes (a stride-1 walk image)
    rxs, tables = [], []
    for rx in regexes(7, 30, "abc"):
        t = sfa.load(sfa.compile(rx))
        if t.info["strides"] & 2 and len(rxs) < 10:
            rxs.append(rx)
            tables.append(t)
    assert len(rxs) == 10
    rng = np.random.default_rng(8)
    lens = rng.integers(0, 50_000, size=40)
    lens[:3] = (0, 1, 300_000)
    off = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    data = text(9, int(off[-1]), "abc")
    jobs = np.array([(d, t) for d in range(lens.size) for t in range(len(rxs))], dtype=np.uint32)
    say("batch", len(jobs), "jobs")
    for piece, units in ((256, 1), (2048, 2), (4096, 4)):
        b = sfa.Batch(tables, off, jobs, sfa.BatchOptions(piece, units))
        got = b.run(to_device(data)).cpu().numpy()
        torch.cuda.synchronize()
        for j, (d, t) in enumerate(jobs):
            assert got[j].tolist() == oracle_result(rxs[t], data[off[d]:off[d + 1]]), (piece, units, d, t)
