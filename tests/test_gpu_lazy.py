"""GPU parity of the on-the-fly D-SFA walk against the CPU oracle.

Tables are compiled without a D-SFA and given a partial one built from a
sample (sfa_compiled_build_lazy); the global-table walk parks pieces that
reach an unbuilt transition and finishes them through the DFA.  Results
(final canonical DFA state, accept) must equal the oracle's Algorithm 2 run
bit for bit: with few pieces parked (a sample like the input), with most
pieces parked (a tiny sample, few states), across the three entry widths of
the global table (u8, u16, u32 ids), with few hot rows in LDS (cold misses
and parking together), over ragged, unaligned, tiny and empty inputs and
many chunk counts.
"""
import functools

import numpy as np
import pytest
import torch

import workloads as W
from oracle.automata import compile_regex
from oracle import scan as oscan

pytestmark = pytest.mark.gpu

sfa = pytest.importorskip("paper_1405_0562_amd")

KW60 = W.c3_keywords(0, count=60)
RX_KW60 = W.c3_regex(KW60)


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


def lazy_table(rx, sample, start_every=256, walk_bytes=4096, max_states=65535, lds_budget=0):
    c = sfa.compile(rx, sfa_cap=0).build_lazy(sample, start_every=start_every, walk_bytes=walk_bytes,
                                               max_states=max_states)
    t = sfa.load(c, profile_sample=sample, lds_budget=lds_budget)
    assert t.info["partial"] == 1 and t.info["table_in_lds"] == 0 and t.info["product_table"] == 0
    return t


def to_device(data, offset=0):
    buf = torch.empty(data.size + offset + 16, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + data.size]
    if data.size:
        view.copy_(torch.from_numpy(np.ascontiguousarray(data)))
    return view


def check(t, rx, data, n_chunks=0, offset=0, tag=""):
    say(tag, rx[:30], "n=%d" % data.size, "chunks=%d" % n_chunks, "off=%d" % offset,
        "states=%d" % t.info["n_sfa"], "width=%d" % t.info["next_bytes"])
    got = sfa.match(t, to_device(data, offset), n_chunks=n_chunks).tolist()
    want = oracle_result(rx, data)
    assert got == want, (tag, data.size, n_chunks, offset, got, want)


@functools.lru_cache(maxsize=None)
def kw_text(seed, n, rate):
    return W.c3_input(seed, n, KW60, rate=rate)


def test_keywords_sample_like_the_input():
    sample = kw_text(100, 1 << 20, 1e-4)
    t = lazy_table(RX_KW60, sample)
    assert t.info["next_bytes"] == 2
    for seed, n in ((1, 8 << 20), (2, (8 << 20) + 13), (3, 3 << 20)):
        check(t, RX_KW60, kw_text(seed, n, 1e-4), tag="kw60")


def test_most_pieces_park():
    """A 2 KiB sample and at most 64 states: nearly every piece reaches an
    unbuilt transition and finishes through the DFA."""
    sample = kw_text(101, 2048, 1e-3)
    t = lazy_table(RX_KW60, sample, start_every=64, walk_bytes=256, max_states=64)
    assert t.info["next_bytes"] == 1
    data = kw_text(4, (1 << 20) + 7, 1e-3)
    for n_chunks in (0, 1, 7, 1000):
        check(t, RX_KW60, data, n_chunks=n_chunks, tag="park")
    check(t, RX_KW60, data, offset=3, tag="park-unaligned")


def test_few_hot_rows_with_parking():
    sample = kw_text(102, 256 << 10, 1e-4)
    t = lazy_table(RX_KW60, sample, max_states=3000, lds_budget=4096)
    assert 0 < t.info["hot_rows"] < t.info["n_sfa"]
    check(t, RX_KW60, kw_text(5, 4 << 20, 1e-4), tag="hot-few")


def test_wide_ids_rn():
    """r_130 sampled from every start: more than 65,535 states, u32 ids."""
    rx = W.rn_regex(130)
    t = lazy_table(rx, W.rn_input(0, 130, 100_000), start_every=1, walk_bytes=400, max_states=70_000)
    assert t.info["next_bytes"] == 4 and t.info["n_sfa"] > 65535
    data = W.rn_input(6, 130, (2 << 20) + 260 * 3)
    check(t, rx, data, tag="rn130")
    check(t, rx, data[:-5], tag="rn130-reject")


def test_transient_heavy_rn_small_sample():
    rx = W.rn_regex(50)
    t = lazy_table(rx, W.rn_input(1, 50, 4000), start_every=100, walk_bytes=1000, max_states=2000)
    data = W.rn_input(7, 50, 1 << 20)
    for n_chunks in (0, 3, 4096):
        check(t, rx, data, n_chunks=n_chunks, tag="rn50")


def test_tiny_and_empty_inputs():
    sample = kw_text(103, 4096, 1e-3)
    t = lazy_table(RX_KW60, sample, max_states=100)
    rng = np.random.default_rng(9)
    alphabet = np.frombuffer(W.ALPHABET_C3, np.uint8)
    for n in (0, 1, 5, 15, 16, 17, 255, 4097):
        check(t, RX_KW60, rng.choice(alphabet, size=n).astype(np.uint8), tag="tiny")
    word = np.frombuffer(KW60[3], np.uint8)
    check(t, RX_KW60, np.concatenate([rng.choice(alphabet, size=1000).astype(np.uint8), word]), tag="tail-hit")
