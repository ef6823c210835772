"""On-the-fly D-SFA construction (the on-the-fly remark of Section 5.1) in
the host compiler, checked on the CPU against the complete construction.

A lazily built state is a mapping reached from the identity by the sample's
runs, so it must be a state of the complete D-SFA (Algorithm 4), and every
built transition must be the DFA applied after the mapping (delta_s(f, c) =
delta o f); transitions no run took stay unbuilt.  Example 1's run over
"abab" (Table 1) builds exactly the states it visits.
"""
import numpy as np
import pytest

from conftest import golden_lines

import workloads as W
import paper_1405_0562_amd as sfa
from oracle.automata import compile_regex
from oracle.sfa import byte_dsfa

UNBUILT = 0xFFFFFFFF


def _lazy(rx, sample, **kw):
    c = sfa.compile(rx, sfa_cap=0)
    assert c.info.n_sfa == 0
    c.build_lazy(sample, **kw)
    assert c.info.sfa_lazy
    return c, c.arrays()


def _check_consistent(a):
    """Every built transition is delta after the mapping; state 0 is the
    identity; all mappings are distinct."""
    n = a["dfa_next"].shape[0]
    maps, nxt, dnext = a["sfa_map"], a["sfa_next"], a["dfa_next"]
    assert maps[0].tolist() == list(range(n))
    assert len({m.tobytes() for m in maps}) == maps.shape[0]
    for f in range(nxt.shape[0]):
        for c in range(nxt.shape[1]):
            t = nxt[f, c]
            if t != UNBUILT:
                assert np.array_equal(maps[t], dnext[maps[f], c]), (f, c)


def test_example1_run_builds_the_visited_states():
    rows = {}
    for line in golden_lines("example1_table1.txt"):
        tok = line.split()
        rows.setdefault(tok[0], []).append(tok[1:])
    table = {k: [int(x) for x in v[0]] for k, v in rows.items() if k.startswith("f") and k[1:].isdigit()}
    c, a = _lazy("(ab)*", b"abab", start_every=4, walk_bytes=4)
    a_cls, b_cls = a["byte_class"][ord("a")], a["byte_class"][ord("b")]
    # the compiler numbers D_1's states in its own canonical order: Table 1's
    # states 0, 1 (after a) and 2 (the sink) are its 0, delta(0, a), delta(0, b)
    perm = [0, int(a["dfa_next"][0, a_cls]), int(a["dfa_next"][0, b_cls])]

    def renamed(f):
        g = [0] * 3
        for q in range(3):
            g[perm[q]] = perm[f[q]]
        return g

    # f0 -a-> f1 -b-> f4 -a-> f1 -b-> f4: three states, in the order reached
    assert c.info.n_sfa == 3
    assert [m.tolist() for m in a["sfa_map"]] == [renamed(table[k]) for k in ("f0", "f1", "f4")]
    nxt = a["sfa_next"]
    assert nxt[0, a_cls] == 1 and nxt[1, b_cls] == 2 and nxt[2, a_cls] == 1
    # transitions never taken stay unbuilt
    assert nxt[0, b_cls] == UNBUILT and nxt[1, a_cls] == UNBUILT and nxt[2, b_cls] == UNBUILT
    _check_consistent(a)


def test_closure_fills_edges_between_built_states():
    # "aab": f0 -a-> f1 -a-> f3 -b-> f3 (f3 = the constant mapping to the
    # sink); the edge f3 -a-> f3 was not taken but its target is built
    c, a = _lazy("(ab)*", b"aab", start_every=3, walk_bytes=3)
    a_cls, b_cls = a["byte_class"][ord("a")], a["byte_class"][ord("b")]
    assert c.info.n_sfa == 3
    sink = int(a["dfa_next"][0, b_cls])
    assert a["sfa_map"][2].tolist() == [sink] * 3
    assert a["sfa_next"][2, a_cls] == 2 and a["sfa_next"][2, b_cls] == 2
    # f1 -b-> f4 leads to a mapping no run reached: unbuilt
    assert a["sfa_next"][1, b_cls] == UNBUILT
    _check_consistent(a)


@pytest.mark.parametrize("rx", [W.REGEX_C1, W.REGEX_C2, W.rn_regex(5), "(([02468][13579]){5})*",
                                W.c3_regex(W.c3_keywords(0)[:4])])
def test_lazy_states_are_states_of_the_complete_dsfa(rx):
    rng = np.random.default_rng(1)
    full, cls = byte_dsfa(compile_regex(rx), cap=100_000)
    alphabet = np.unique(np.concatenate([np.frombuffer(b"abcdefghijklmnopqrstuvwxyz 0123456789", np.uint8),
                                         rng.integers(0, 256, 8, dtype=np.uint8)]))
    sample = rng.choice(alphabet, size=20_000).astype(np.uint8)
    c, a = _lazy(rx, sample, start_every=97, walk_bytes=500)
    _check_consistent(a)
    full_maps = {m.tobytes() for m in np.asarray(full.maps, dtype=np.int64)}
    assert all(m.tobytes() in full_maps for m in a["sfa_map"])
    assert c.info.n_sfa <= full.m


def test_long_sample_reaches_every_state():
    """Runs over a long random text from many starts build the whole D-SFA
    of a small automaton: the same set of mappings as Algorithm 4."""
    rx = W.REGEX_C2
    full, _ = byte_dsfa(compile_regex(rx), cap=100_000)
    sample = np.random.default_rng(2).choice(np.frombuffer(b"abc", np.uint8), size=50_000).astype(np.uint8)
    c, a = _lazy(rx, sample, start_every=13, walk_bytes=64)
    assert c.info.n_sfa == full.m
    assert {m.tobytes() for m in a["sfa_map"]} == {m.tobytes() for m in np.asarray(full.maps, dtype=np.int64)}


def test_max_states_and_arguments():
    rx = W.rn_regex(20)
    sample = W.rn_input(0, 20, 40_000)
    c, a = _lazy(rx, sample, start_every=7, walk_bytes=300, max_states=50)
    assert c.info.n_sfa == 50
    _check_consistent(a)
    assert (a["sfa_next"] == UNBUILT).any()
    # rebuilding from another sample replaces the partial D-SFA
    c.build_lazy(sample[:100], start_every=100, walk_bytes=100, max_states=1000)
    assert c.info.n_sfa <= 101
    _check_consistent(c.arrays())
    with pytest.raises(sfa.SfaError):
        c.build_lazy(sample, start_every=0)
    full = sfa.compile(W.REGEX_C2)
    with pytest.raises(sfa.SfaError):
        full.build_lazy(b"ab")


def test_partial_table_plans_a_global_walk():
    """A partial D-SFA gets no LDS image and no product table: its device
    size is the global table plus the hot image (checked without a device)."""
    import ctypes
    from paper_1405_0562_amd import _capi
    from paper_1405_0562_amd._capi import lib, check
    c, _ = _lazy(W.REGEX_C2, b"abab" * 100, start_every=8, walk_bytes=16)
    complete = sfa.compile(W.REGEX_C2)
    sizes = []
    for comp in (c, complete):
        d = comp.desc()
        nb = ctypes.c_size_t()
        check(lib().sfa_table_device_bytes(ctypes.byref(d), None, ctypes.byref(nb)))
        sizes.append(nb.value)
    assert sizes[0] < sizes[1]   # the complete one carries LDS images (and a product table)
