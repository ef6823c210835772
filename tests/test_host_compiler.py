"""The product's host compiler (C++, in libsfa.so) against the oracle.

Both build the canonical minimal complete DFA independently (position
automaton + Hopcroft vs Thompson + Moore), so their tables must be equal
entry by entry; the D-SFA construction follows the same worklist order, so
the mapping tables must be equal too.  Host logic only: no GPU involved.
"""
import random
import re

import numpy as np
import pytest

from regexgen import random_regex

import workloads as W
import paper_1405_0562_amd as sfa
from oracle.automata import compile_regex
from oracle.regex import ParseError as OracleParseError, parse
from oracle.sfa import byte_dsfa, OverCap


def _same(rx, sfa_cap=65535):
    c = sfa.compile(rx, sfa_cap=sfa_cap)
    a = c.arrays()
    d = compile_regex(rx)
    try:
        s, cls = byte_dsfa(d, cap=sfa_cap)
    except OverCap:
        s = None
    assert c.info.n_dfa == d.n and c.info.q0 == 0
    assert np.array_equal(a["dfa_next"][:, a["byte_class"]], d.delta)
    if s is None:
        assert c.info.n_sfa == 0 and c.info.sfa_over_cap
        return c
    assert np.array_equal(a["byte_class"], cls)
    assert np.array_equal(a["dfa_next"][:, a["byte_class"]], d.delta)
    assert np.array_equal(a["dfa_accept"], d.accept)
    assert c.info.n_sfa == s.m
    assert np.array_equal(a["sfa_map"], s.maps)
    assert np.array_equal(a["sfa_next"], s.nxt)
    return c


NAMED = ["(ab)*", W.REGEX_C1, W.REGEX_C2, W.rn_regex(5), W.rn_regex(20), W.ra_regex(5),
         "(([02468][13579]){5})*", "[ap]*[al][alp]{5}", "(m|(t|c([mt]*c){3})[cmt])*",
         ".*(T.*T.*Y.*P.*P.*R.*O.*M.*P.*T.*)", "", "()", "a|", "(|a)+", r"\x00\xff.", r"[^\x00-\xfe]*"]


@pytest.mark.parametrize("rx", NAMED)
def test_named_regexes_equal_oracle(rx):
    _same(rx)


def test_c3_keyword_regex_equal_oracle():
    for seed in (0, 1):
        _same(W.c3_regex(W.c3_keywords(seed)))


def test_c4_c5_families_equal_oracle():
    for rx in W.c4_regexes(0) + W.c5_regexes(0):
        _same(rx)


def test_random_regexes_equal_oracle():
    rng = random.Random(11)
    done = 0
    while done < 150:
        rx = random_regex(rng, "abc\n")
        try:
            compile_regex(rx, max_dfa_states=400)
        except OverflowError:
            continue
        _same(rx, sfa_cap=5000)
        done += 1


def test_parse_errors_agree():
    bad = ["*a", "a**", "(a", "a)", "[a", "[b-a]", "\\q", "a{2}{3}", "a{3,2}", "a{1001}", "[\\d-z]", "\\x4"]
    for rx in bad:
        with pytest.raises(OracleParseError):
            parse(rx)
        with pytest.raises(sfa.ParseError):
            sfa.compile(rx)
    for rx in ["a{", "a{,}", "{", "}", "]", "a{x}", "x{2,", r"\{2\}"]:
        parse(rx)
        _same(rx)
        assert re.compile(rx.encode())


def test_sfa_cap_and_dfa_cap():
    c = sfa.compile(W.REGEX_C2, sfa_cap=10)
    assert c.info.n_sfa == 0 and c.info.sfa_over_cap and c.info.n_dfa == 33
    c = sfa.compile(W.REGEX_C2, sfa_cap=0)
    assert c.info.n_sfa == 0 and not c.info.sfa_over_cap
    c = sfa.compile(W.REGEX_C2, sfa_cap=64)
    assert c.info.n_sfa == 64
    with pytest.raises(sfa.SfaError) as e:
        sfa.compile("[ap]*[al][alp]{10}", dfa_cap=100)
    assert e.value.status == 3


def test_rn_construction_counts_and_speed():
    c = sfa.compile(W.rn_regex(50))
    assert (c.info.n_dfa, c.info.n_sfa) == (101, 10100)
    assert c.info.sfa_seconds < 5.0


# --------------------------------------------------------------------------
# N-SFA compilation (position automaton, correspondences)
# --------------------------------------------------------------------------
from oracle import nsfa as ON  # noqa: E402


def _nsfa_table_result(arr, c, w: bytes):
    f = 0
    for b in w:
        f = arr["sfa_next"][f, arr["byte_class"][b]]
    q = int(arr["sfa_map"][f, arr["q0"]])
    return c.nsfa_set(q), bool(arr["dfa_accept"][q])


def _check_nsfa(rx, alphabet, rng, words=60):
    c = sfa.compile_nsfa(rx)
    a = ON.glushkov(rx)
    s = ON.build_nsfa(a)
    assert c.info.n_sfa == s.m and c.info.n_positions + 1 == a.n, rx
    sets, final, n_nfa = c.nsfa_sets()
    assert n_nfa == a.n and c.nsfa_set(0) == a.initial
    assert sum(int(x) << (64 * i) for i, x in enumerate(final)) == a.final
    arr = c.arrays()
    assert list(arr["sfa_map"][0]) == list(range(c.info.n_dfa))      # state 0 is the identity
    for _ in range(words):
        w = bytes(rng.choice(alphabet) for _ in range(rng.randrange(0, 50)))
        want = ON.nfa_run(a, w)
        assert _nsfa_table_result(arr, c, w) == (want, bool(want & a.final)), (rx, w)


@pytest.mark.parametrize("rx", ["(ab)*", W.REGEX_C1, W.REGEX_C2, ".*abc.*", "(a|bc)*c", "", "a?b?c?",
                                W.rn_regex(3)])
def test_nsfa_named_regexes_equal_oracle(rx):
    _check_nsfa(rx, b"abc0123456789", random.Random(2))


def test_nsfa_workload_families_equal_oracle():
    rng = random.Random(5)
    for rx in W.c4_regexes(0) + W.c5_regexes(1)[:6]:
        _check_nsfa(rx, W.ALPHABET_C4, rng, words=20)


def test_nsfa_random_regexes_equal_oracle():
    rng = random.Random(11)
    done = 0
    while done < 40:
        rx = random_regex(rng, "abc", depth=3)
        try:
            s = ON.build_nsfa(ON.glushkov(rx), cap=3000)
        except ON.OverCap:
            continue
        _check_nsfa(rx, b"abcd", rng, words=15)
        done += 1


def test_nsfa_cap_and_sets_of_a_dsfa():
    c = sfa.compile_nsfa(W.REGEX_C2, nsfa_cap=10)
    assert c.info.n_sfa == 0 and c.info.sfa_over_cap
    # the subset automaton remains (for the speculative matcher)
    arr = c.arrays()
    w = b"ab" * 50 + b"aabbb"
    q = 0
    for b in w:
        q = arr["dfa_next"][q, arr["byte_class"][b]]
    a = ON.glushkov(W.REGEX_C2)
    assert c.nsfa_set(int(q)) == ON.nfa_run(a, w)
    with pytest.raises(ValueError):
        sfa.compile(W.REGEX_C2).nsfa_sets()
