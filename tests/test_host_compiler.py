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
