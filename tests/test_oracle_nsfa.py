"""Pins of the N-SFA oracle (SFA built from an NFA, Sections 4 and 5.1).

Each check compares the oracle with something it does not compute itself:
the position counts of the regexes, the independent set-of-positions matcher
and the DFA oracle, Theorem 1's bound, closure and associativity of the
composition, Theorem 2 against the plain NFA run, and Table 1's D-SFA (the
N-SFA of (ab)* from its position automaton realises the same monoid).
"""
import itertools
import random

import pytest

from oracle import nsfa as N
from oracle.automata import compile_regex, run_dfa
from oracle.regex import matches
from tests.conftest import golden_lines

REGEXES = ["(ab)*", "(a|b)*a(a|b){2}", "a{2,3}b?", "(a|bc)*c", ".*abc.*", "(a*b*)*", "[ab]{0,2}(ba)+", "",
           "((a|b)(a|b))*", "a?b?c?"]


@pytest.mark.parametrize("rx,count", [("(ab)*", 3), ("(a|b)*a(a|b){4}", 12), ("a{2,3}", 4), ("a+", 3),
                                      ("", 1), ("(a|b)?c", 4), ("[0-4]{5}", 6)])
def test_position_automaton_sizes(rx, count):
    # one state per byte-set leaf after writing out bounded repeats, plus the initial state
    assert N.glushkov(rx).n == count


@pytest.mark.parametrize("rx", REGEXES)
def test_nfa_language_is_the_regex_language(rx):
    a = N.glushkov(rx)
    d = compile_regex(rx)
    for k in range(0, 7):
        for w in itertools.product(b"abc", repeat=k):
            w = bytes(w)
            want = matches(rx, w)
            assert N.accepts(a, w) == want, (rx, w)
            assert bool(d.accept[run_dfa(d, w)]) == want


@pytest.mark.parametrize("rx", REGEXES)
def test_nsfa_bound_and_closure(rx):
    a = N.glushkov(rx)
    s = N.build_nsfa(a)
    assert s.m <= 2 ** (a.n * a.n)                      # Theorem 1
    index = {f: i for i, f in enumerate(s.maps)}
    assert len(index) == s.m                            # all distinct
    assert s.maps[0] == tuple(1 << q for q in range(a.n))
    for f in s.maps:                                    # closed under reverse composition
        for g in s.maps:
            assert N.compose(f, g) in index


@pytest.mark.parametrize("rx", REGEXES[:6])
def test_composition_is_associative(rx):
    s = N.build_nsfa(N.glushkov(rx))
    rng = random.Random(3)
    for _ in range(200):
        f, g, h = (s.maps[rng.randrange(s.m)] for _ in range(3))
        assert N.compose(N.compose(f, g), h) == N.compose(f, N.compose(g, h))


@pytest.mark.parametrize("rx", REGEXES)
def test_any_split_equals_the_nfa_run(rx):
    a = N.glushkov(rx)
    s = N.build_nsfa(a)
    rng = random.Random(7)
    for _ in range(60):
        w = bytes(rng.choice(b"abcx") for _ in range(rng.randrange(0, 40)))
        want = N.nfa_run(a, w)
        for p in (1, 2, 3, 7):
            fin, acc = N.nsfa_parallel(s, w, p)
            assert fin == want and acc == bool(want & a.final), (rx, w, p)
        cuts = sorted(rng.randrange(0, len(w) + 1) for _ in range(rng.randrange(0, 5)))
        bounds = list(zip([0] + cuts, cuts + [len(w)]))
        assert N.nsfa_parallel(s, w, bounds=bounds)[0] == want


def test_walk_equals_composition_of_letters():
    # Lemma 1: the state reached on uv is f_u . f_v
    s = N.build_nsfa(N.glushkov("(a|bc)*c"))
    rng = random.Random(1)
    for _ in range(100):
        u = bytes(rng.choice(b"abc") for _ in range(rng.randrange(0, 9)))
        v = bytes(rng.choice(b"abc") for _ in range(rng.randrange(0, 9)))
        fu, fv, fuv = (s.maps[N.nsfa_walk(s, x)] for x in (u, v, u + v))
        assert N.compose(fu, fv) == fuv


def test_ab_star_realises_table1_monoid():
    # Table 1 lists the six D-SFA states of (ab)* over {a, b}.  The N-SFA of
    # its position automaton (3 states: initial, a, b) is another automaton
    # for the same language, with six states as well; two words reach the
    # same N-SFA state exactly when they reach the same D-SFA state of Table 1.
    rows = {}
    for line in golden_lines("example1_table1.txt"):
        parts = line.split()
        if parts[0].startswith("f") and parts[0][1:].isdigit():
            rows[parts[0]] = tuple(int(x) for x in parts[1:])
        if parts[0] == "dfa":
            rows["dfa_" + parts[1]] = tuple(int(x) for x in parts[2:])
    table1 = {v: k for k, v in rows.items() if k.startswith("f")}

    def dsfa_state(w):
        f = rows["f0"]
        for ch in w:
            col = rows["dfa_" + chr(ch)]
            f = tuple(col[x] for x in f)
        return table1[f]

    s = N.build_nsfa(N.glushkov("(ab)*"))
    assert s.m == len(table1) == 6
    words = [bytes(w) for k in range(7) for w in itertools.product(b"ab", repeat=k)]
    pairs = {(N.nsfa_walk(s, w), dsfa_state(w)) for w in words}
    left = {p[0] for p in pairs}
    right = {p[1] for p in pairs}
    assert len(pairs) == len(left) == len(right) == 6       # a bijection between the two state sets
    # and the run over "abab" ends in an accepting state of both
    assert s.accepting(N.nsfa_walk(s, b"abab")) and dsfa_state(b"abab") in ("f0", "f4")


def test_over_cap():
    with pytest.raises(N.OverCap):
        N.build_nsfa(N.glushkov("(a|b)*a(a|b){3}"), cap=5)
