"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (fixtures under tests/golden/), closed forms, textbook facts,
brute force on tiny inputs and Python's own regex engine.
"""
import itertools
import random
import re

import numpy as np
import pytest

from conftest import golden_lines
from regexgen import random_regex

import workloads as W
from oracle.automata import compile_regex, run_dfa, byte_classes, Dfa, canonicalize, minimize
from oracle.regex import parse, matches, ParseError
from oracle.sfa import (build_dsfa, byte_dsfa, paper_counts, compose, sfa_parallel,
                        sfa_walk, speculative_chunk, speculative_parallel, chunks_of, OverCap)
from oracle import scan as oscan


# --------------------------------------------------------------------------
# P1 / P2: Examples 1 and 2 (Table 1) of the paper
# --------------------------------------------------------------------------
def _example1():
    rows = {}
    for line in golden_lines("example1_table1.txt"):
        tok = line.split()
        rows.setdefault(tok[0], []).append(tok[1:])
    sym = {r[0]: [int(x) for x in r[1:]] for r in rows["dfa"]}
    delta = np.array([[sym["a"][q], sym["b"][q]] for q in range(3)])
    table = {k: [int(x) for x in v[0]] for k, v in rows.items() if re.fullmatch(r"f\d+", k)}
    final = rows["final"][0]
    run = rows["run"][0]
    return delta, table, final, run


def test_table1_mappings_and_order():
    delta, table, final, _ = _example1()
    s = build_dsfa(delta, 0, np.array([True, False, False]))
    assert s.m == 6
    # FIFO worklist with symbol a before b numbers the states exactly as Table 1
    for i in range(6):
        assert s.maps[i].tolist() == table["f%d" % i], i
    assert [("f%d" % i) for i in range(6) if s.accept[i]] == final


def test_example1_run_abab():
    delta, table, _, run = _example1()
    s = build_dsfa(delta, 0, np.array([True, False, False]))
    word, states = run[0], run[1:]
    cur = 0
    seen = ["f0"]
    for ch in word:
        cur = int(s.nxt[cur, "ab".index(ch)])
        seen.append("f%d" % cur)
    assert seen == states
    assert s.maps[cur][0] == 0 and s.accept[cur]


def test_example2_parallel_run():
    delta, _, _, _ = _example1()
    s = build_dsfa(delta, 0, np.array([True, False, False]))
    cls = np.zeros(256, dtype=np.int64)
    cls[ord("b")] = 1
    lines = [l.split() for l in golden_lines("example2_parallel.txt")]
    chunks = [(t[1], int(t[2][1:])) for t in lines if t[0] == "chunk"]
    for word, f in chunks:
        assert sfa_walk(s, cls, word.encode()) == f
    for t in lines:
        if t[0] == "compose":
            a, b, c = (int(x[1:]) for x in t[1:])
            assert compose(s.maps[a], s.maps[b]).tolist() == s.maps[c].tolist()
        if t[0] == "sequential":
            q = int(t[1])
            for _, f in chunks:
                q = int(s.maps[f][q])
            assert q == int(t[2])
    word = "".join(w for w, _ in chunks).encode()
    cuts = list(itertools.accumulate(len(w) for w, _ in chunks))
    res = sfa_parallel(s, cls, word, bounds=list(zip([0] + cuts[:-1], cuts)))
    assert res["chunk_states"] == [f for _, f in chunks]
    assert res["q_parallel"] == res["q_sequential"] == 0


# --------------------------------------------------------------------------
# P3: state counts printed in Section 6 and their closed forms
# --------------------------------------------------------------------------
def _printed_counts():
    out = []
    for line in golden_lines("state_counts.txt"):
        rx, d, s, where = line.split("\t")
        out.append((rx, int(d), int(s), where))
    return out


@pytest.mark.parametrize("row", [r for r in _printed_counts() if "500" not in r[0]], ids=lambda r: r[0])
def test_printed_state_counts(row):
    rx, nd, ns, _ = row
    d = compile_regex(rx)
    s, _ = byte_dsfa(d)
    assert paper_counts(d, s) == (nd, ns)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_rn_closed_form(n):
    # r_n: the DFA is a cycle of 2n states plus the sink; the D-SFA has one
    # loop of 2n mappings per DFA start state: 4n^2 + 2n - 1 without the sink
    d = compile_regex(W.rn_regex(n))
    s, _ = byte_dsfa(d)
    assert d.n == 2 * n + 1 and s.m == 4 * n * n + 2 * n
    assert paper_counts(d, s) == (2 * n, 4 * n * n + 2 * n - 1)


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_ra_closed_form(n):
    d = compile_regex(W.ra_regex(n))
    s, _ = byte_dsfa(d)
    assert paper_counts(d, s) == (2 * n + 2, 4 * n * n + 2 * n)


def test_printed_counts_at_500_follow_closed_forms():
    rows = {r[0]: r for r in _printed_counts()}
    n = 500
    assert rows[W.rn_regex(n)][1:3] == (2 * n, 4 * n * n + 2 * n - 1)
    assert rows[W.ra_regex(n)][1:3] == (2 * n + 2, 4 * n * n + 2 * n)


def test_c1_regex_counts():
    d = compile_regex(W.REGEX_C1)
    s, cls = byte_dsfa(d)
    assert (d.n, s.m, int(cls.max()) + 1) == (11, 22, 3)


# --------------------------------------------------------------------------
# P4: (a|b)*a(a|b){4} accepts exactly when the fifth byte from the end is 'a'
# --------------------------------------------------------------------------
def test_c2_closed_form():
    d = compile_regex(W.REGEX_C2)
    s, _ = byte_dsfa(d)
    assert (d.n, s.m) == (33, 64)
    rng = np.random.default_rng(0)
    for n in list(range(0, 12)) + [100, 1000, 4097]:
        for _ in range(5):
            w = bytes(rng.choice([97, 98], size=n).astype(np.uint8))
            q = oscan.scan(d, w)
            assert bool(d.accept[q]) == (n >= 5 and w[n - 5] == ord("a"))


# --------------------------------------------------------------------------
# P5 / P6: the explosion facts of Section 7.2
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_fact2_full_transformation_monoid_regex(n):
    # (m|(t|c([mt]*c){n-2})[cmt])*: minimal DFA with n states over {c,m,t}
    # whose D-SFA has n^n states (the byte sink adds one state and one mapping)
    d = compile_regex("(m|(t|c([mt]*c){%d})[cmt])*" % (n - 2))
    s, _ = byte_dsfa(d)
    assert paper_counts(d, s) == (n, n ** n)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_fact2_textbook_generators(n):
    # An n-cycle, a transposition and a rank-(n-1) idempotent generate the
    # full transformation monoid, of size n^n.
    cyc = [(q + 1) % n for q in range(n)]
    tr = [1, 0] + list(range(2, n))
    idem = [0, 0] + list(range(2, n))
    delta = np.array([cyc, tr, idem]).T
    s = build_dsfa(delta, 0, np.array([True] + [False] * (n - 1)))
    assert s.m == n ** n


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_fact1_dfa_explosion(n):
    # [ap]*[al][alp]{n-2}: the n-state NFA determinises to 2^n minimal states
    # (every bit pattern, the empty set being the sink)
    d = compile_regex("[ap]*[al][alp]{%d}" % (n - 2))
    assert d.n == 2 ** n


def test_overcap():
    d = compile_regex(W.REGEX_C2)
    with pytest.raises(OverCap):
        byte_dsfa(d, cap=10)


# --------------------------------------------------------------------------
# P7..P10, P13: invariants
# --------------------------------------------------------------------------
SMALL = ["(ab)*", W.REGEX_C1, W.REGEX_C2, "(a|ba)*b?", ".*abc.*", "(a*b*)*c", "[^a]*a.{2}", "(x|y)+z{2,3}"]


@pytest.mark.parametrize("rx", SMALL)
def test_size_bound_and_closure(rx):
    d = compile_regex(rx)
    s, _ = byte_dsfa(d)
    assert s.m <= d.n ** d.n                       # Theorem 1
    keys = {m.tobytes(): i for i, m in enumerate(s.maps)}
    if s.m <= 400:
        for a in range(s.m):                       # Lemma 1: f_u . f_v = f_uv is a state
            for b in range(s.m):
                assert compose(s.maps[a], s.maps[b]).tobytes() in keys


@pytest.mark.parametrize("rx", SMALL)
def test_associativity(rx):
    d = compile_regex(rx)
    s, _ = byte_dsfa(d)
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b, c = (s.maps[i] for i in rng.integers(0, s.m, size=3))
        assert np.array_equal(compose(compose(a, b), c), compose(a, compose(b, c)))
    # and non-commutativity is real for at least one pair in Table 1's SFA
    if rx == "(ab)*":
        assert any(not np.array_equal(compose(x, y), compose(y, x)) for x in s.maps for y in s.maps)


@pytest.mark.parametrize("rx", SMALL)
def test_split_invariance_and_speculation(rx):
    # Theorem 2: any division of w gives the same result; Algorithm 3's
    # per-chunk table T_i equals the mapping of the chunk's SFA state
    d = compile_regex(rx)
    s, cls = byte_dsfa(d)
    rng = random.Random(rx)
    alpha = bytes(sorted(set(re.sub(rb"[^a-z0-9]", b"", rx.encode())))) or b"ab"
    for _ in range(30):
        n = rng.randint(0, 60)
        w = bytes(rng.choice(alpha + b"#") for _ in range(n))
        q = run_dfa(d, w)
        for p in (1, 2, 3, 7, n + 3):
            res = sfa_parallel(s, cls, w, p)
            assert res["q_parallel"] == res["q_sequential"] == q
            assert speculative_parallel(d, w, p) == q
            for (lo, hi), f in zip(chunks_of(n, p), res["chunk_states"]):
                assert speculative_chunk(d, w[lo:hi]).tolist() == s.maps[f].tolist()


def test_chunks_cover_exactly():
    for n in (0, 1, 5, 100, 101):
        for p in (1, 2, 3, 7, 200):
            ch = chunks_of(n, p)
            assert len(ch) == p and ch[0][0] == 0 and ch[-1][1] == n
            assert all(ch[i][1] == ch[i + 1][0] for i in range(p - 1))


# --------------------------------------------------------------------------
# P11 / P12: brute force and Python's regex engine
# --------------------------------------------------------------------------
BRUTE = [("ab", 12, ["(ab)*", "(a|b)*a(a|b){2}", "(a*b*)*", "a(ba)*b?|b+", "((ab|ba){2})*", "(a{2,3}|b)+"]),
         ("abc", 8, ["(a|bc)*c?", "[ab]*c[^a]{1,2}", "(c|a(b|c)*)+", ".*abc.*"])]


@pytest.mark.parametrize("alpha,maxlen,rx", [(a, m, r) for a, m, rs in BRUTE for r in rs])
def test_bruteforce_all_short_strings(alpha, maxlen, rx):
    d = compile_regex(rx)
    ast = parse(rx)
    for n in range(maxlen + 1):
        for t in itertools.product(alpha.encode(), repeat=n):
            w = bytes(t)
            assert bool(d.accept[run_dfa(d, w)]) == matches(ast, w), (rx, w)


def test_random_regexes_against_python_re():
    rng = random.Random(7)
    checked = 0
    while checked < 120:
        rx = random_regex(rng, "abc")
        try:
            d = compile_regex(rx, max_dfa_states=500)
        except OverflowError:
            continue
        checked += 1
        pat = re.compile(rx.encode(), re.DOTALL)
        for _ in range(25):
            w = bytes(rng.choice(b"abcd\n") for _ in range(rng.randint(0, 10)))
            want = pat.fullmatch(w) is not None
            assert bool(d.accept[run_dfa(d, w)]) == want, (rx, w)
            assert matches(rx, w) == want, (rx, w)


def test_parser_rejects_what_python_rejects():
    for bad in ["*a", "a**", "(a", "a)", "[a", "[b-a]", "\\q", "a{2}{3}", "a{3,2}"]:
        with pytest.raises(ParseError):
            parse(bad)
        with pytest.raises(re.error):
            re.compile(bad.encode())


def test_escapes_and_classes_match_python():
    rng = random.Random(3)
    pats = [r"\d+\s?\w*", r"[\x00-\x1f]+", r"[^\n]*\n", r"\.\*\(", r"[]a]+", r"[a-]+", r"a{,2}b",
            r"x{2,}", r"\D\W\S", r"[\d\s]*", "a{b", r"\t\r\f\v\0"]
    for p in pats:
        d = compile_regex(p)
        pat = re.compile(p.encode(), re.DOTALL)
        for _ in range(300):
            w = bytes(rng.choice(b"ab12 \t\n.*(]-x{}\x00\x05\xff") for _ in range(rng.randint(0, 6)))
            assert bool(d.accept[run_dfa(d, w)]) == (pat.fullmatch(w) is not None), (p, w)


# --------------------------------------------------------------------------
# Minimality and canonical numbering
# --------------------------------------------------------------------------
@pytest.mark.parametrize("rx", SMALL + ["(a|b)*abb", "((a|b)(a|b))*"])
def test_minimal_states_pairwise_distinguishable(rx):
    # Myhill-Nerode by brute force: every two states are told apart by some
    # word over the class representatives.  Breadth-first over words, keeping
    # for each word the vector of states reached from every start state; stop
    # once a whole length adds no new distinction.
    d = compile_regex(rx)
    _, reps = byte_classes(d)
    n = d.n
    start = np.arange(n)
    sig = [tuple(d.accept[start].tolist())]
    frontier = {start.tobytes(): start}
    groups = len(set(zip(*sig)))
    for _ in range(n):
        nxt = {}
        for vec in frontier.values():
            for r in reps.tolist():
                v = d.delta[vec, r]
                nxt.setdefault(v.tobytes(), v)
        frontier = nxt
        for v in frontier.values():
            sig.append(tuple(d.accept[v].tolist()))
        g = len(set(zip(*sig)))
        if g == groups:
            break
        groups = g
    assert groups == n


@pytest.mark.parametrize("rx", SMALL)
def test_canonical_numbering_is_isomorphism_invariant(rx):
    d = compile_regex(rx)
    rng = np.random.default_rng(5)
    for _ in range(5):
        perm = rng.permutation(d.n)           # old -> new id
        inv = np.argsort(perm)
        shuffled = Dfa(perm[d.delta[inv]], int(perm[d.q0]), d.accept[inv])
        again = canonicalize(minimize(shuffled))
        assert np.array_equal(again.delta, d.delta) and np.array_equal(again.accept, d.accept)


def test_canonical_bfs_order_property():
    # every state other than q0 is first reached from a lower-numbered state,
    # and discovery ids increase along (state, byte) order
    for rx in SMALL:
        d = compile_regex(rx)
        nxt_new = 1
        for q in range(d.n):
            for b in range(256):
                t = int(d.delta[q, b])
                if t >= nxt_new:
                    assert t == nxt_new
                    nxt_new += 1


# --------------------------------------------------------------------------
# seqscan.c against the Python loop
# --------------------------------------------------------------------------
def test_seqscan_c_matches_python_loop():
    d = compile_regex(W.REGEX_C1)
    for seed in range(4):
        w = W.c1_input(seed, n=2000)
        assert oscan.scan(d, w) == run_dfa(d, bytes(w))
        for q in range(d.n):
            assert oscan.scan(d, w[:37], q=q) == run_dfa(d, bytes(w[:37]), q)


# --------------------------------------------------------------------------
# cpu_sfa.c (Algorithm 5 on host threads) against Example 1's D-SFA, the
# Python Algorithm 5 and Algorithm 2
# --------------------------------------------------------------------------
def test_cpu_sfa_on_example1():
    delta, _, _, _ = _example1()
    s = build_dsfa(delta, 0, np.array([True, False, False]))
    cls = np.full(256, 1, dtype=np.int64)          # every byte but 'a' acts as b
    cls[ord("a")] = 0
    t = oscan.SfaTables(s, cls)
    word = b"ab" * 7
    for p in range(1, 17):
        q, states = oscan.sfa_parallel(t, word, p)
        ref = sfa_parallel(s, cls, word, p=p)
        assert states == ref["chunk_states"], p
        assert q == ref["q_sequential"] == 0, p
    q, _ = oscan.sfa_parallel(t, word + b"a", 3)
    assert q == 1                                   # (ab)*a ends in state 1 (Table 1's DFA)


@pytest.mark.parametrize("rx", [W.REGEX_C1, W.REGEX_C2, ".*(abc|bcd|cab).*", "(a|b)*a(a|b){2}c?"])
def test_cpu_sfa_matches_sequential_dfa(rx):
    d = compile_regex(rx)
    s, cls = byte_dsfa(d)
    t = oscan.SfaTables(s, cls)
    rng = np.random.default_rng(11)
    alpha = np.frombuffer(b"0123456789abcd", dtype=np.uint8)
    for n in (0, 1, 5, 97, 4096 + 3, 100_003):
        w = (W.c1_input(3, n=n - n % 2) if rx == W.REGEX_C1 and n >= 10 else rng.choice(alpha, size=n).astype(np.uint8))
        want = oscan.scan(d, w)
        for p in (1, 2, 3, 8, 16, 33, n + 5):
            q, states = oscan.sfa_parallel(t, w, p)
            assert q == want, (rx, n, p)
            if n <= 4096 + 3 and p <= 16:
                ref = sfa_parallel(s, cls, bytes(w), p=p)
                assert states == ref["chunk_states"], (rx, n, p)
