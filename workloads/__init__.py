"""Seeded synthetic workloads for SFA regular-expression matching.

This module only draws bytes and regex strings from seeded generators.  It
holds none of the matching arithmetic (no automata, no transition tables), so
both the CPU oracle (``oracle/``) and the HIP path may use it without sharing
any part of the method.

Every generator takes an explicit ``seed`` and uses numpy's PCG64 generator,
so a (workload, seed) pair always produces the same bytes on any machine.

Workloads (sizes follow the paper's experiments and the single-stream,
batched and served forms built here):

* ``c1``: the overhead experiment's regex shape (Section 6.3), with the digit
  ranges of the scalability regexes r_n (Section 6.2):
  ``(([0-4][5-9]){5})*`` over ~1 MiB of strings from the language, with one
  byte replaced with probability 1/2 so that accept and reject both occur.
* ``c2``: ``(a|b)*a(a|b){4}`` over uniform bytes from {a, b}; 256 MiB by
  default (a k-th-from-last DFA with 33 complete states).
* ``c3``: ``.*(w1|...|w20).*`` with 20 seeded 8-letter lowercase keywords over
  uniform bytes from ``a..z`` plus space, keywords planted at a per-byte rate.
* ``c4``: documents with lognormal lengths over a 32-symbol alphabet, and
  8 seeded regexes from three families whose minimal DFA sizes are known in
  closed form (keyword search, k-th from last, counted cycles).
* ``c5``: request streams with Pareto lengths over 16 regexes of the same
  families, with Poisson arrival times.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "REGEX_C1", "REGEX_C2", "C1_N", "C2_N", "C3_N",
    "rng_for", "c1_input", "c2_input", "c3_keywords", "c3_regex", "c3_input",
    "uniform_over", "ALPHABET_C4", "family_regex", "c4_regexes", "c4_doc_lengths",
    "c4_docs", "c5_regexes", "c5_requests", "Request", "rn_regex", "ra_regex", "rn_input",
]

REGEX_C1 = "(([0-4][5-9]){5})*"
REGEX_C2 = "(a|b)*a(a|b){4}"

# Every word of REGEX_C1 has a length that is a multiple of 10, so the input
# is the largest multiple of 10 not above 1 MiB.
C1_N = 10 * ((1 << 20) // 10)        # 1,048,570 bytes
C2_N = 1 << 28                        # 256 MiB
C3_N = 1 << 32                        # 4 GiB

ALPHABET_C3 = b"abcdefghijklmnopqrstuvwxyz "
ALPHABET_C4 = b"abcdefghijklmnopqrstuvwxyz012345"


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """Independent PCG64 stream for (seed, stream)."""
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def rn_regex(n: int) -> str:
    """The scalability regex r_n of Section 6.2: ([0-4]{n}[5-9]{n})*."""
    return "([0-4]{%d}[5-9]{%d})*" % (n, n)


def ra_regex(n: int) -> str:
    """r_n | a*, the variant of Section 6.2 run on an all-'a' text."""
    return rn_regex(n) + "|a*"


def uniform_over(rng: np.random.Generator, alphabet: bytes, n: int,
                 block: int = 1 << 26) -> np.ndarray:
    """n bytes drawn uniformly and independently from ``alphabet``."""
    alpha = np.frombuffer(alphabet, dtype=np.uint8)
    out = np.empty(n, dtype=np.uint8)
    k = len(alpha)
    if k == 2:
        # one random bit per byte, drawn 8 at a time
        for lo in range(0, n, block):
            hi = min(n, lo + block)
            m = hi - lo
            raw = np.frombuffer(rng.bytes((m + 7) // 8), dtype=np.uint8)
            bits = np.unpackbits(raw)[:m]
            out[lo:hi] = alpha[bits]
        return out
    for lo in range(0, n, block):
        hi = min(n, lo + block)
        idx = rng.integers(0, k, size=hi - lo, dtype=np.uint8)
        out[lo:hi] = alpha[idx]
    return out


def rn_input(seed: int, n: int, size: int) -> np.ndarray:
    """A word of r_n: ``size // (2n)`` blocks of n uniform digits from 0-4
    followed by n uniform digits from 5-9 (the accepted texts of the
    scalability experiment, Section 6.2)."""
    blocks = size // (2 * n)
    rng = rng_for(seed, 11)
    out = np.empty(blocks * 2 * n, dtype=np.uint8)
    view = out.reshape(blocks, 2, n)
    step = max(1, (1 << 26) // (2 * n))
    for lo in range(0, blocks, step):
        hi = min(blocks, lo + step)
        view[lo:hi] = rng.integers(0, 5, size=(hi - lo, 2, n), dtype=np.uint8) + np.array([48, 53], np.uint8)[None, :, None]
    return out


def c1_input(seed: int, n: int = C1_N) -> np.ndarray:
    """Strings of (([0-4][5-9]){5})*: n/2 pairs (low digit, high digit).

    With probability 1/2 one uniformly chosen position is replaced by a
    uniformly chosen *different* byte value (0..255), which usually makes the
    word leave the language.
    """
    if n % 2:
        raise ValueError("c1 input length must be even")
    rng = rng_for(seed, 1)
    pairs = n // 2
    lo = rng.integers(ord("0"), ord("4") + 1, size=pairs, dtype=np.uint8)
    hi = rng.integers(ord("5"), ord("9") + 1, size=pairs, dtype=np.uint8)
    out = np.empty(n, dtype=np.uint8)
    out[0::2] = lo
    out[1::2] = hi
    if n and rng.random() < 0.5:
        pos = int(rng.integers(0, n))
        delta = int(rng.integers(1, 256))
        out[pos] = (int(out[pos]) + delta) & 0xFF
    return out


def c2_input(seed: int, n: int = C2_N) -> np.ndarray:
    """n bytes uniform over {a, b}."""
    return uniform_over(rng_for(seed, 2), b"ab", n)


def c3_keywords(seed: int, count: int = 20, length: int = 8) -> list[bytes]:
    """``count`` keywords of ``length`` letters, each uniform over a..z."""
    rng = rng_for(seed, 3)
    letters = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz", dtype=np.uint8)
    return [bytes(letters[rng.integers(0, 26, size=length)]) for _ in range(count)]


def c3_regex(keywords: list[bytes]) -> str:
    return ".*(" + "|".join(k.decode() for k in keywords) + ").*"


def c3_input(seed: int, n: int, keywords: list[bytes], rate: float = 1e-6) -> np.ndarray:
    """Uniform bytes over a..z and space, with keywords planted.

    Each byte position independently starts a plant with probability
    ``rate``; a plant overwrites the next len(keyword) bytes with a keyword
    chosen uniformly (plants that would run past the end are dropped).
    """
    rng = rng_for(seed, 4)
    out = uniform_over(rng, ALPHABET_C3, n)
    if rate > 0 and keywords:
        klen = len(keywords[0])
        count = int(rng.binomial(n, rate))
        if count and n > klen:
            pos = np.sort(rng.integers(0, n - klen, size=count))
            which = rng.integers(0, len(keywords), size=count)
            for p, w in zip(pos.tolist(), which.tolist()):
                out[p:p + klen] = np.frombuffer(keywords[w], dtype=np.uint8)
    return out


# ---------------------------------------------------------------------------
# Batched / served workloads: regex families with closed-form DFA sizes.
# ---------------------------------------------------------------------------

def _escape_symbol(b: int) -> str:
    c = chr(b)
    return c if c.isalnum() else "\\x%02x" % b


def _class_of(symbols: np.ndarray) -> str:
    return "[" + "".join(_escape_symbol(int(b)) for b in sorted(set(symbols.tolist()))) + "]"


def family_regex(rng: np.random.Generator, family: int, alphabet: bytes = ALPHABET_C4) -> str:
    """One regex from a family whose minimal DFA size is known in closed form.

    family 0, keyword search ``.*w.*`` with |w| = 7..15
        (|w| + 1 minimal DFA states);
    family 1, k-th from last ``.*x.{m}`` with m = 2..5
        (2^(m+1) states);
    family 2, counted cycle ``(([A][B]){k})*`` with disjoint random symbol
        classes A and B and k = 4..31 (2k + 1 states with the sink).
    """
    alpha = np.frombuffer(alphabet, dtype=np.uint8)
    if family == 0:
        ln = int(rng.integers(7, 16))
        w = alpha[rng.integers(0, len(alpha), size=ln)]
        return ".*" + "".join(_escape_symbol(int(b)) for b in w) + ".*"
    if family == 1:
        m = int(rng.integers(2, 6))
        x = int(alpha[rng.integers(0, len(alpha))])
        return ".*" + _escape_symbol(x) + ".{%d}" % m
    if family == 2:
        k = int(rng.integers(4, 32))
        perm = rng.permutation(alpha)
        na = int(rng.integers(1, len(alpha) // 2))
        nb = int(rng.integers(1, len(alpha) // 2))
        a, b = perm[:na], perm[na:na + nb]
        return "((%s%s){%d})*" % (_class_of(a), _class_of(b), k)
    raise ValueError(family)


def c4_regexes(seed: int, count: int = 8) -> list[str]:
    rng = rng_for(seed, 5)
    return [family_regex(rng, i % 3) for i in range(count)]


def c4_doc_lengths(seed: int, n_docs: int = 10_000, median: int = 4096,
                   sigma: float = 2.0, max_len: int = 16 << 20) -> np.ndarray:
    """Lognormal lengths (median ``median``), clipped to [1, max_len]."""
    rng = rng_for(seed, 6)
    x = rng.lognormal(mean=math.log(median), sigma=sigma, size=n_docs)
    return np.clip(np.rint(x), 1, max_len).astype(np.int64)


def c4_docs(seed: int, n_docs: int = 10_000, **kw) -> tuple[np.ndarray, np.ndarray]:
    """Concatenated documents and their offsets ``off[n_docs + 1]``."""
    lens = c4_doc_lengths(seed, n_docs, **kw)
    off = np.zeros(n_docs + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    data = uniform_over(rng_for(seed, 7), ALPHABET_C4, int(off[-1]))
    return data, off


def c5_regexes(seed: int, count: int = 16) -> list[str]:
    rng = rng_for(seed, 8)
    return [family_regex(rng, i % 3) for i in range(count)]


@dataclass
class Request:
    arrival_s: float      # arrival time relative to the start of the stream
    table: int            # index into the regex list
    data: np.ndarray      # uint8 bytes


def c5_requests(seed: int, n_req: int, qps: float, n_tables: int = 16,
                alpha: float = 1.2, xm: int = 1024, max_len: int = 64 << 20) -> list[Request]:
    """Poisson arrivals at ``qps``; Pareto(alpha, xm) lengths truncated at max_len."""
    rng = rng_for(seed, 9)
    gaps = rng.exponential(1.0 / qps, size=n_req)
    t = np.cumsum(gaps)
    u = rng.random(n_req)
    lens = np.minimum(np.floor(xm / np.power(1.0 - u, 1.0 / alpha)), max_len).astype(np.int64)
    tables = rng.integers(0, n_tables, size=n_req)
    out = []
    drng = rng_for(seed, 10)
    for i in range(n_req):
        out.append(Request(float(t[i]), int(tables[i]),
                           uniform_over(drng, ALPHABET_C4, int(lens[i]))))
    return out
