"""Byte-regex parser and a direct language matcher (oracle, test infrastructure).

Syntax (the regex language every component accepts):

* alphabet: the 256 byte values; the pattern is ASCII text;
* ``.`` matches any byte, newline included;
* ``[...]`` / ``[^...]`` byte sets with ranges ``a-z``; ``]`` first is a
  literal, ``-`` first or last is a literal; escapes allowed inside;
* escapes: ``\\n \\t \\r \\f \\v \\0 \\xHH``, the ASCII classes
  ``\\d \\D \\w \\W \\s \\S``, and a backslash before any non-alphanumeric
  character makes it literal;
* grouping ``( )``, alternation ``|`` (empty alternatives allowed),
  repetition ``*``, ``+``, ``?``, ``{n}``, ``{n,}``, ``{,m}``, ``{n,m}``
  (a ``{`` that does not start a valid bound is a literal);
* stacked quantifiers (``a**``, ``a*?``) and a quantifier with nothing before
  it are errors;
* matching is whole-input membership, as in the definition of the accepted
  language (Section 2.2); a search is written with explicit ``.*``.

AST nodes are tuples:
``('eps',)``, ``('set', mask)`` (bit b of the int ``mask`` = byte b),
``('cat', [nodes])``, ``('alt', [nodes])``, ``('star', node)``,
``('rep', node, lo, hi)`` with ``hi = None`` for no upper bound.
"""
from __future__ import annotations

from functools import lru_cache

ALL = (1 << 256) - 1
MAX_REPEAT = 1000


class ParseError(ValueError):
    pass


def _mask_of(chars) -> int:
    m = 0
    for c in chars:
        m |= 1 << c
    return m


_DIGIT = _mask_of(range(ord("0"), ord("9") + 1))
_WORD = _mask_of(list(range(ord("a"), ord("z") + 1)) + list(range(ord("A"), ord("Z") + 1))
                 + list(range(ord("0"), ord("9") + 1)) + [ord("_")])
_SPACE = _mask_of(b" \t\n\r\f\v")
_CLASS_ESC = {"d": _DIGIT, "D": ALL & ~_DIGIT, "w": _WORD, "W": ALL & ~_WORD,
              "s": _SPACE, "S": ALL & ~_SPACE}
_CHAR_ESC = {"n": 10, "t": 9, "r": 13, "f": 12, "v": 11, "0": 0}


class _Parser:
    def __init__(self, text: str):
        self.s = text
        self.i = 0

    def peek(self):
        return self.s[self.i] if self.i < len(self.s) else None

    def take(self):
        c = self.peek()
        if c is None:
            raise ParseError("unexpected end of pattern")
        self.i += 1
        return c

    # escape after a backslash: returns ('byte', b) or ('mask', m)
    def escape(self):
        c = self.take()
        if c in _CLASS_ESC:
            return ("mask", _CLASS_ESC[c])
        if c in _CHAR_ESC:
            return ("byte", _CHAR_ESC[c])
        if c == "x":
            h = self.s[self.i:self.i + 2]
            if len(h) != 2 or any(ch not in "0123456789abcdefABCDEF" for ch in h):
                raise ParseError("bad \\x escape at %d" % self.i)
            self.i += 2
            return ("byte", int(h, 16))
        if c.isalnum():
            raise ParseError("unknown escape \\%s" % c)
        if ord(c) > 127:
            raise ParseError("non-ASCII pattern character")
        return ("byte", ord(c))

    def bracket(self) -> int:
        neg = False
        if self.peek() == "^":
            neg = True
            self.i += 1
        mask = 0
        first = True
        while True:
            c = self.peek()
            if c is None:
                raise ParseError("unterminated [")
            if c == "]" and not first:
                self.i += 1
                break
            first = False
            lo = self._bracket_item()
            if self.peek() == "-" and self.i + 1 < len(self.s) and self.s[self.i + 1] != "]":
                self.i += 1
                hi = self._bracket_item()
                if lo[0] != "byte" or hi[0] != "byte":
                    raise ParseError("class escape in a range")
                if hi[1] < lo[1]:
                    raise ParseError("reversed range")
                mask |= _mask_of(range(lo[1], hi[1] + 1))
            else:
                mask |= (1 << lo[1]) if lo[0] == "byte" else lo[1]
        return (ALL & ~mask) if neg else mask

    def _bracket_item(self):
        c = self.take()
        if c == "\\":
            return self.escape()
        if ord(c) > 127:
            raise ParseError("non-ASCII pattern character")
        return ("byte", ord(c))

    def alt(self):
        branches = [self.concat()]
        while self.peek() == "|":
            self.i += 1
            branches.append(self.concat())
        return branches[0] if len(branches) == 1 else ("alt", branches)

    def concat(self):
        items = []
        while self.peek() is not None and self.peek() not in "|)":
            items.append(self.repeat())
        if not items:
            return ("eps",)
        return items[0] if len(items) == 1 else ("cat", items)

    def bound(self):
        """Parse {n}, {n,}, {,m}, {n,m} at self.i (pointing at '{'), or None."""
        j = self.i + 1
        s = self.s

        def digits(k):
            e = k
            while e < len(s) and s[e].isdigit():
                e += 1
            return e

        e1 = digits(j)
        lo_txt = s[j:e1]
        if e1 < len(s) and s[e1] == "}":
            if not lo_txt:
                return None
            self.i = e1 + 1
            n = int(lo_txt)
            return n, n
        if e1 < len(s) and s[e1] == ",":
            e2 = digits(e1 + 1)
            hi_txt = s[e1 + 1:e2]
            if e2 < len(s) and s[e2] == "}":
                if not lo_txt and not hi_txt:
                    return None
                self.i = e2 + 1
                lo = int(lo_txt) if lo_txt else 0
                hi = int(hi_txt) if hi_txt else None
                return lo, hi
        return None

    def repeat(self):
        node = self.atom()
        quantified = False
        while True:
            c = self.peek()
            if c in ("*", "+", "?"):
                q = (0, None) if c == "*" else (1, None) if c == "+" else (0, 1)
                self.i += 1
            elif c == "{":
                q = self.bound()
                if q is None:
                    break
            else:
                break
            if quantified:
                raise ParseError("multiple repeat at %d" % self.i)
            quantified = True
            lo, hi = q
            if hi is not None and hi < lo:
                raise ParseError("bad repeat bounds")
            if lo > MAX_REPEAT or (hi is not None and hi > MAX_REPEAT):
                raise ParseError("repeat bound too large")
            node = ("star", node) if (lo, hi) == (0, None) else ("rep", node, lo, hi)
        return node

    def atom(self):
        c = self.take()
        if c == "(":
            node = self.alt()
            if self.peek() != ")":
                raise ParseError("missing )")
            self.i += 1
            return node
        if c in "*+?":
            raise ParseError("nothing to repeat at %d" % (self.i - 1))
        if c == "{":
            self.i -= 1
            if self.bound() is not None:
                raise ParseError("nothing to repeat at %d" % self.i)
            self.i += 1
            return ("set", 1 << ord("{"))
        if c == ")":
            raise ParseError("unbalanced )")
        if c == ".":
            return ("set", ALL)
        if c == "[":
            return ("set", self.bracket())
        if c == "\\":
            kind, v = self.escape()
            return ("set", (1 << v) if kind == "byte" else v)
        if ord(c) > 127:
            raise ParseError("non-ASCII pattern character")
        return ("set", 1 << ord(c))


def parse(pattern: str):
    """Parse ``pattern`` into an AST (raises ParseError)."""
    p = _Parser(pattern)
    node = p.alt()
    if p.i != len(pattern):
        raise ParseError("unbalanced ) at %d" % p.i)
    return node


def _ends(node, s: bytes, i: int) -> frozenset:
    """All j such that s[i:j] is in the language of ``node``.

    Written from the meaning of each construct (a byte set reads one byte,
    concatenation chains, alternation unions, star is the least fixed point of
    zero or more repetitions); no automaton is involved.
    """
    kind = node[0]
    if kind == "eps":
        return frozenset((i,))
    if kind == "set":
        return frozenset((i + 1,)) if i < len(s) and (node[1] >> s[i]) & 1 else frozenset()
    if kind == "cat":
        cur = {i}
        for sub in node[1]:
            nxt = set()
            for k in cur:
                nxt |= _ends(sub, s, k)
            cur = nxt
            if not cur:
                break
        return frozenset(cur)
    if kind == "alt":
        out = set()
        for sub in node[1]:
            out |= _ends(sub, s, i)
        return frozenset(out)
    if kind == "star":
        seen = {i}
        frontier = [i]
        while frontier:
            k = frontier.pop()
            for j in _ends(node[1], s, k):
                if j not in seen:
                    seen.add(j)
                    frontier.append(j)
        return frozenset(seen)
    if kind == "rep":
        sub, lo, hi = node[1], node[2], node[3]
        cur = {i}
        for _ in range(lo):
            nxt = set()
            for k in cur:
                nxt |= _ends(sub, s, k)
            cur = nxt
        if hi is None:
            return _star_from(sub, s, cur)
        out = set(cur)
        for _ in range(hi - lo):
            nxt = set()
            for k in cur:
                nxt |= _ends(sub, s, k)
            cur = nxt - out
            out |= nxt
            if not cur:
                break
        return frozenset(out)
    raise ValueError(kind)


def _star_from(sub, s, starts) -> frozenset:
    seen = set(starts)
    frontier = list(starts)
    while frontier:
        k = frontier.pop()
        for j in _ends(sub, s, k):
            if j not in seen:
                seen.add(j)
                frontier.append(j)
    return frozenset(seen)


def matches(pattern_or_ast, data: bytes) -> bool:
    """Whole-input membership of ``data`` in the language (no automata).

    Cost grows quickly with input length: for short strings only.
    """
    ast = parse(pattern_or_ast) if isinstance(pattern_or_ast, str) else pattern_or_ast
    return len(data) in _ends(ast, bytes(data), 0)
