"""N-SFA oracle (test infrastructure only): the SFA built from an NFA.

Only the tests, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg use this module; the product never imports it.

* ``glushkov``: the position automaton (McNaughton-Yamada / Glushkov, the
  NFA the paper's construction starts from, Section 6.1).  State 0 is the
  initial state; states 1..P are the byte-set leaves of the regex in left to
  right order, with a bounded repeat r{lo,hi} written out as lo copies of r
  followed by hi - lo optional copies (or one starred copy when hi is
  unbounded).  From the definitions: first, last, follow and nullable.
* ``nfa_run``: the NFA's sequential computation -- the set of states reached
  from I (the plain definition of a run; Section 2.2).
* ``build_nsfa``: Algorithm 4 (correspondence construction, Section 5.1) on
  the NFA: states are mappings Q -> P(Q), stored as one bit mask per NFA
  state; delta_s(f, s)(q) is the union of delta(q', s) over q' in f(q).
  FIFO worklist, byte classes ascending, identity = state 0.
* ``compose``: reverse composition on correspondences, (f . g)(q) = union of
  g(p) over p in f(q) (Section 2.1).
* ``nsfa_parallel``: Algorithm 5 -- chunk walks from f_I, ordered
  composition, S_fin = union of f_fin(q) over q in I.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .regex import parse


class OverCap(RuntimeError):
    pass


@dataclass
class Nfa:
    """Epsilon-free NFA: state 0 initial; sets[p] is the byte mask of position p."""
    sets: list = field(default_factory=lambda: [0])
    first: frozenset = frozenset()
    follow: list = field(default_factory=lambda: [set()])
    last: frozenset = frozenset()
    nullable: bool = True

    @property
    def n(self) -> int:
        return len(self.sets)

    @property
    def initial(self) -> int:
        return 1                                   # mask of I = {0}

    @property
    def final(self) -> int:
        m = 1 if self.nullable else 0
        for p in self.last:
            m |= 1 << p
        return m

    def successors(self, q: int) -> set:
        return set(self.first) if q == 0 else self.follow[q]

    def delta(self, q: int, b: int) -> int:
        """Mask of the states reached from q on byte b."""
        m = 0
        for p in self.successors(q):
            if (self.sets[p] >> b) & 1:
                m |= 1 << p
        return m


def glushkov(pattern_or_ast) -> Nfa:
    ast = parse(pattern_or_ast) if isinstance(pattern_or_ast, str) else pattern_or_ast
    a = Nfa()

    def build(node):
        """(nullable, first, last) of node; allocates its positions in order."""
        kind = node[0]
        if kind == "eps":
            return True, frozenset(), frozenset()
        if kind == "set":
            p = len(a.sets)
            a.sets.append(node[1])
            a.follow.append(set())
            return False, frozenset([p]), frozenset([p])
        if kind == "cat":
            acc = (True, frozenset(), frozenset())
            for kid in node[1]:
                acc = cat(acc, build(kid))
            return acc
        if kind == "alt":
            nul, fi, la = False, frozenset(), frozenset()
            for kid in node[1]:
                n2, f2, l2 = build(kid)
                nul, fi, la = nul or n2, fi | f2, la | l2
            return nul, fi, la
        if kind == "star":
            return star(build(node[1]))
        if kind == "rep":
            _, sub, lo, hi = node
            acc = (True, frozenset(), frozenset())
            for _ in range(lo):
                acc = cat(acc, build(sub))
            if hi is None:
                acc = cat(acc, star(build(sub)))
            else:
                for _ in range(hi - lo):
                    _, f2, l2 = build(sub)
                    acc = cat(acc, (True, f2, l2))
            return acc
        raise ValueError(kind)

    def cat(x, y):
        nx, fx, lx = x
        ny, fy, ly = y
        for p in lx:                       # every last of x is followed by every first of y
            a.follow[p] |= fy
        return nx and ny, fx | fy if nx else fx, ly | lx if ny else ly

    def star(x):
        _, fx, lx = x
        for p in lx:
            a.follow[p] |= fx
        return True, fx, lx

    a.nullable, a.first, a.last = build(ast)
    return a


def nfa_byte_classes(a: Nfa) -> tuple[np.ndarray, list[int]]:
    """Bytes grouped by their membership in every position's set (bytes of a
    class have identical transitions from every state); classes numbered by
    smallest member byte.  Returns (cls[256], representative byte per class)."""
    sig = {}
    cls = np.zeros(256, dtype=np.int64)
    reps = []
    for b in range(256):
        key = tuple((s >> b) & 1 for s in a.sets[1:])
        if key not in sig:
            sig[key] = len(reps)
            reps.append(b)
        cls[b] = sig[key]
    return cls, reps


def nfa_run(a: Nfa, data: bytes, start: int | None = None) -> int:
    """Mask of the states reached from ``start`` (default I) after ``data``."""
    s = a.initial if start is None else start
    for b in data:
        t = 0
        q = 0
        m = s
        while m:
            if m & 1:
                t |= a.delta(q, b)
            m >>= 1
            q += 1
        s = t
    return s


def accepts(a: Nfa, data: bytes) -> bool:
    return bool(nfa_run(a, data) & a.final)


@dataclass
class Nsfa:
    nfa: Nfa
    maps: list            # maps[i] = tuple of masks, maps[i][q] = f_i(q)
    next: np.ndarray      # [m, C]
    cls: np.ndarray       # [256]

    @property
    def m(self) -> int:
        return len(self.maps)

    def accepting(self, i: int) -> bool:
        """F_s: some initial state's image meets F."""
        return bool(apply_initial(self.nfa, self.maps[i]) & self.nfa.final)


def build_nsfa(a: Nfa, cap: int | None = None) -> Nsfa:
    cls, reps = nfa_byte_classes(a)
    n = a.n
    # column of each class: delta(q, representative byte)
    cols = [[a.delta(q, b) for q in range(n)] for b in reps]
    ident = tuple(1 << q for q in range(n))
    index = {ident: 0}
    maps = [ident]
    rows = []
    work = deque([0])
    while work:
        i = work.popleft()
        f = maps[i]
        row = []
        for c in range(len(reps)):
            col = cols[c]
            g = []
            for q in range(n):
                m, t, p = f[q], 0, 0
                while m:
                    if m & 1:
                        t |= col[p]
                    m >>= 1
                    p += 1
                g.append(t)
            g = tuple(g)
            j = index.get(g)
            if j is None:
                if cap is not None and len(maps) >= cap:
                    raise OverCap("N-SFA has more than %d states" % cap)
                j = index[g] = len(maps)
                maps.append(g)
                work.append(j)
            row.append(j)
        rows.append((i, row))
    nxt = np.zeros((len(maps), len(reps)), dtype=np.int64)
    for i, row in rows:
        nxt[i] = row
    return Nsfa(a, maps, nxt, cls)


def compose(f, g) -> tuple:
    """Reverse composition of correspondences: (f . g)(q) = U_{p in f(q)} g(p)."""
    out = []
    for m in f:
        t, p = 0, 0
        while m:
            if m & 1:
                t |= g[p]
            m >>= 1
            p += 1
        out.append(t)
    return tuple(out)


def apply_initial(a: Nfa, f) -> int:
    """S = U_{q in I} f(q) (the last step of Algorithm 5)."""
    s, m, q = 0, a.initial, 0
    while m:
        if m & 1:
            s |= f[q]
        m >>= 1
        q += 1
    return s


def nsfa_walk(s: Nsfa, data: bytes, state: int = 0) -> int:
    for b in data:
        state = int(s.next[state, s.cls[b]])
    return state


def nsfa_parallel(s: Nsfa, data: bytes, p: int | None = None, bounds=None) -> tuple[int, bool]:
    """Algorithm 5 on an N-SFA: (mask of S_fin, accept)."""
    from .sfa import chunks_of
    if bounds is None:
        bounds = chunks_of(len(data), p or 1)
    f = s.maps[0]
    for lo, hi in bounds:
        f = compose(f, s.maps[nsfa_walk(s, data[lo:hi])])
    fin = apply_initial(s.nfa, f)
    return fin, bool(fin & s.nfa.final)
