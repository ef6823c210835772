"""Regex -> NFA -> DFA -> minimal canonical DFA (oracle, test infrastructure).

Independent of the product's host compiler: Thompson's construction (the
product uses a position automaton), subset construction over all 256 bytes
(Algorithm 1, Section 2.3) with a FIFO worklist, Moore's partition refinement
for minimisation (the experiments of Section 6.1 minimise the DFA before
building the D-SFA), and a canonical renumbering.

Canonical numbering: breadth-first search from the start state, following
bytes 0..255 in ascending order, each state numbered when first discovered.
Two minimal complete DFAs of the same language are isomorphic, so this
numbering makes their state ids equal.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np

from .regex import parse


# ---------------------------------------------------------------------------
# Thompson NFA
# ---------------------------------------------------------------------------
class Nfa:
    """NFA with epsilon moves; ``edges[q]`` lists (byte mask, target)."""

    def __init__(self):
        self.eps: list[list[int]] = []
        self.edges: list[list[tuple[int, int]]] = []
        self.start = -1
        self.final = -1

    def state(self) -> int:
        self.eps.append([])
        self.edges.append([])
        return len(self.eps) - 1

    def build(self, node) -> tuple[int, int]:
        kind = node[0]
        s = self.state()
        if kind == "eps":
            e = self.state()
            self.eps[s].append(e)
            return s, e
        if kind == "set":
            e = self.state()
            if node[1]:
                self.edges[s].append((node[1], e))
            return s, e
        if kind == "cat":
            cur = s
            for sub in node[1]:
                a, b = self.build(sub)
                self.eps[cur].append(a)
                cur = b
            return s, cur
        if kind == "alt":
            e = self.state()
            for sub in node[1]:
                a, b = self.build(sub)
                self.eps[s].append(a)
                self.eps[b].append(e)
            return s, e
        if kind == "star":
            e = self.state()
            a, b = self.build(node[1])
            self.eps[s] += [a, e]
            self.eps[b] += [a, e]
            return s, e
        if kind == "rep":
            sub, lo, hi = node[1], node[2], node[3]
            cur = s
            for _ in range(lo):
                a, b = self.build(sub)
                self.eps[cur].append(a)
                cur = b
            if hi is None:
                a, b = self.build(("star", sub))
                self.eps[cur].append(a)
                cur = b
            else:
                for _ in range(hi - lo):
                    a, b = self.build(sub)
                    e = self.state()
                    self.eps[cur] += [a, e]
                    self.eps[b].append(e)
                    cur = e
            return s, cur
        raise ValueError(kind)


def thompson(ast) -> Nfa:
    nfa = Nfa()
    nfa.start, nfa.final = nfa.build(ast)
    return nfa


# ---------------------------------------------------------------------------
# DFA
# ---------------------------------------------------------------------------
@dataclass
class Dfa:
    """Complete DFA over ``k`` symbols: ``delta[q, a]``, start ``q0``."""
    delta: np.ndarray      # (n, k) int64
    q0: int
    accept: np.ndarray     # (n,) bool

    @property
    def n(self) -> int:
        return int(self.delta.shape[0])


def subset_construction(nfa: Nfa, max_states: int = 1 << 16) -> Dfa:
    """Algorithm 1 over the 256 byte values; the empty subset is the sink."""
    closure_cache: dict[frozenset, frozenset] = {}

    def closure(states) -> frozenset:
        key = frozenset(states)
        hit = closure_cache.get(key)
        if hit is not None:
            return hit
        seen = set(key)
        stack = list(key)
        while stack:
            q = stack.pop()
            for t in nfa.eps[q]:
                if t not in seen:
                    seen.add(t)
                    stack.append(t)
        out = frozenset(seen)
        closure_cache[key] = out
        return out

    start = closure([nfa.start])
    index = {start: 0}
    order = [start]
    rows = []
    worklist = deque([start])          # Q_tmp, taken in FIFO order
    while worklist:
        S = worklist.popleft()
        by_mask: dict[int, set] = {}
        for q in S:
            for mask, t in nfa.edges[q]:
                by_mask.setdefault(mask, set()).add(t)
        row = np.empty(256, dtype=np.int64)
        for b in range(256):
            nxt = set()
            for mask, ts in by_mask.items():
                if (mask >> b) & 1:
                    nxt |= ts
            T = closure(nxt)
            j = index.get(T)
            if j is None:
                j = len(order)
                if j >= max_states:
                    raise OverflowError("DFA exceeds %d states" % max_states)
                index[T] = j
                order.append(T)
                worklist.append(T)
            row[b] = j
        rows.append(row)
    delta = np.stack(rows)
    accept = np.array([nfa.final in S for S in order], dtype=bool)
    return Dfa(delta, 0, accept)


def minimize(d: Dfa) -> Dfa:
    """Moore's algorithm: refine {accepting, rejecting} until stable.

    Two states stay together iff they agree on acceptance and, for every
    symbol, their successors are in the same block.  Assumes all states are
    reachable (true for the output of subset construction).
    """
    block = d.accept.astype(np.int64)
    nblocks = len(set(block.tolist()))
    while True:
        sig: dict[tuple, int] = {}
        new = np.empty(d.n, dtype=np.int64)
        succ = block[d.delta]
        for q in range(d.n):
            key = (int(block[q]), succ[q].tobytes())
            new[q] = sig.setdefault(key, len(sig))
        block = new
        if len(sig) == nblocks:
            break
        nblocks = len(sig)
    k = d.delta.shape[1]
    delta = np.zeros((nblocks, k), dtype=np.int64)
    accept = np.zeros(nblocks, dtype=bool)
    for q in range(d.n):
        delta[block[q]] = block[d.delta[q]]
        accept[block[q]] = d.accept[q]
    return Dfa(delta, int(block[d.q0]), accept)


def canonicalize(d: Dfa) -> Dfa:
    """Renumber states breadth-first from q0, symbols in ascending order."""
    new_id = {d.q0: 0}
    order = [d.q0]
    i = 0
    while i < len(order):
        q = order[i]
        i += 1
        for t in d.delta[q].tolist():
            if t not in new_id:
                new_id[t] = len(order)
                order.append(t)
    n = len(order)
    delta = np.empty((n, d.delta.shape[1]), dtype=np.int64)
    accept = np.empty(n, dtype=bool)
    for q_old, q_new in new_id.items():
        delta[q_new] = [new_id[t] for t in d.delta[q_old].tolist()]
        accept[q_new] = d.accept[q_old]
    return Dfa(delta, 0, accept)


def compile_regex(pattern: str, max_dfa_states: int = 1 << 16) -> Dfa:
    """Minimal complete DFA over bytes, canonically numbered (q0 = 0)."""
    nfa = thompson(parse(pattern))
    return canonicalize(minimize(subset_construction(nfa, max_dfa_states)))


def byte_classes(d: Dfa) -> tuple[np.ndarray, np.ndarray]:
    """Coarsest partition of the bytes by identical DFA columns.

    Returns (cls[256], reps[C]): class ids are ordered by the smallest byte
    of each class, and reps[c] is that smallest byte.
    """
    cls = np.empty(256, dtype=np.int64)
    seen: dict[bytes, int] = {}
    reps = []
    for b in range(256):
        key = d.delta[:, b].tobytes()
        c = seen.get(key)
        if c is None:
            c = len(reps)
            seen[key] = c
            reps.append(b)
        cls[b] = c
    return cls, np.array(reps, dtype=np.int64)


def run_dfa(d: Dfa, data: bytes, q: int | None = None) -> int:
    """Algorithm 2 in Python (small inputs): every byte is read, no early exit."""
    q = d.q0 if q is None else q
    delta = d.delta.tolist()
    for b in bytes(data):
        q = delta[q][b]
    return q
