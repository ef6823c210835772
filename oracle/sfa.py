"""D-SFA construction and parallel SFA / speculative DFA runs (oracle).

Test infrastructure only.  Notation follows the paper:

* a D-SFA state is a transformation f: Q -> Q of the DFA's states, stored
  as a tuple ``f[q]`` (Definition 3 with singleton images);
* reverse composition (Section 2.1): (f . g)(q) = g(f(q)), i.e. apply f
  first, then g;
* the D-SFA transition on symbol a is f -> f . delta^a, which for a DFA is
  f_next(q) = delta(f(q), a) (Algorithm 4 with the deterministic
  simplification of Section 5.1);
* the start state is the identity f_I; F_s = {f : f(q0) is accepting}.

Worklist order in Algorithm 4 is not fixed by the paper; this oracle takes
mappings first-in first-out, symbols in ascending order, the identity as id 0.
The *set* of states does not depend on that order.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np

from .automata import Dfa, byte_classes


class OverCap(RuntimeError):
    pass


@dataclass
class Dsfa:
    maps: np.ndarray       # (m, n): maps[s, q] = f_s(q)
    nxt: np.ndarray        # (m, k): D-SFA transition on symbol a
    accept: np.ndarray     # (m,) bool: f_s(q0) accepting
    q0: int

    @property
    def m(self) -> int:
        return int(self.maps.shape[0])


def build_dsfa(delta: np.ndarray, q0: int, accept: np.ndarray, cap: int | None = None) -> Dsfa:
    """Correspondence construction (Algorithm 4) for a DFA given as delta[q, a].

    ``delta`` has one column per symbol; for a byte DFA pass one
    representative column per byte class (``byte_dsfa``), since bytes with
    identical columns have identical bound transitions delta^a and hence
    identical D-SFA transitions.
    """
    delta = np.asarray(delta, dtype=np.int64)
    n, k = delta.shape
    cols = [delta[:, a].copy() for a in range(k)]   # delta^a as arrays
    ident = np.arange(n, dtype=np.int64)
    ids = {ident.tobytes(): 0}
    maps = [ident]
    rows = []
    work = deque([0])
    while work:
        s = work.popleft()
        f = maps[s]
        row = []
        for a in range(k):
            g = cols[a][f]                    # f_next(q) = delta(f(q), a)
            key = g.tobytes()
            t = ids.get(key)
            if t is None:
                t = len(maps)
                if cap is not None and t >= cap:
                    raise OverCap("D-SFA exceeds %d states" % cap)
                ids[key] = t
                maps.append(g)
                work.append(t)
            row.append(t)
        rows.append((s, row))
    m = len(maps)
    nxt = np.empty((m, k), dtype=np.int64)
    for s, row in rows:
        nxt[s] = row
    M = np.stack(maps)
    acc = np.asarray(accept, dtype=bool)[M[:, q0]]
    return Dsfa(M, nxt, acc, q0)


def byte_dsfa(d: Dfa, cap: int | None = None) -> tuple[Dsfa, np.ndarray]:
    """D-SFA of a byte DFA over its byte classes; returns (dsfa, cls[256])."""
    cls, reps = byte_classes(d)
    return build_dsfa(d.delta[:, reps], d.q0, d.accept, cap), cls


def compose(f, g) -> np.ndarray:
    """Reverse composition f . g := g o f (Section 2.1)."""
    return np.asarray(g)[np.asarray(f)]


def paper_counts(d: Dfa, s: Dsfa) -> tuple[int, int]:
    """(|D|, |S_d|) without the sink and without the all-sink mapping.

    The experiment captions of Section 6 count states this way; Example 1
    (Table 1) counts the sink and the constant-sink mapping f_3.
    """
    sinks = [q for q in range(d.n) if not d.accept[q] and np.all(d.delta[q] == q)]
    nd = d.n - len(sinks)
    ns = s.m
    for z in sinks:
        if np.any(np.all(s.maps == z, axis=1)):
            ns -= 1
    return nd, ns


# ---------------------------------------------------------------------------
# Algorithm 5 (parallel SFA computation) and Algorithm 3 (speculative DFA)
# written as plain sequential loops over the chunks.  Small inputs only.
# ---------------------------------------------------------------------------

def chunks_of(n: int, p: int) -> list[tuple[int, int]]:
    """Split [0, n) into p chunks [c*L, min((c+1)*L, n)), L = ceil(n/p)."""
    L = -(-n // p) if n else 0
    return [(min(c * L, n), min((c + 1) * L, n)) for c in range(p)]


def sfa_walk(s: Dsfa, cls: np.ndarray, data: bytes, state: int = 0) -> int:
    """f_i <- delta_s[f_i, sigma] for each byte, from ``state`` (f_I = 0)."""
    nxt = s.nxt.tolist()
    cl = cls.tolist()
    for b in bytes(data):
        state = nxt[state][cl[b]]
    return state


def sfa_parallel(s: Dsfa, cls: np.ndarray, data: bytes, p: int | None = None,
                 bounds: list[tuple[int, int]] | None = None) -> dict:
    """Algorithm 5: per-chunk walks from f_I, then both reductions.

    The chunks are ``chunks_of(len(data), p)`` or the explicit ``bounds``
    (any division of the word is allowed, Theorem 2).

    Returns the chunk states, the parallel-reduction result f_fin(q0) (a tree
    over the chunk mappings in text order) and the sequential-reduction
    result (q <- f_i(q) for i = 1..p starting from q0).
    """
    data = bytes(data)
    if bounds is None:
        bounds = chunks_of(len(data), p)
    fs = [sfa_walk(s, cls, data[a:b]) for a, b in bounds]
    level = [s.maps[f] for f in fs]
    while len(level) > 1:
        nxt = [compose(level[i], level[i + 1]) for i in range(0, len(level) - 1, 2)]
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    q_par = int(level[0][s.q0]) if level else s.q0
    q_seq = s.q0
    for f in fs:
        q_seq = int(s.maps[f][q_seq])
    return {"chunk_states": fs, "q_parallel": q_par, "q_sequential": q_seq}


def speculative_chunk(d: Dfa, data: bytes) -> np.ndarray:
    """Algorithm 3 for one chunk: T[q] <- delta(T[q], sigma) for all q."""
    T = np.arange(d.n, dtype=np.int64)
    for b in bytes(data):
        T = d.delta[T, b]
    return T


def speculative_parallel(d: Dfa, data: bytes, p: int) -> int:
    """Algorithm 3 with sequential reduction: q <- T_i[q] for i = 1..p."""
    data = bytes(data)
    q = d.q0
    for a, b in chunks_of(len(data), p):
        q = int(speculative_chunk(d, data[a:b])[q])
    return q
