"""Algorithm 2 (sequential DFA computation, seqscan.c) and Algorithm 5 (the
parallel SFA computation on host threads, cpu_sfa.c) over large inputs.

Test infrastructure only.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .automata import Dfa
from .build import SO, build

_lib = None


def _load():
    global _lib
    if _lib is None:
        import os
        if not os.path.exists(SO):
            build(force=False)
        lib = ctypes.CDLL(SO)
        lib.oracle_seqscan.restype = ctypes.c_uint32
        lib.oracle_seqscan.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64]
        lib.oracle_sfa_parallel.restype = ctypes.c_uint32
        lib.oracle_sfa_parallel.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p]
        _lib = lib
    return _lib


def table_u32(d: Dfa) -> np.ndarray:
    if d.delta.shape[1] != 256:
        raise ValueError("byte DFA expected")
    return np.ascontiguousarray(d.delta, dtype=np.uint32)


def scan(d: Dfa, data, q: int | None = None, table: np.ndarray | None = None) -> int:
    """Final state of the DFA after reading all of ``data`` from ``q`` (default q0)."""
    lib = _load()
    t = table_u32(d) if table is None else table
    arr = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else data,
                               dtype=np.uint8)
    q = d.q0 if q is None else q
    return int(lib.oracle_seqscan(t.ctypes.data, q, arr.ctypes.data, arr.size))


def match(d: Dfa, data) -> tuple[int, bool]:
    """(final canonical state, accept) -- the result the matcher must reproduce."""
    q = scan(d, data)
    return q, bool(d.accept[q])


class SfaTables:
    """A D-SFA (oracle.sfa.Dsfa over byte classes ``cls``) in the layout of
    cpu_sfa.c: a 256-column transition table of 32-bit ids and the mapping
    rows."""

    def __init__(self, s, cls: np.ndarray):
        cls = np.asarray(cls, dtype=np.int64)
        self.nxt = np.ascontiguousarray(np.asarray(s.nxt)[:, cls], dtype=np.uint32)   # [m, 256]
        self.maps = np.ascontiguousarray(s.maps, dtype=np.uint32)                     # [m, n]
        self.n = int(self.maps.shape[1])
        self.q0 = int(s.q0)


def sfa_parallel(t: SfaTables, data, p: int) -> tuple[int, list[int]]:
    """Algorithm 5 on p host threads (cpu_sfa.c): (final DFA state, chunk states)."""
    lib = _load()
    arr = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else data,
                               dtype=np.uint8)
    states = np.zeros(max(1, p), dtype=np.uint32)
    q = lib.oracle_sfa_parallel(t.nxt.ctypes.data, t.maps.ctypes.data, t.n, t.q0, arr.ctypes.data, arr.size,
                                p, states.ctypes.data)
    if q == 0xFFFFFFFF:
        raise MemoryError("cpu_sfa: host allocation failed")
    return int(q), states[:max(1, p)].tolist()
