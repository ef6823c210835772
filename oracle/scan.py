"""Algorithm 2 (sequential DFA computation) over large inputs via seqscan.c.

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
