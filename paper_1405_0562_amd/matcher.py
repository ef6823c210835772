"""Python face of the SFA matcher: compile, load, match.

Every step of matching runs in libsfa.so (host compiler in C++, kernels in
HIP); this module only marshals arguments.  PyTorch provides device memory
and streams.
"""
from __future__ import annotations

import ctypes
from collections import OrderedDict
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi
from ._capi import check, lib

DEFAULT_SFA_CAP = 65535


@dataclass
class CompileInfo:
    n_dfa: int
    n_sfa: int
    n_classes: int
    q0: int
    n_positions: int
    sfa_over_cap: bool
    dfa_seconds: float
    sfa_seconds: float
    sfa_lazy: bool = False


class Compiled:
    """Result of the host compiler: canonical minimal DFA and (if built) its D-SFA,
    or (``nsfa=True``) the subset automaton of the position NFA and its N-SFA."""

    def __init__(self, pattern: str, sfa_cap: int = DEFAULT_SFA_CAP, dfa_cap: int = 0, nsfa: bool = False):
        self.pattern = pattern
        self.is_nsfa = nsfa
        raw = pattern.encode("latin-1")
        h = ctypes.c_void_p()
        entry = lib().sfa_compile_nsfa if nsfa else lib().sfa_compile
        check(entry(raw, len(raw), sfa_cap, dfa_cap, ctypes.byref(h)))
        self._h = h
        self._sets = None
        self._refresh_info()

    def _refresh_info(self):
        ci = _capi.CompileInfo()
        check(lib().sfa_compiled_info(self._h, ctypes.byref(ci)))
        self.info = CompileInfo(ci.n_dfa, ci.n_sfa, ci.n_classes, ci.q0, ci.n_positions,
                                bool(ci.sfa_over_cap), ci.dfa_seconds, ci.sfa_seconds, bool(ci.sfa_lazy))

    def build_lazy(self, sample, start_every: int = 256, walk_bytes: int = 4096,
                   max_states: int = DEFAULT_SFA_CAP) -> "Compiled":
        """On-the-fly D-SFA for a compilation without one: only the states that
        runs over ``sample`` (walk_bytes each, one every start_every bytes,
        from the identity) reach are built; the rest stay unbuilt and pieces
        that reach them finish through the DFA.  Returns self."""
        x = np.ascontiguousarray(np.frombuffer(sample, dtype=np.uint8) if isinstance(sample, (bytes, bytearray))
                                 else np.asarray(sample, dtype=np.uint8))
        check(lib().sfa_compiled_build_lazy(self._h, ctypes.c_void_p(x.ctypes.data if x.size else 0), x.size,
                                            start_every, walk_bytes, max_states))
        self._refresh_info()
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().sfa_compiled_free(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    def desc(self) -> _capi.TableDesc:
        d = _capi.TableDesc()
        check(lib().sfa_compiled_desc(self._h, ctypes.byref(d)))
        return d

    def arrays(self) -> dict:
        """Copies of the host tables (for inspection and tests)."""
        d = self.desc()
        n, m, C = d.n_dfa, d.n_sfa, d.n_classes

        def arr(ptr, count, dtype):
            if count == 0 or not ptr:
                return np.zeros(0, dtype=dtype)
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)

        return {
            "byte_class": arr(d.byte_class, 256, np.int64),
            "dfa_next": arr(d.dfa_next, n * C, np.int64).reshape(n, C),
            "dfa_accept": arr(d.dfa_accept, n, np.int64).astype(bool),
            "sfa_next": arr(d.sfa_next, m * C, np.int64).reshape(m, C),
            "sfa_map": arr(d.sfa_map, m * n, np.int64).reshape(m, n),
            "q0": d.q0,
        }


    def nsfa_sets(self) -> tuple[np.ndarray, np.ndarray, int]:
        """N-SFA compilations: (sets[n_dfa, words] as uint64, final[words], n_nfa)."""
        if not self.is_nsfa:
            raise ValueError("not an N-SFA compilation")
        if self._sets is None:
            s = _capi.NsfaSets()
            check(lib().sfa_compiled_nsfa_sets(self._h, ctypes.byref(s)))
            n, w = self.info.n_dfa, s.words
            sets = np.ctypeslib.as_array(s.sets, shape=(n * w,)).copy().reshape(n, w)
            final = np.ctypeslib.as_array(s.final_set, shape=(w,)).copy()
            self._sets = (sets, final, s.n_nfa)
        return self._sets

    def nsfa_set(self, state: int) -> int:
        """The NFA states of a result state of an N-SFA match, as a bit mask."""
        sets, _, _ = self.nsfa_sets()
        return sum(int(x) << (64 * i) for i, x in enumerate(sets[state]))


def compile(pattern: str, sfa_cap: int = DEFAULT_SFA_CAP, dfa_cap: int = 0) -> Compiled:  # noqa: A001
    return Compiled(pattern, sfa_cap, dfa_cap)


def compile_nsfa(pattern: str, nsfa_cap: int = DEFAULT_SFA_CAP, dfa_cap: int = 0) -> Compiled:
    """N-SFA of the regex's position automaton (Definition 3, Algorithm 4);
    load and match it like a D-SFA compilation, then read the final NFA
    state set of a result with ``Compiled.nsfa_set(state)``."""
    return Compiled(pattern, nsfa_cap, dfa_cap, nsfa=True)


def _stream_ptr(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Table:
    """A compiled automaton resident in device memory (HBM)."""

    MAX_CALLS = 256   # prepared call shapes kept per table

    def __init__(self, compiled: Compiled, device=None, force_global: bool = False, lds_budget: int = 0,
                 renumber: int = 0, profile_sample: np.ndarray | None = None, product: bool = True, stream=None):
        self.compiled = compiled
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        desc = compiled.desc()
        sample = None if profile_sample is None else np.ascontiguousarray(profile_sample, dtype=np.uint8)
        opts = _capi.LoadOptions(int(force_global), int(lds_budget), int(renumber), int(not product),
                                 ctypes.c_void_p(sample.ctypes.data) if sample is not None else None,
                                 0 if sample is None else sample.size)
        nbytes = ctypes.c_size_t()
        check(lib().sfa_table_device_bytes(ctypes.byref(desc), ctypes.byref(opts), ctypes.byref(nbytes)))
        with torch.cuda.device(self.device):
            load_stream = torch.cuda.current_stream() if stream is None else stream
            with torch.cuda.stream(load_stream):
                self.buf = torch.empty(max(256, nbytes.value), dtype=torch.uint8, device=self.device)
            h = ctypes.c_void_p()
            check(lib().sfa_load_table(ctypes.byref(desc), ctypes.byref(opts), ctypes.c_void_p(self.buf.data_ptr()),
                                       nbytes.value, ctypes.c_void_p(_stream_ptr(load_stream)), ctypes.byref(h)))
            self._h = h
            # launches on other streams wait for the upload
            self._uploaded = torch.cuda.Event()
            self._uploaded.record(load_stream)
        self._load_stream = _stream_ptr(load_stream)
        self._synced = {self._load_stream}
        ti = _capi.TableInfo()
        check(lib().sfa_table_get_info(self._h, ctypes.byref(ti)))
        self.info = {f: getattr(ti, f) for f, _ in _capi.TableInfo._fields_}
        self._ws = {}
        self._calls = OrderedDict()   # (entry point, n, n_chunks, stream, plan) -> (fn, plan args, bytes)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().sfa_free_table(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @property
    def walkable(self) -> bool:
        """True when sfa_match can walk this table's D-SFA (else only the
        speculative matcher applies: no D-SFA within the cap, or a global
        table with more byte classes than the walk takes)."""
        return self.info["n_sfa"] > 0 and (self.info["table_in_lds"] or self.info["n_classes"] <= 128)

    def _stream_ready(self, stream) -> None:
        """Makes `stream` wait for the table upload (once per stream)."""
        sp = _stream_ptr(stream)
        if sp not in self._synced:
            (torch.cuda.current_stream() if stream is None else stream).wait_event(self._uploaded)
            self._synced.add(sp)

    def workspace(self, n: int, n_chunks: int, stream=None, need: int | None = None) -> torch.Tensor:
        """A zero-filled workspace large enough for (n, n_chunks), cached per stream.

        The kernels leave the workspace's control words zero after every
        call, so a cached workspace is reused without clearing; calls on one
        stream never overlap.  The workspace is allocated and cleared on the
        launch stream itself.
        """
        if need is None:
            nb = ctypes.c_size_t()
            check(lib().sfa_match_workspace_bytes(self._h, n, n_chunks, ctypes.byref(nb)))
            need = nb.value
        key = _stream_ptr(stream)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            with torch.cuda.stream(torch.cuda.current_stream() if stream is None else stream):
                ws = torch.zeros(max(need, 4096), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws


def load(compiled: Compiled, **kw) -> Table:
    return Table(compiled, **kw)


def _prepare(fn_name: str, table: Table, n: int, n_chunks: int, plan: dict | None):
    """Entry point, plan arguments and workspace bytes of one call shape."""
    nb = ctypes.c_size_t()
    check(lib().sfa_match_workspace_bytes(table.handle, n, n_chunks, ctypes.byref(nb)))
    if plan is None:
        return getattr(lib(), fn_name), None, nb.value
    p = _capi.Plan(*(int(plan.get(f, 0)) for f, _ in _capi.Plan._fields_))
    return lib().sfa_match_ex, p, nb.value


def _match(fn_name: str, table: Table, data: torch.Tensor, n_chunks: int, out: torch.Tensor | None, stream,
           plan: dict | None = None):
    if data.dtype != torch.uint8 or not data.is_cuda or data.dim() != 1 or not data.is_contiguous():
        raise ValueError("data must be a contiguous 1-D torch.uint8 tensor on a HIP device")
    if data.device != table.device:
        raise ValueError("data and table are on different devices")
    n = data.numel()
    sp = _stream_ptr(stream)
    key = (fn_name, n, n_chunks, sp, None if plan is None else tuple(sorted(plan.items())))
    call = table._calls.get(key)
    if call is None:
        call = table._calls[key] = _prepare(fn_name, table, n, n_chunks, plan)
        if len(table._calls) > Table.MAX_CALLS:
            table._calls.popitem(last=False)
    else:
        table._calls.move_to_end(key)
    fn, p, need = call
    table._stream_ready(stream)
    ws = table.workspace(n, n_chunks, stream, need)
    if out is None:
        with torch.cuda.stream(torch.cuda.current_stream() if stream is None else stream):
            out = torch.empty(2, dtype=torch.int32, device=table.device)
    if p is not None:
        st = fn(table.handle, data.data_ptr() if n else None, n, n_chunks, ctypes.byref(p), ws.data_ptr(), ws.numel(),
                out.data_ptr(), sp or None)
    else:
        st = fn(table.handle, data.data_ptr() if n else None, n, n_chunks, ws.data_ptr(), ws.numel(),
                out.data_ptr(), sp or None)
    check(st)
    return out


def match(table: Table, data: torch.Tensor, n_chunks: int = 0, out: torch.Tensor | None = None,
          stream=None, plan: dict | None = None) -> torch.Tensor:
    """Algorithm 5 on the device; returns int32[2] = (final state, accept) on the device.

    ``plan`` (optional) is a dict with any of the sfa_plan fields ("stride", "pieces",
    "load_bytes", "depth", "block_threads", "lanes_per_chunk").  A table
    without a walkable D-SFA (none within the state cap, or a global table
    with more than 128 byte classes) is matched by the speculative kernel
    (Algorithm 3) instead, with the same result.
    """
    if not table.walkable:
        if plan is not None:
            raise ValueError("a launch plan applies to the D-SFA walk; this table has no walkable D-SFA")
        return _match("sfa_match_speculative", table, data, n_chunks, out, stream)
    return _match("sfa_match", table, data, n_chunks, out, stream, plan)


def stream_read(data: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """The streaming-read reference kernel: reads ``data`` (uint8, 16-byte
    aligned, on the device) once and XORs its 32-bit words into ``out``
    (one int32 on the device).  Used to measure the read-only HBM rate."""
    if data.dtype != torch.uint8 or not data.is_cuda or not data.is_contiguous():
        raise ValueError("data must be a contiguous torch.uint8 tensor on the GPU")
    if out.dtype != torch.int32 or not out.is_cuda or out.numel() < 1:
        raise ValueError("out must be an int32 tensor on the GPU")
    check(lib().sfa_stream_read(ctypes.c_void_p(data.data_ptr()), data.numel(), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(_stream_ptr(stream))))
    return out


def match_speculative(table: Table, data: torch.Tensor, n_chunks: int = 0, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
    """Algorithm 3 on the device; same result as ``match``."""
    return _match("sfa_match_speculative", table, data, n_chunks, out, stream)
