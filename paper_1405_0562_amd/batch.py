"""Batched matching: many (document, table) jobs in one persistent launch.

``Batch`` wraps one host plan (sfa_batch_create) and its device workspace;
``Batch.run`` only enqueues the batch kernel (sfa_match_batch, one launch),
so it can be captured into a HIP graph (``GraphBatch``) and replayed.  ``Autotuner`` picks
the piece length and pieces per lane for a batch shape by timing candidates
on the device and caches the choice on disk.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi
from ._capi import check, lib
from .matcher import Table, _stream_ptr


@dataclass(frozen=True)
class BatchOptions:
    piece_bytes: int = 0      # 0 = library default (4096)
    units_per_lane: int = 0   # 0 = library default (2)
    force_global: bool = False


class Batch:
    """A planned batch: tables x documents -> jobs, with its device workspace.

    ``doc_off`` holds n_docs + 1 byte offsets into the data tensor passed to
    ``run``; ``jobs`` is an (n_jobs, 2) array of (document, table index).
    """

    def __init__(self, tables: list[Table], doc_off, jobs, options: BatchOptions = BatchOptions(), stream=None,
                 ws: torch.Tensor | None = None, out: torch.Tensor | None = None):
        if not tables:
            raise ValueError("at least one table is required")
        self.tables = list(tables)
        self.device = self.tables[0].device
        self.doc_off = np.ascontiguousarray(np.asarray(doc_off, dtype=np.uint64))
        self.jobs = np.ascontiguousarray(np.asarray(jobs, dtype=np.uint32).reshape(-1, 2))
        self.options = options
        n_docs = self.doc_off.size - 1
        if n_docs < 0:
            raise ValueError("doc_off needs n_docs + 1 entries")
        handles = (ctypes.c_void_p * len(self.tables))(*[t.handle.value for t in self.tables])
        opts = _capi.BatchOptions(options.piece_bytes, 0, options.units_per_lane, int(options.force_global))
        h = ctypes.c_void_p()
        check(lib().sfa_batch_create(handles, len(self.tables), ctypes.c_void_p(self.doc_off.ctypes.data), n_docs,
                                     ctypes.c_void_p(self.jobs.ctypes.data), self.jobs.shape[0],
                                     ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        info = _capi.BatchInfo()
        check(lib().sfa_batch_get_info(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _capi.BatchInfo._fields_}
        # a caller's workspace and output buffers are used when they are large
        # enough (a server keeps them per stream, so no launch allocates)
        need = max(256, self.info["workspace_bytes"])
        with torch.cuda.device(self.device):
            if ws is not None and ws.dtype == torch.uint8 and ws.numel() >= need and ws.data_ptr() % 256 == 0:
                self.ws = ws
            else:
                self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            if out is not None and out.dtype == torch.int32 and out.shape[0] >= self.jobs.shape[0]:
                self.out = out[:self.jobs.shape[0]]
            else:
                self.out = torch.empty((self.jobs.shape[0], 2), dtype=torch.int32, device=self.device)
            check(lib().sfa_batch_upload(self._h, ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                         ctypes.c_void_p(_stream_ptr(stream))))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().sfa_batch_free(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    @property
    def n_jobs(self) -> int:
        return int(self.jobs.shape[0])

    def run(self, data: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Enqueue the batch on ``stream``; returns int32 (n_jobs, 2) = (state, accept)."""
        if data.dtype != torch.uint8 or data.device != self.device or not data.is_contiguous():
            raise ValueError("data must be a contiguous torch.uint8 tensor on the tables' device")
        if data.numel() < int(self.doc_off[-1]):
            raise ValueError("data is shorter than the last document offset")
        out = self.out if out is None else out
        check(lib().sfa_match_batch(self._h, ctypes.c_void_p(data.data_ptr() if data.numel() else 0),
                                    ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream_ptr(stream))))
        return out


class GraphBatch:
    """A batch captured once into a HIP graph and replayed.

    The graph holds only the batch kernel (no memset, no allocation); the
    data tensor is captured by address, so new document bytes are copied into
    ``self.data`` before each replay.
    """

    def __init__(self, batch: Batch, data: torch.Tensor):
        self.batch = batch
        self.data = data
        self.graph = torch.cuda.CUDAGraph(keep_graph=True)   # the captured graph stays inspectable
        side = torch.cuda.Stream(device=batch.device)
        side.wait_stream(torch.cuda.current_stream(batch.device))
        with torch.cuda.stream(side):
            batch.run(self.data, stream=side)          # warm-up outside the capture
        torch.cuda.current_stream(batch.device).wait_stream(side)
        torch.cuda.synchronize(batch.device)
        with torch.cuda.graph(self.graph):
            batch.run(self.data)
        self.graph.instantiate()

    def replay(self) -> torch.Tensor:
        self.graph.replay()
        return self.batch.out


def match_batch(tables: list[Table], data: torch.Tensor, doc_off, jobs, options: BatchOptions = BatchOptions(),
                stream=None) -> torch.Tensor:
    """One-shot batch: plan, upload, run; returns (n_jobs, 2) int32 on the device."""
    b = Batch(tables, doc_off, jobs, options, stream=stream)
    out = b.run(data, stream=stream)
    # keep the plan (and its workspace) alive until the stream has used them
    torch.cuda.current_stream(b.device).synchronize() if stream is None else stream.synchronize()
    return out.clone()


def shape_key(tables: list[Table], doc_off, jobs) -> str:
    """Autotune cache key: device, table shapes and a length histogram."""
    lens = np.diff(np.asarray(doc_off, dtype=np.int64))
    hist = np.bincount(np.clip(np.log2(np.maximum(lens, 1)).astype(int), 0, 40), minlength=41)
    props = torch.cuda.get_device_properties(tables[0].device)
    sig = {
        "device": props.name, "cus": props.multi_processor_count,
        "tables": [(t.info["n_dfa"], t.info["n_sfa"], t.info["n_classes"]) for t in tables],
        "jobs": int(np.asarray(jobs).reshape(-1, 2).shape[0]),
        "hist": (hist / max(1, hist.sum())).round(2).tolist(),
    }
    return hashlib.sha1(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:16]


class Autotuner:
    """Times candidate batch options on the device and remembers the best.

    Candidates cover the piece length (work per lane, balance between long and
    short documents), pieces per lane (ILP vs lane count) and the placement
    of the walk tables (staged in LDS by every block, or read through L1/L2
    from global memory).  Results are cached in a JSON file keyed by
    ``shape_key``.
    """

    PIECES = (1024, 2048, 4096, 8192, 16384)
    UNITS = (1, 2, 4)
    PLACEMENTS = (False, True)   # force_global

    def __init__(self, cache_path: str | None = None, reps: int = 3):
        self.cache_path = cache_path or os.path.join(os.path.expanduser("~"), ".cache", "paper_1405_0562_amd",
                                                     "autotune.json")
        self.reps = reps
        self.cache = {}
        if os.path.exists(self.cache_path):
            try:
                with open(self.cache_path) as fh:
                    self.cache = json.load(fh)
            except (OSError, ValueError):
                self.cache = {}

    def _save(self):
        try:
            os.makedirs(os.path.dirname(self.cache_path), exist_ok=True)
            with open(self.cache_path, "w") as fh:
                json.dump(self.cache, fh, indent=1)
        except OSError:
            pass

    def time_options(self, tables, data, doc_off, jobs, options: BatchOptions) -> float:
        b = Batch(tables, doc_off, jobs, options)
        b.run(data)
        torch.cuda.synchronize(b.device)
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(self.reps):
            b.run(data)
        end.record()
        torch.cuda.synchronize(b.device)
        return start.elapsed_time(end) / self.reps

    def tune(self, tables, data, doc_off, jobs, force: bool = False) -> tuple[BatchOptions, dict]:
        key = shape_key(tables, doc_off, jobs)
        if key in self.cache and not force:
            c = self.cache[key]
            return BatchOptions(c["piece_bytes"], c["units_per_lane"], bool(c.get("force_global", False))), c
        trials = []
        for glob in self.PLACEMENTS:
            for piece in self.PIECES:
                for units in self.UNITS:
                    opt = BatchOptions(piece, units, glob)
                    ms = self.time_options(tables, data, doc_off, jobs, opt)
                    trials.append({"piece_bytes": piece, "units_per_lane": units, "force_global": glob, "ms": ms})
        best = min(trials, key=lambda t: t["ms"])
        entry = dict(best, trials=trials)
        self.cache[key] = entry
        self._save()
        return BatchOptions(best["piece_bytes"], best["units_per_lane"], best["force_global"]), entry
