"""ctypes declarations of the C ABI in include/sfa.h (argument marshalling only).

The shared library is built in-tree (``paper_1405_0562_amd/libsfa.so``); if
it is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfa.so")

SFA_ABI_VERSION = 2

STATUS = {
    0: "SFA_OK", 1: "SFA_ERR_INVALID_ARG", 2: "SFA_ERR_PARSE", 3: "SFA_ERR_DFA_TOO_LARGE",
    4: "SFA_ERR_OVER_CAP", 5: "SFA_ERR_NO_DEVICE", 6: "SFA_ERR_UNSUPPORTED_ARCH",
    7: "SFA_ERR_BUFFER_TOO_SMALL", 8: "SFA_ERR_HIP", 9: "SFA_ERR_NO_SFA", 10: "SFA_ERR_HOST_ALLOC",
}


class SfaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class ParseError(SfaError, ValueError):
    pass


class CompileInfo(ctypes.Structure):
    _fields_ = [("n_dfa", ctypes.c_uint32), ("n_sfa", ctypes.c_uint32), ("n_classes", ctypes.c_uint32),
                ("q0", ctypes.c_uint32), ("n_positions", ctypes.c_uint32), ("sfa_over_cap", ctypes.c_uint32),
                ("dfa_seconds", ctypes.c_double), ("sfa_seconds", ctypes.c_double),
                ("sfa_lazy", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class TableDesc(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("n_dfa", ctypes.c_uint32), ("n_sfa", ctypes.c_uint32),
                ("n_classes", ctypes.c_uint32), ("q0", ctypes.c_uint32),
                ("byte_class", ctypes.POINTER(ctypes.c_uint8)),
                ("dfa_next", ctypes.POINTER(ctypes.c_uint32)),
                ("dfa_accept", ctypes.POINTER(ctypes.c_uint8)),
                ("sfa_next", ctypes.POINTER(ctypes.c_uint32)),
                ("sfa_map", ctypes.POINTER(ctypes.c_uint32))]


class LoadOptions(ctypes.Structure):
    _fields_ = [("force_global", ctypes.c_uint32), ("lds_budget", ctypes.c_uint32),
                ("renumber", ctypes.c_uint32), ("no_product", ctypes.c_uint32),
                ("profile_sample", ctypes.c_void_p), ("profile_bytes", ctypes.c_uint64)]


class NsfaSets(ctypes.Structure):
    _fields_ = [("n_nfa", ctypes.c_uint32), ("words", ctypes.c_uint32),
                ("sets", ctypes.POINTER(ctypes.c_uint64)), ("final_set", ctypes.POINTER(ctypes.c_uint64))]


class TableInfo(ctypes.Structure):
    _fields_ = [("n_dfa", ctypes.c_uint32), ("n_sfa", ctypes.c_uint32), ("n_classes", ctypes.c_uint32),
                ("q0", ctypes.c_uint32), ("next_bytes", ctypes.c_uint32), ("map_bytes", ctypes.c_uint32),
                ("table_in_lds", ctypes.c_uint32), ("hot_rows", ctypes.c_uint32),
                ("strides", ctypes.c_uint32), ("product_table", ctypes.c_uint32),
                ("device_bytes", ctypes.c_uint64), ("partial", ctypes.c_uint32), ("vector_redo", ctypes.c_uint32)]


class Plan(ctypes.Structure):
    _fields_ = [("stride", ctypes.c_uint32), ("pieces", ctypes.c_uint32), ("load_bytes", ctypes.c_uint32),
                ("depth", ctypes.c_uint32), ("block_threads", ctypes.c_uint32), ("lanes_per_chunk", ctypes.c_uint32)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("piece_bytes", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("units_per_lane", ctypes.c_uint32), ("force_global", ctypes.c_uint32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_jobs", ctypes.c_uint32), ("n_docs", ctypes.c_uint32), ("n_units", ctypes.c_uint64),
                ("n_item_map_entries", ctypes.c_uint64), ("piece_bytes", ctypes.c_uint32),
                ("units_per_lane", ctypes.c_uint32), ("tables_in_lds", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("workspace_bytes", ctypes.c_uint64)]


_P = ctypes.c_void_p
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t

# name -> (restype, argtypes); exactly the functions declared in include/sfa.h
SIGNATURES = {
    "sfa_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sfa_last_error": (ctypes.c_char_p, []),
    "sfa_abi_version": (_U32, []),
    "sfa_compile": (ctypes.c_int, [ctypes.c_char_p, _SZ, _U32, _U32, ctypes.POINTER(_P)]),
    "sfa_compiled_info": (ctypes.c_int, [_P, ctypes.POINTER(CompileInfo)]),
    "sfa_compile_nsfa": (ctypes.c_int, [ctypes.c_char_p, _SZ, _U32, _U32, ctypes.POINTER(_P)]),
    "sfa_compiled_nsfa_sets": (ctypes.c_int, [_P, ctypes.POINTER(NsfaSets)]),
    "sfa_compiled_free": (None, [_P]),
    "sfa_compiled_desc": (ctypes.c_int, [_P, ctypes.POINTER(TableDesc)]),
    "sfa_compiled_build_lazy": (ctypes.c_int, [_P, _P, _U64, _U32, _U32, _U32]),
    "sfa_table_device_bytes": (ctypes.c_int, [ctypes.POINTER(TableDesc), ctypes.POINTER(LoadOptions),
                                              ctypes.POINTER(_SZ)]),
    "sfa_load_table": (ctypes.c_int, [ctypes.POINTER(TableDesc), ctypes.POINTER(LoadOptions), _P, _SZ, _P,
                                      ctypes.POINTER(_P)]),
    "sfa_table_get_info": (ctypes.c_int, [_P, ctypes.POINTER(TableInfo)]),
    "sfa_free_table": (ctypes.c_int, [_P]),
    "sfa_match_workspace_bytes": (ctypes.c_int, [_P, _U64, _U32, ctypes.POINTER(_SZ)]),
    "sfa_match": (ctypes.c_int, [_P, _P, _U64, _U32, _P, _SZ, _P, _P]),
    "sfa_match_speculative": (ctypes.c_int, [_P, _P, _U64, _U32, _P, _SZ, _P, _P]),
    "sfa_match_noalloc": (ctypes.c_int, [_P, _P, _U64, _U32, _P, _P]),
    "sfa_match_ex": (ctypes.c_int, [_P, _P, _U64, _U32, ctypes.POINTER(Plan), _P, _SZ, _P, _P]),
    "sfa_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), _U32, _P, _U32, _P, _U32,
                                        ctypes.POINTER(BatchOptions), ctypes.POINTER(_P)]),
    "sfa_batch_get_info": (ctypes.c_int, [_P, ctypes.POINTER(BatchInfo)]),
    "sfa_batch_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(_SZ)]),
    "sfa_batch_upload": (ctypes.c_int, [_P, _P, _SZ, _P]),
    "sfa_match_batch": (ctypes.c_int, [_P, _P, _P, _SZ, _P, _P]),
    "sfa_batch_free": (None, [_P]),
    "sfa_stream_read": (ctypes.c_int, [_P, _U64, _P, _P]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libsfa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsfa.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.sfa_abi_version() != SFA_ABI_VERSION:
            raise RuntimeError("libsfa.so ABI version mismatch")
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != 0:
        msg = lib().sfa_last_error().decode(errors="replace")
        cls = ParseError if status == 2 else SfaError
        raise cls(status, msg)
