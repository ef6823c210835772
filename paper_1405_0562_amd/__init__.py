"""MI355X-native data-parallel regular-expression matching with simultaneous
finite automata (Sin'ya, Matsuzaki, Sassa, ICPP 2013).

    import paper_1405_0562_amd as sfa
    c = sfa.compile("(a|b)*a(a|b){4}")        # host: regex -> DFA -> D-SFA
    t = sfa.load(c)                            # tables into HBM
    state, accept = sfa.match(t, x).tolist()   # x: torch.uint8 on the GPU

The matcher is libsfa.so (C ABI in include/sfa.h); this package binds it.
"""
from ._capi import SfaError, ParseError, lib  # noqa: F401
from .matcher import Compiled, Table, compile, compile_nsfa, load, match, match_speculative, stream_read  # noqa: F401
from .batch import Autotuner, Batch, BatchOptions, GraphBatch, match_batch  # noqa: F401
