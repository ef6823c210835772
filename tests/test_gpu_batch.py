"""GPU parity of the batched form against the oracle, job by job.

Each job (document, regex) is checked bit-exactly against the oracle's own
DFA run over the document (Algorithm 2 in plain C).  Covers all-pairs batches
of the batching workload at reduced size, random job lists (duplicates, empty
and unaligned documents, a subset of tables per document), jobs long enough
to span work items, tables read from global memory, and graph replay.
"""
import functools

import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle.automata import compile_regex
from oracle import scan as oscan

pytestmark = pytest.mark.gpu

sfa = pytest.importorskip("paper_1405_0562_amd")


def say(*a):
    print("[gpu-case]", *a, flush=True)


@functools.lru_cache(maxsize=None)
def oracle_dfa(rx):
    d = compile_regex(rx)
    return d, oscan.table_u32(d)


def oracle_jobs(regexes, data, doc_off, jobs):
    out = np.empty((len(jobs), 2), dtype=np.int64)
    for i, (d, t) in enumerate(jobs):
        dfa, tab = oracle_dfa(regexes[t])
        q = oscan.scan(dfa, data[doc_off[d]:doc_off[d + 1]], table=tab)
        out[i] = (q, int(dfa.accept[q]))
    return out


@functools.lru_cache(maxsize=None)
def tables_for(regexes):
    return [sfa.load(sfa.compile(rx)) for rx in regexes]


def small_docs(seed, n_docs, max_len=1 << 18):
    lens = np.minimum(W.c4_doc_lengths(seed, n_docs), max_len)
    off = np.zeros(n_docs + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    data = W.uniform_over(W.rng_for(seed, 7), W.ALPHABET_C4, int(off[-1]))
    return data, off


def run_batch(regexes, data, off, jobs, **opt):
    tabs = tables_for(tuple(regexes))
    say("batch", len(regexes), "tables", len(off) - 1, "docs", len(jobs), "jobs", opt)
    b = sfa.Batch(tabs, off, jobs, sfa.BatchOptions(**opt))
    x = torch.from_numpy(data).cuda() if data.size else torch.empty(0, dtype=torch.uint8, device="cuda")
    got = b.run(x).cpu().numpy()
    return got, b


@pytest.mark.parametrize("piece", [1024, 4096])
def test_all_pairs_reduced_batch_workload(piece):
    regexes = W.c4_regexes(0)
    data, off = small_docs(1, 300)
    jobs = np.array([(d, t) for d in range(300) for t in range(len(regexes))], dtype=np.uint32)
    got, b = run_batch(regexes, data, off, jobs, piece_bytes=piece)
    want = oracle_jobs(regexes, data, off, jobs)
    assert np.array_equal(got, want)
    assert b.info["tables_in_lds"] == 1


def test_random_jobs_duplicates_empty_and_unaligned_docs():
    rng = np.random.default_rng(5)
    regexes = W.c5_regexes(1)
    lens = rng.integers(0, 5000, size=120)
    lens[::17] = 0
    off = np.zeros(121, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    off[1:] += 3                      # every document starts 3 bytes into the buffer (unaligned)
    off[0] = 3
    data = W.uniform_over(W.rng_for(6, 7), W.ALPHABET_C4, int(off[-1]))
    jobs = np.stack([rng.integers(0, 120, size=700), rng.integers(0, len(regexes), size=700)], axis=1).astype(np.uint32)
    for units in (1, 2, 4):
        got, _ = run_batch(regexes, data, off, jobs, piece_bytes=256, units_per_lane=units)
        assert np.array_equal(got, oracle_jobs(regexes, data, off, jobs))


def test_jobs_spanning_work_items():
    """Jobs whose pieces lie in several work items: per-item mappings and one
    arrival per item, with pieces less than an item apart (few jobs per
    document) and more than an item apart (more jobs per document than units
    per item)."""
    regexes = W.c4_regexes(2)[:4]
    lens = np.array([1, 100, 70_000, 300_000, 5, 131_072, 0, 4099], dtype=np.int64)
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    data = W.uniform_over(W.rng_for(9, 7), W.ALPHABET_C4, int(off[-1]))
    x = torch.from_numpy(data).cuda()
    few = np.array([(d, t) for d in range(len(lens)) for t in range(4)], dtype=np.uint32)
    many = np.array([(d, j % 4) for d in range(len(lens)) for j in range(70)], dtype=np.uint32)
    for jobs in (few, many):
        want = oracle_jobs(regexes, data, off, jobs)
        for units in (1, 2, 4):
            got, b = run_batch(regexes, data, off, jobs, piece_bytes=128, units_per_lane=units)
            assert b.info["n_item_map_entries"] > 0
            assert np.array_equal(got, want), (jobs.shape, units)
            # the arrival counters reset themselves: the same workspace serves again
            for _ in range(3):
                assert np.array_equal(b.run(x).cpu().numpy(), want)


def test_global_tables_and_c1_c2_regexes():
    regexes = [W.REGEX_C1, W.REGEX_C2, "(ab)*", ".*\\xff.*"]
    rng = np.random.default_rng(3)
    parts = [W.c1_input(1, n=10_000), W.c2_input(2, n=9_999), np.frombuffer(b"ab" * 500, dtype=np.uint8),
             rng.integers(0, 256, size=4097, dtype=np.uint8)]
    data = np.concatenate(parts)
    off = np.concatenate([[0], np.cumsum([p.size for p in parts])])
    jobs = np.array([(d, t) for d in range(4) for t in range(4)], dtype=np.uint32)
    for fg in (False, True):
        got, b = run_batch(regexes, data, off, jobs, force_global=fg)
        assert b.info["tables_in_lds"] == (0 if fg else 1)
        assert np.array_equal(got, oracle_jobs(regexes, data, off, jobs))


def test_batch_matches_single_stream_path():
    regexes = W.c4_regexes(3)
    data, off = small_docs(4, 40)
    jobs = np.array([(d, t) for d in range(40) for t in range(len(regexes))], dtype=np.uint32)
    got, _ = run_batch(regexes, data, off, jobs)
    tabs = tables_for(tuple(regexes))
    x = torch.from_numpy(data).cuda()
    for i, (d, t) in enumerate(jobs):
        single = sfa.match(tabs[t], x[off[d]:off[d + 1]].contiguous()).tolist()
        assert single == got[i].tolist()


def graph_node_types(graph):
    """Node types of a captured graph (0 = kernel), through the HIP runtime."""
    hip = ctypes.CDLL("libamdhip64.so")
    raw = graph.raw_cuda_graph()
    if not isinstance(raw, int):   # a capsule around the pointer
        get = ctypes.pythonapi.PyCapsule_GetPointer
        get.restype, get.argtypes = ctypes.c_void_p, [ctypes.py_object, ctypes.c_char_p]
        raw = get(raw, None)
    g = ctypes.c_void_p(raw)
    n = ctypes.c_size_t(0)
    assert hip.hipGraphGetNodes(g, None, ctypes.byref(n)) == 0
    nodes = (ctypes.c_void_p * n.value)()
    assert hip.hipGraphGetNodes(g, nodes, ctypes.byref(n)) == 0
    types = []
    for nd in nodes:
        t = ctypes.c_int(-1)
        assert hip.hipGraphNodeGetType(ctypes.c_void_p(nd), ctypes.byref(t)) == 0
        types.append(t.value)
    return types


def test_graph_replay_with_new_data():
    regexes = W.c4_regexes(4)
    data, off = small_docs(8, 100)
    jobs = np.array([(d, t) for d in range(100) for t in range(len(regexes))], dtype=np.uint32)
    tabs = tables_for(tuple(regexes))
    b = sfa.Batch(tabs, off, jobs)
    x = torch.from_numpy(data).cuda()
    g = sfa.GraphBatch(b, x)
    assert graph_node_types(g.graph) == [0]      # one node, a kernel: the whole batch is one launch
    for rep in range(3):
        new = W.uniform_over(W.rng_for(100 + rep, 7), W.ALPHABET_C4, data.size)
        g.data.copy_(torch.from_numpy(new))
        torch.cuda.synchronize()
        say("graph replay", rep)
        got = g.replay().cpu().numpy()
        eager = b.run(g.data).cpu().numpy()          # eager work between replays
        want = oracle_jobs(regexes, new, off, jobs)
        assert np.array_equal(got, want)
        assert np.array_equal(eager, want)


def test_autotuner_picks_a_valid_option(tmp_path):
    regexes = W.c4_regexes(5)[:3]
    data, off = small_docs(10, 60)
    jobs = np.array([(d, t) for d in range(60) for t in range(3)], dtype=np.uint32)
    tabs = tables_for(tuple(regexes))
    x = torch.from_numpy(data).cuda()
    tuner = sfa.Autotuner(cache_path=str(tmp_path / "tune.json"), reps=1)
    opt, entry = tuner.tune(tabs, x, off, jobs)
    assert opt.piece_bytes in sfa.Autotuner.PIECES and len(entry["trials"]) == 30
    assert {t["force_global"] for t in entry["trials"]} == {False, True}   # LDS and L2 placement both timed
    b = sfa.Batch(tabs, off, jobs, opt)
    assert np.array_equal(b.run(x).cpu().numpy(), oracle_jobs(regexes, data, off, jobs))
    opt2, _ = sfa.Autotuner(cache_path=str(tmp_path / "tune.json")).tune(tabs, x, off, jobs)
    assert opt2 == opt
