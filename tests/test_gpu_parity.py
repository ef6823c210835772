"""GPU parity: the HIP matcher (through the C ABI) against the CPU oracle.

Bit-exact comparison of (final canonical DFA state, accept) on seeded
synthetic inputs: the oracle builds its own DFA from the regex and runs
Algorithm 2 in plain C; the GPU path uses the product's host compiler and
kernels.  Covers every workload at oracle-friendly sizes plus the full sizes
of the single-stream workloads in the launch configuration the benchmark
times, and the edge cases (empty and tiny inputs, ragged tails, unaligned
base pointers, more chunks than bytes, all byte values, global-memory tables,
tables without a D-SFA).
"""
import functools

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


def oracle_result(rx, data):
    d, tab = oracle_dfa(rx)
    q = oscan.scan(d, data, table=tab)
    return [q, int(d.accept[q])]


@functools.lru_cache(maxsize=None)
def gpu_table(rx, force_global=False, sfa_cap=65535):
    c = sfa.compile(rx, sfa_cap=sfa_cap)
    return sfa.load(c, force_global=force_global)


def to_device(data: np.ndarray, offset: int = 0) -> torch.Tensor:
    n = data.size
    buf = torch.empty(n + offset + 16, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + n]
    if n:
        view.copy_(torch.from_numpy(np.ascontiguousarray(data)))
    return view


def run(rx, data, n_chunks=0, offset=0, speculative=False, force_global=False, sfa_cap=65535, x=None):
    t = gpu_table(rx, force_global, sfa_cap)
    say(rx[:40], "n=%d" % data.size, "chunks=%d" % n_chunks, "off=%d" % offset,
        "spec" if speculative else "sfa", "global" if force_global else "")
    if x is None:
        x = to_device(data, offset)
    fn = sfa.match_speculative if speculative else sfa.match
    out = fn(t, x, n_chunks=n_chunks)
    return out.tolist()


def check(rx, data, **kw):
    got = run(rx, data, **kw)
    want = oracle_result(rx, data)
    assert got == want, (rx, data.size, kw, got, want)
    return got


# --------------------------------------------------------------------------
# single-stream workloads
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(16))
def test_c1_all_seeds(seed):
    data = W.c1_input(seed)
    got = check(W.REGEX_C1, data, n_chunks=256)
    check(W.REGEX_C1, data, n_chunks=256, speculative=True)
    assert got[1] in (0, 1)


def test_c1_accept_and_reject_both_occur():
    res = {oracle_result(W.REGEX_C1, W.c1_input(s))[1] for s in range(16)}
    assert res == {0, 1}


@pytest.mark.parametrize("n_chunks", [0, 1, 7, 256, 4096, 65536])
def test_c2_reduced(n_chunks):
    data = W.c2_input(3, n=(1 << 22) + 13)
    check(W.REGEX_C2, data, n_chunks=n_chunks)
    check(W.REGEX_C2, data, n_chunks=n_chunks, speculative=True)


@pytest.mark.parametrize("seed", [0, 1])
def test_c2_full_size_bench_config(seed):
    data = W.c2_input(seed)                       # 256 MiB
    x = to_device(data)
    want = oracle_result(W.REGEX_C2, data)
    assert run(W.REGEX_C2, data, n_chunks=65536, x=x) == want
    assert run(W.REGEX_C2, data, n_chunks=65536, speculative=True, x=x) == want
    assert run(W.REGEX_C2, data, n_chunks=0, x=x) == want
    # closed form: accept iff the fifth byte from the end is 'a'
    assert want[1] == int(data[-5] == ord("a"))


def test_c3_reduced_with_and_without_plants():
    kws = W.c3_keywords(0)
    rx = W.c3_regex(kws)
    for rate in (0.0, 2e-6):
        data = W.c3_input(5, 1 << 24, kws, rate=rate)
        check(rx, data, n_chunks=0)
        check(rx, data, n_chunks=4096, speculative=True)
        check(rx, data, n_chunks=1000, force_global=True)


def test_c3_over_cap_uses_speculative():
    kws = W.c3_keywords(1)
    rx = W.c3_regex(kws)
    data = W.c3_input(6, 1 << 20, kws, rate=1e-5)
    t = gpu_table(rx, False, 1000)
    assert t.info["n_sfa"] == 0 and not t.walkable
    # match() falls back to the speculative kernel by itself
    check(rx, data, sfa_cap=1000)
    check(rx, data, speculative=True, sfa_cap=1000)
    # the C entry point itself reports the missing D-SFA
    ws = t.workspace(data.size, 0)
    out = torch.empty(2, dtype=torch.int32, device="cuda")
    x = to_device(data)
    assert sfa.lib().sfa_match(t.handle, x.data_ptr(), data.size, 0, ws.data_ptr(), ws.numel(),
                               out.data_ptr(), None) == 9
    with pytest.raises(ValueError):
        sfa.match(t, x, plan=dict(pieces=2))


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------
EDGE_RX = ["(ab)*", W.REGEX_C1, W.REGEX_C2, ".*\\xff.*", "[\\x80-\\xff]*", "(.{3})*x?"]


@pytest.mark.parametrize("rx", EDGE_RX)
def test_edge_lengths_and_chunk_counts(rx):
    rng = np.random.default_rng(abs(hash(rx)) % 1000)
    for n in [0, 1, 2, 15, 16, 17, 255, 4095, 4096, 4097, 65537]:
        data = rng.integers(0, 256, size=n, dtype=np.uint8)
        if rx in ("(ab)*", W.REGEX_C2):
            data = np.frombuffer((b"ab" * (n // 2 + 1))[:n], dtype=np.uint8).copy()
        for p in [0, 1, 2, 3, 255, 256, 257, n + 5]:
            if p > 1 << 20:
                continue
            check(rx, data, n_chunks=p)
        check(rx, data, n_chunks=3, speculative=True)


@pytest.mark.parametrize("offset", range(1, 16))
def test_unaligned_base(offset):
    data = W.c2_input(offset, n=100_003)
    check(W.REGEX_C2, data, n_chunks=97, offset=offset)
    check(W.REGEX_C2, data, n_chunks=97, offset=offset, speculative=True)
    check(W.REGEX_C1, W.c1_input(offset, n=50_000), n_chunks=33, offset=offset)


@pytest.mark.parametrize("offset", [0, 1, 7, 15])
def test_ragged_sizes_rounded_chunks_and_shifted_boundaries(offset):
    # the walk rounds the chunk length up to whole load steps and moves the
    # boundaries back by the base's misalignment: sizes and chunk counts that
    # are not powers of two, on every plan family, against the sequential scan
    for rx, data in ((W.REGEX_C2, W.c2_input(30 + offset, n=(1 << 22) + 12_345)),
                     (W.REGEX_C1, W.c1_input(30 + offset, n=(1 << 21) + 4_002))):
        want = oracle_result(rx, data)
        x = to_device(data, offset)
        c = sfa.compile(rx)
        for t in (sfa.load(c), sfa.load(c, force_global=True), sfa.load(c, product=False)):
            for n_chunks in (0, 7, 1000, 4093, 65535, 65536, 131071):
                say(rx[:20], "offset", offset, "chunks", n_chunks, t.info)
                assert sfa.match(t, x, n_chunks=n_chunks).tolist() == want, (rx, offset, n_chunks, t.info)
        t = sfa.load(c)
        for plan in (dict(pieces=1, load_bytes=128, depth=2, block_threads=512, lanes_per_chunk=2),
                     dict(pieces=2, load_bytes=128, depth=4), dict(stride=1, pieces=8, load_bytes=32, depth=2)):
            for n_chunks in (1000, 65535):
                assert sfa.match(t, x, n_chunks=n_chunks, plan=plan).tolist() == want, (rx, offset, plan)


def test_all_byte_values_and_early_sink():
    rng = np.random.default_rng(9)
    data = rng.integers(0, 256, size=1 << 20, dtype=np.uint8)
    for rx in [".*\\x00\\xff.*", "[^\\x7f]*", W.REGEX_C1, "(\\d|\\s|\\w)*"]:
        check(rx, data, n_chunks=512)
        check(rx, data, n_chunks=512, speculative=True)


def test_forced_global_table_and_lds_table_agree():
    data = W.c2_input(11, n=3_000_001)
    a = check(W.REGEX_C2, data, n_chunks=2048, force_global=True)
    b = check(W.REGEX_C2, data, n_chunks=2048)
    assert a == b
    assert gpu_table(W.REGEX_C2, True).info["table_in_lds"] == 0
    assert gpu_table(W.REGEX_C2, False).info["table_in_lds"] == 1


def test_rn_and_all_a_text():
    rx = W.ra_regex(20)
    data = np.full(1 << 22, ord("a"), dtype=np.uint8)
    check(rx, data)
    check(W.rn_regex(20), (np.arange(1 << 20) // 20 % 2 * 5 + 48 + np.arange(1 << 20) % 5).astype(np.uint8))


def test_workspace_reuse_across_sizes():
    t = gpu_table(W.REGEX_C1)
    for seed, n in [(1, 1_000_000), (2, 1000), (3, 500_000), (4, 0), (5, 10)]:
        data = W.c1_input(seed, n=n)
        assert run(W.REGEX_C1, data, n_chunks=0) == oracle_result(W.REGEX_C1, data)


# --------------------------------------------------------------------------
# renumbered D-SFA ids and the hot-row global walk
# --------------------------------------------------------------------------
def run_table(t, rx, data, n_chunks=0):
    say(rx[:40], "n=%d" % data.size, "chunks=%d" % n_chunks, "info", t.info)
    return sfa.match(t, to_device(data), n_chunks=n_chunks).tolist()


@pytest.mark.parametrize("rx", [W.REGEX_C1, W.REGEX_C2, "(ab)*", W.rn_regex(7)])
def test_renumbered_ids_and_hot_rows_keep_results(rx):
    rng = np.random.default_rng(21)
    data = (W.c2_input(21, n=300_001) if rx in (W.REGEX_C2, "(ab)*")
            else W.c1_input(21, n=300_000) if rx == W.REGEX_C1
            else rng.choice(np.frombuffer(b"0123456789", np.uint8), size=300_000))
    want = oracle_result(rx, data)
    c = sfa.compile(rx)
    # LDS image path with renumbered ids
    t1 = sfa.load(c, renumber=1)
    assert run_table(t1, rx, data, 777) == want
    # global walk, all rows hot
    t2 = sfa.load(c, force_global=True)
    assert t2.info["hot_rows"] == c.info.n_sfa
    assert run_table(t2, rx, data, 777) == want
    # global walk, only a few rows hot (the rest read from global memory)
    t3 = sfa.load(c, force_global=True, lds_budget=16)
    assert 0 < t3.info["hot_rows"] < c.info.n_sfa
    assert run_table(t3, rx, data, 777) == want
    # no renumbering at all
    t4 = sfa.load(c, force_global=True, lds_budget=16, renumber=2)
    assert run_table(t4, rx, data, 777) == want


def test_c3_hot_rows_with_profile_sample():
    kws = W.c3_keywords(2)
    rx = W.c3_regex(kws)
    data = W.c3_input(7, 1 << 24, kws, rate=3e-6)
    want = oracle_result(rx, data)
    c = sfa.compile(rx)
    t = sfa.load(c, profile_sample=data[: 1 << 20])
    assert 0 < t.info["hot_rows"] < c.info.n_sfa
    assert run_table(t, rx, data) == want
    t2 = sfa.load(c)            # profile from uniformly random classes
    assert run_table(t2, rx, data, 4096) == want
    # a few staged rows: most steps of most pieces read the global table
    t3 = sfa.load(c, lds_budget=256)
    assert 0 < t3.info["hot_rows"] <= 4
    assert run_table(t3, rx, data, 4096) == want
    assert run_table(t3, rx, data) == want


# --------------------------------------------------------------------------
# grid composition: one level, two levels, top level read from global memory
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n_chunks", [1 << 16, (1 << 20) + 3, 1 << 22])
def test_many_blocks_two_level_grid_composition(n_chunks):
    # 2^20 chunks of the LDS walk are 4096 blocks: more block mappings than
    # one block's LDS holds, so runs of blocks are composed first
    data = W.c2_input(12, n=(1 << 22) + 1001)
    check(W.REGEX_C2, data, n_chunks=n_chunks)
    check(W.REGEX_C2, data, n_chunks=n_chunks, force_global=True)
    check(W.REGEX_C2, data, n_chunks=n_chunks, speculative=True)


def test_speculative_c3_many_chunks_global_top_level():
    # 65,536 speculative chunks of a ~130-state DFA: 16,384 block mappings in
    # runs of ~60, whose ~270 run mappings exceed the staging LDS
    kws = W.c3_keywords(0)
    rx = W.c3_regex(kws)
    data = W.c3_input(8, 1 << 23, kws, rate=4e-6)
    check(rx, data, n_chunks=65536, speculative=True)
    check(rx, data, n_chunks=65536)


def test_workspace_shared_by_one_and_two_level_plans():
    # calls with different grid plans share one cached workspace: the control
    # words must stay zero between them whatever the previous plan wrote
    data = W.c2_input(13, n=(1 << 22) + 77)
    want = oracle_result(W.REGEX_C2, data)
    x = to_device(data)
    for n_chunks, spec in [(65536, False), (65536, True), (1 << 20, False), (4096, True), (7, False),
                           (1 << 22, False), (65536, True), (0, False), (1 << 20, True)]:
        assert run(W.REGEX_C2, data, n_chunks=n_chunks, speculative=spec, x=x) == want, (n_chunks, spec)


# --------------------------------------------------------------------------
# composition through the product table vs through the mappings; every
# launch plan of the walk kernels
# --------------------------------------------------------------------------
PRODUCT_RX = [W.REGEX_C1, W.REGEX_C2, "(ab)*", W.rn_regex(3), ".*abc.*", "(a|b)*a(a|b){2}", ".*"]


def small_text(rx, seed, n):
    if rx == W.REGEX_C1:
        return W.c1_input(seed, n=n - n % 2)
    if rx == W.rn_regex(3):
        rng = np.random.default_rng(seed)
        return rng.choice(np.frombuffer(b"0123456789", np.uint8), size=n)
    return W.uniform_over(W.rng_for(seed, 3), np.frombuffer(b"abc", np.uint8), n)


@pytest.mark.parametrize("rx", PRODUCT_RX)
def test_product_and_mapping_composition_agree(rx):
    data = small_text(rx, 31, (1 << 20) + 333)
    want = oracle_result(rx, data)
    c = sfa.compile(rx)
    tp = sfa.load(c)
    tm = sfa.load(c, product=False)
    tg = sfa.load(c, force_global=True)
    assert tp.info["product_table"] == int(c.info.n_sfa <= 128)
    assert tm.info["product_table"] == 0
    assert tg.info["product_table"] == tp.info["product_table"]
    x = to_device(data)
    for n_chunks in (0, 1, 3, 777, 65536, 1 << 20, 1 << 22):
        for t in (tp, tm, tg):
            say(rx[:30], "chunks", n_chunks, "product", t.info["product_table"], "lds", t.info["table_in_lds"])
            assert sfa.match(t, x, n_chunks=n_chunks).tolist() == want, (n_chunks, t.info)


LDS_SHAPES = [(1, 64, 2, 256), (1, 128, 2, 256), (1, 128, 4, 256), (2, 64, 2, 256), (2, 64, 4, 256),
              (2, 128, 2, 256), (2, 128, 3, 256), (2, 128, 4, 256), (3, 128, 3, 256), (4, 64, 2, 256), (8, 32, 2, 256),
              (1, 64, 2, 512), (1, 128, 2, 512), (1, 128, 3, 512), (1, 128, 4, 512), (2, 64, 2, 512), (2, 64, 4, 512),
              (2, 128, 2, 512), (2, 128, 3, 512), (4, 32, 2, 512), (4, 64, 2, 512),
              (1, 32, 2, 1024), (1, 64, 2, 1024), (1, 128, 2, 1024), (2, 32, 2, 1024), (2, 64, 2, 1024)]


@pytest.mark.parametrize("product", [True, False])
@pytest.mark.parametrize("rx", [W.REGEX_C1, W.REGEX_C2])
def test_every_lds_launch_plan(rx, product):
    data = small_text(rx, 41, (2 << 20) + 4099)
    want = oracle_result(rx, data)
    t = sfa.load(sfa.compile(rx), product=product)
    assert t.info["strides"] == 2 | 4 | 16
    x = to_device(data)
    for stride in (1, 2, 4):
        for (k, g, d, tb) in LDS_SHAPES:
            for lpc in (1, 4):
                for n_chunks in (1000, 65536):
                    plan = dict(stride=stride, pieces=k, load_bytes=g, depth=d, block_threads=tb,
                                lanes_per_chunk=lpc)
                    got = sfa.match(t, x, n_chunks=n_chunks, plan=plan).tolist()
                    assert got == want, (plan, n_chunks)


GLOBAL_SHAPES = [(1, 64, 2, 256), (2, 64, 2, 256), (4, 32, 2, 256), (4, 64, 2, 256),
                 (1, 128, 2, 256), (2, 128, 2, 256), (4, 128, 2, 256),
                 (1, 64, 2, 512), (2, 64, 2, 512), (4, 32, 2, 512), (4, 64, 2, 512),
                 (1, 128, 2, 512), (2, 128, 2, 512), (2, 128, 3, 512),
                 (2, 128, 1, 512), (3, 128, 1, 512), (4, 128, 1, 512),
                 (1, 64, 2, 1024), (2, 64, 2, 1024), (1, 128, 2, 1024), (2, 128, 1, 1024)]


@pytest.mark.parametrize("product", [True, False])
def test_every_global_launch_plan(product):
    rx = W.REGEX_C2
    data = small_text(rx, 43, (2 << 20) + 17)
    want = oracle_result(rx, data)
    for lds_budget in (0, 256):          # all rows staged / only a few rows staged
        t = sfa.load(sfa.compile(rx), force_global=True, product=product, lds_budget=lds_budget)
        x = to_device(data)
        for k, g, d, tb in GLOBAL_SHAPES:
            for n_chunks in (0, 1000, 65536):
                plan = dict(pieces=k, load_bytes=g, depth=d, block_threads=tb)
                assert sfa.match(t, x, n_chunks=n_chunks, plan=plan).tolist() == want, (plan, n_chunks, t.info)


def test_vector_rewalks_of_cold_words():
    # a profile whose visits mostly miss the few staged rows switches the
    # global walk to vector re-walks of cold words (complete and partial
    # D-SFAs); both must still equal the oracle
    rx = W.rn_regex(40)
    sample = W.rn_input(9, 40, 1 << 20)
    words = W.rn_input(10, 40, (4 << 20) + 80 * 3)
    full = sfa.load(sfa.compile(rx, sfa_cap=100_000), profile_sample=sample, lds_budget=2048)
    lazy = sfa.load(sfa.compile(rx, sfa_cap=0).build_lazy(sample, start_every=64, walk_bytes=512, max_states=2000),
                    profile_sample=sample, lds_budget=256)
    wide = dict(pieces=2, load_bytes=128, depth=1, block_threads=1024)
    for t in (full, lazy):
        assert t.info["vector_redo"] == 1 and t.info["table_in_lds"] == 0
        for data in (words, words[: (1 << 20) + 77]):
            want = oracle_result(rx, data)
            for n_chunks in (0, 1000, 65536):
                assert run_table(t, rx, data, n_chunks) == want, (t.info["partial"], n_chunks)
            # the shape large inputs get by default (chunks of 1 KiB or more)
            x = to_device(data)
            for n_chunks in (500, 1000):
                assert sfa.match(t, x, n_chunks=n_chunks, plan=wide).tolist() == want, (t.info["partial"], n_chunks)


def test_dsfa_over_65536_states_uses_32_bit_ids():
    # r_128 has 4*128^2 + 2*128 = 65,792 D-SFA states: 32-bit walk-table
    # entries, read by the global-table walk with hot rows in LDS
    rx = W.rn_regex(128)
    c = sfa.compile(rx, sfa_cap=70_000)
    assert c.info.n_sfa == 65_792
    t = sfa.load(c)
    assert t.info["next_bytes"] == 4 and t.info["table_in_lds"] == 0 and t.info["hot_rows"] > 0
    words = W.rn_input(5, 128, (4 << 20) + 256 * 7)
    rng = np.random.default_rng(4)
    noise = rng.choice(np.frombuffer(b"0123456789", np.uint8), size=(1 << 20) + 3)
    for data in (words, noise, words[: (1 << 20) + 77]):
        want = oracle_result(rx, data)
        for n_chunks in (0, 1000, 65536):
            assert run_table(t, rx, data, n_chunks) == want, n_chunks


@pytest.mark.parametrize("n", [0, 15, 16, 4096 + 7, (1 << 20) + 13, 1 << 24])
def test_stream_read_reference_reads_every_byte(n):
    # the streaming-read reference folds every 32-bit word and tail byte of
    # its input into the XOR checksum; compared with numpy's XOR of the same
    rng = np.random.default_rng(n)
    data = rng.integers(0, 256, size=n, dtype=np.uint8)
    words = np.frombuffer(data[: n - n % 16].tobytes(), dtype=np.uint32)
    want = int(np.bitwise_xor.reduce(words)) if words.size else 0
    for b in data[n - n % 16:]:
        want ^= int(b)
    x = to_device(data)
    acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    sfa.stream_read(x, acc)
    assert (int(acc.item()) & 0xFFFFFFFF) == want
    if n:                           # a misaligned base is rejected by the host, not read
        with pytest.raises(sfa.SfaError):
            sfa.stream_read(to_device(data, 1), acc)
