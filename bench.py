"""Benchmark: single-stream SFA matching throughput on one MI355X.

A step is one sfa_match call (Algorithm 5: chunk walks from the identity,
ordered composition, apply to q0) over one device-resident input.  The
default workload is the keyword regex .*(w1|...|w20).* (20 seeded 8-letter
keywords) over 4 GiB of text over a-z and space with keywords planted at
rate 1e-6; its D-SFA (about 18 K states) is walked from a global table with
its most visited rows in LDS.  Beside it, in the same run and each with its
own roofline, the regex (a|b)*a(a|b){4} (LDS-resident D-SFA) over 4 GiB and
over 256 MiB (65,536 chunks; several copies rotated so that consecutive
steps do not hit in the 256 MB Infinity Cache).

Prints one JSON line (see the keys below).  The oracle (sequential DFA,
Algorithm 2, plain C on one host core) is timed beside it on a bounded
sample and checks every GPU result over all the bytes.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "input GB/s matched vs HBM peak; batched docs/s and p99 latency vs plain path"

WORKLOADS = {
    # name: (regex builder, n bytes, n_chunks, generator)
    "c2": dict(desc="regex (a|b)*a(a|b){4}, 256 MiB uniform over {a,b}, 65536 chunks (LDS-resident table)",
               n=1 << 28, n_chunks=65536),
    "c2_4g": dict(desc="regex (a|b)*a(a|b){4}, 4 GiB uniform over {a,b}, library-chosen chunks (LDS-resident table)",
                  n=1 << 32, n_chunks=0),
    "c3": dict(desc="regex .*(w1|...|w20).* with 20 seeded 8-letter keywords, 4 GiB uniform over a-z and space, "
                    "keywords planted at rate 1e-6, library-chosen chunks",
               n=1 << 32, n_chunks=0),
}


def cached_input(name: str, seed: int, cache_dir: str | None):
    """make_input, stored as .npy files under cache_dir when given (repeated
    profiler passes over the same workload then skip the generation)."""
    import numpy as np
    if not cache_dir:
        return make_input(name, seed)
    os.makedirs(cache_dir, exist_ok=True)
    base = os.path.join(cache_dir, "%s_seed%d" % (name, seed))
    try:
        rx = open(base + ".regex", encoding="latin-1").read()
        data = np.load(base + ".npy", mmap_mode="r")
        prof = np.load(base + ".profile.npy") if os.path.exists(base + ".profile.npy") else None
        return rx, np.ascontiguousarray(data), prof
    except OSError:
        pass
    rx, data, prof = make_input(name, seed)
    np.save(base + ".npy", data)
    if prof is not None:
        np.save(base + ".profile.npy", prof)
    with open(base + ".regex", "w", encoding="latin-1") as fh:
        fh.write(rx)
    return rx, data, prof


def make_input(name: str, seed: int):
    """(regex, input bytes, profile sample or None).  The keyword workload's
    table ranks its hot rows by a walk over an independent 1 MiB sample of
    the same text distribution (another seed), not over the input."""
    import workloads as W
    if name.startswith("c2"):
        return W.REGEX_C2, W.c2_input(seed, WORKLOADS[name]["n"]), None
    if name == "c3":
        kws = W.c3_keywords(seed)
        return (W.c3_regex(kws), W.c3_input(seed, WORKLOADS[name]["n"], kws, rate=1e-6),
                W.c3_input(seed + 1000, 1 << 20, kws, rate=1e-6))
    raise ValueError(name)


def host_threads() -> int:
    """Host threads the all-cores baseline uses: the CPUs this process may
    run on, at most 16 (one GPU's share of the box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rx, data, budget_s: float):
    """The oracle beside the GPU: Algorithm 2 in C on one core over a
    bounded sample (its first full pass is also the parity check), and
    Algorithm 5 in C on all host threads (one chunk per thread, 256-column
    D-SFA table, sequential reduction), construction excluded."""
    from oracle.automata import compile_regex
    from oracle.sfa import byte_dsfa, OverCap
    from oracle import scan
    d = compile_regex(rx)
    tab = scan.table_u32(d)
    t0 = time.perf_counter()
    full_q = scan.scan(d, data, table=tab)          # one full pass: also the parity check
    t_full = time.perf_counter() - t0
    reps, total_bytes, elapsed = 1, data.size, t_full
    while elapsed < budget_s:
        t0 = time.perf_counter()
        scan.scan(d, data, table=tab)
        elapsed += time.perf_counter() - t0
        total_bytes += data.size
        reps += 1
    out = {
        "value": total_bytes / elapsed / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
        "sample": "%d full pass(es) of the same %d-byte input, %.1f s (Algorithm 2, sequential DFA, C, one core)"
                  % (reps, data.size, elapsed),
    }
    threads = host_threads()
    try:
        sd, cls = byte_dsfa(d, cap=1 << 20)
        st = scan.SfaTables(sd, cls)
        q5, _ = scan.sfa_parallel(st, data, threads)      # warm pass, also checked
        reps5, el5 = 0, 0.0
        while el5 < min(budget_s, 5.0) or reps5 < 1:
            t0 = time.perf_counter()
            q5, _ = scan.sfa_parallel(st, data, threads)
            el5 += time.perf_counter() - t0
            reps5 += 1
        out["algorithm5_all_cores"] = {
            "value": reps5 * data.size / el5 / 1e9, "unit": "GB/s", "cores": threads, "cpu": cpu_model(),
            "kind": "oracle", "result_equals_algorithm2": q5 == full_q,
            "sample": "%d full pass(es), %d chunks (one per thread), %d-state D-SFA with 256-column rows"
                      % (reps5, threads, sd.m)}
    except OverCap:
        out["algorithm5_all_cores"] = None
    return out, [full_q, int(d.accept[full_q])]


def cpu_baseline_sizes(rx, inputs, budget_s: float = 0.2):
    """The oracle (Algorithm 2 in C, one core) timed per input of the
    crossover study: seconds per pass and its result for each input."""
    from oracle.automata import compile_regex
    from oracle import scan
    d = compile_regex(rx)
    tab = scan.table_u32(d)
    out = []
    for data in inputs:
        q = scan.scan(d, data, table=tab)
        reps, elapsed = 0, 0.0
        while elapsed < budget_s or reps < 3:
            t0 = time.perf_counter()
            scan.scan(d, data, table=tab)
            elapsed += time.perf_counter() - t0
            reps += 1
        out.append((elapsed / reps, [q, int(d.accept[q])]))
    return out


def crossover_study(seed: int):
    """Small inputs: one sfa_match call end to end (launch to result on the
    host) with the input already in device memory, and with a copy from
    pinned host memory first, against one pass of the oracle's sequential
    DFA on one host core.  The regex is the overhead experiment's shape."""
    import numpy as np
    import torch
    import paper_1405_0562_amd as sfa
    import workloads as W
    rx = W.REGEX_C1
    sizes = [1 << k for k in range(10, 25, 2)]
    inputs = [W.c1_input(seed, n=(s // 10) * 10) for s in sizes]
    table = sfa.load(sfa.compile(rx))
    out = torch.empty(2, dtype=torch.int32, device="cuda")
    rows = []
    cpu = cpu_baseline_sizes(rx, inputs)
    for data, (cpu_s, want) in zip(inputs, cpu):
        pinned = torch.from_numpy(data).pin_memory()
        dev = pinned.cuda()
        for _ in range(3):
            sfa.match(table, dev, out=out).tolist()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            got = sfa.match(table, dev, out=out).tolist()
        resident_s = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            dev.copy_(pinned, non_blocking=True)
            got2 = sfa.match(table, dev, out=out).tolist()
        h2d_s = (time.perf_counter() - t0) / reps
        rows.append({"bytes": int(data.size), "gpu_resident_us": resident_s * 1e6, "gpu_with_h2d_us": h2d_s * 1e6,
                     "cpu_oracle_us": cpu_s * 1e6, "parity": got == want and got2 == want})
    cross = lambda key: next((r["bytes"] for r in rows if r[key] < r["cpu_oracle_us"]), None)
    return {"regex": rx, "rows": rows,
            "crossover_bytes_resident": cross("gpu_resident_us"),
            "crossover_bytes_with_h2d": cross("gpu_with_h2d_us")}


def rn_study(seed: int, size: int):
    """Scalability regexes r_n (Section 6.2) on ~1 GiB accepted texts, and
    r_n | a* on all-'a' text: host construction time, where the D-SFA is
    placed (LDS image, global table with hot rows, or over the state cap and
    matched by the speculative kernel), GPU throughput, and the oracle's
    sequential DFA on one core over the same bytes (also the parity check).
    Two tables over the default cap are also matched through an on-the-fly
    D-SFA (the on-the-fly remark of Section 5.1) built from the first MiB of
    their input: r500, and a 60-keyword dictionary on keyword text."""
    import numpy as np
    import torch
    import paper_1405_0562_amd as sfa
    import workloads as W
    big = 1_100_000   # state cap that admits the D-SFAs of r500 and r_a (about 10^6 states)
    kw60 = W.c3_keywords(seed, count=60)
    # on-the-fly rows: (runs start every, run bytes) of the sample walk; r500's
    # runs match the walk's pieces at this size (512 bytes), whose starts
    # fall on 125 phases of the 1000-byte period
    cases = [("r5", W.rn_regex(5), 5, None, None), ("r50", W.rn_regex(50), 50, None, None),
             ("r500, default cap", W.rn_regex(500), 500, None, None),
             ("r500, default cap, on the fly", W.rn_regex(500), 500, None, (512, 512)),
             ("r500", W.rn_regex(500), 500, big, None),
             ("r_a", W.ra_regex(500), None, big, None),
             ("60 keywords, default cap", W.c3_regex(kw60), -1, None, None),
             ("60 keywords, default cap, on the fly", W.c3_regex(kw60), -1, None, (256, 4096))]
    rows = []
    out = torch.empty(2, dtype=torch.int32, device="cuda")
    inputs = {}
    for name, rx, n, cap, lazy in cases:
        print("[rn study] %s: building input and automata" % name, file=sys.stderr, flush=True)
        if n not in inputs:
            inputs.clear()
            inputs[n] = (W.rn_input(seed, n, size) if n and n > 0 else
                         W.c3_input(seed, size, kw60, rate=1e-6) if n == -1 else np.full(size, ord("a"), dtype=np.uint8))
        data = inputs[n]
        t0 = time.perf_counter()
        if lazy:
            comp = sfa.compile(rx, sfa_cap=0).build_lazy(data[:1 << 20], start_every=lazy[0], walk_bytes=lazy[1])
        else:
            comp = sfa.compile(rx) if cap is None else sfa.compile(rx, sfa_cap=cap)
        compile_s = time.perf_counter() - t0
        # hot rows (global-table walk) ranked by a walk over the first MiB
        table = sfa.load(comp, profile_sample=data[:1 << 20])
        x = torch.from_numpy(data).cuda()
        use_sfa = comp.info.n_sfa > 0
        fn = sfa.match if use_sfa else sfa.match_speculative
        fn(table, x, out=out)
        torch.cuda.synchronize()
        reps = 3
        s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_ev.record()
        for _ in range(reps):
            fn(table, x, out=out)
        e_ev.record()
        torch.cuda.synchronize()
        ms = s_ev.elapsed_time(e_ev) / reps
        got = out.tolist()
        del x
        print("[rn study] %s: GPU %.3f ms; timing the oracle" % (name, ms), file=sys.stderr, flush=True)
        (cpu_s, want), = cpu_baseline_sizes(rx, [data], budget_s=0.0)
        info = table.info
        comp_info = (comp.info.n_dfa, comp.info.n_sfa)
        vec = ", vector re-walks of cold words" if info["vector_redo"] else ""
        placement = ("speculative (D-SFA over the state cap)" if not use_sfa else
                     "on the fly from the first MiB (runs of %d bytes every %d), global table, %d hot rows in LDS%s"
                     % (lazy[1], lazy[0], info["hot_rows"], vec) if lazy else
                     "LDS image, strides %s" % [s for s, bit in ((1, 2), (2, 4), (4, 16)) if info["strides"] & bit]
                     if info["table_in_lds"] else "global table, %d hot rows in LDS%s" % (info["hot_rows"], vec))
        del table, comp
        rows.append({"regex": name, "n_dfa": comp_info[0], "n_sfa": comp_info[1],
                     "compile_s": compile_s, "placement": placement, "product_table": info["product_table"],
                     "bytes": int(data.size), "gpu_gbs": data.size / (ms * 1e-3) / 1e9, "gpu_ms": ms,
                     "cpu_oracle_gbs": data.size / cpu_s / 1e9, "result": got, "oracle_result": want,
                     "parity": got == want})
    return {"rows": rows}


def batch_study(seed: int, n_docs: int, piece: int, units: int, reps: int):
    """The batch kernel alone on the batching workload with fixed options
    (for profiler passes): plan, upload, ``reps`` launches, parity of the
    last launch against the oracle on a sample of the documents."""
    import numpy as np
    import torch
    import paper_1405_0562_amd as sfa
    import workloads as W
    from oracle.automata import compile_regex
    from oracle import scan

    regexes = W.c4_regexes(seed)
    tables = [sfa.load(sfa.compile(rx)) for rx in regexes]
    data, off = W.c4_docs(seed, n_docs)
    x = torch.from_numpy(data).cuda()
    nt = len(tables)
    jobs = np.array([(d, t) for d in range(n_docs) for t in range(nt)], dtype=np.uint32)
    b = sfa.Batch(tables, off, jobs, sfa.BatchOptions(piece, units))
    b.run(x)
    torch.cuda.synchronize()
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record()
    for _ in range(reps):
        b.run(x)
    e_ev.record()
    torch.cuda.synchronize()
    ms = s_ev.elapsed_time(e_ev) / reps
    got = b.out.cpu().numpy()
    dfas = [compile_regex(rx) for rx in regexes]
    tabs = [scan.table_u32(d) for d in dfas]
    ok = True
    for d in range(0, n_docs, max(1, n_docs // 500)):
        doc = data[off[d]:off[d + 1]]
        for t in range(nt):
            q = scan.scan(dfas[t], doc, table=tabs[t])
            ok = ok and got[d * nt + t].tolist() == [q, int(dfas[t].accept[q])]
    return {"workload": "%d docs x %d regexes, %d bytes" % (n_docs, nt, int(off[-1])),
            "options": {"piece_bytes": piece, "units_per_lane": units, "tables_in_lds": b.info["tables_in_lds"]},
            "n_units": b.info["n_units"], "launches": reps + 1, "batch_ms": ms,
            "docs_per_s": n_docs / (ms * 1e-3), "parity_sampled": ok}


def cpu_baseline_nfa_sets(rx, inputs):
    """The oracle's NFA run (position automaton, from I) over each input:
    (final state set as a bit mask, accept) -- the N-SFA result's definition."""
    from oracle import nsfa as onsfa
    a = onsfa.glushkov(rx)
    out = []
    for data in inputs:
        s = onsfa.nfa_run(a, bytes(data))
        out.append((s, bool(s & a.final)))
    return out


def nsfa_study(seed: int, size: int):
    """D-SFA (minimal DFA) against N-SFA (position automaton) matching of the
    same regex on the same bytes: state counts, placement and throughput.
    Accept bits are checked against the oracle's sequential DFA over all the
    bytes, and the N-SFA's final NFA state set against the oracle's NFA run
    on a 1 MiB prefix."""
    import numpy as np
    import torch
    import paper_1405_0562_amd as sfa
    import workloads as W
    kw = W.c4_regexes(seed)[0]
    text = W.uniform_over(W.rng_for(seed, 3), W.ALPHABET_C4, size)
    cases = [(W.REGEX_C2, W.c2_input(seed, size)), (kw, text), (W.REGEX_C1, W.c1_input(seed, size - size % 10))]
    rows = []
    out = torch.empty(2, dtype=torch.int32, device="cuda")
    for rx, data in cases:
        print("[nsfa study] %s" % rx[:40], file=sys.stderr, flush=True)
        x = torch.from_numpy(data).cuda()
        prefix = torch.from_numpy(data[: 1 << 20].copy()).cuda()
        (cpu_s, want), = cpu_baseline_sizes(rx, [data], budget_s=0.0)
        (want_set, want_acc), = cpu_baseline_nfa_sets(rx, [data[: 1 << 20]])
        row = {"regex": rx if len(rx) < 60 else rx[:57] + "...", "bytes": int(data.size)}
        for kind in ("dsfa", "nsfa"):
            comp = sfa.compile_nsfa(rx) if kind == "nsfa" else sfa.compile(rx)
            table = sfa.load(comp)
            sfa.match(table, x, out=out)
            torch.cuda.synchronize()
            s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s_ev.record()
            for _ in range(10):
                sfa.match(table, x, out=out)
            e_ev.record()
            torch.cuda.synchronize()
            ms = s_ev.elapsed_time(e_ev) / 10
            q, acc = out.tolist()
            entry = {"dfa_states": comp.info.n_dfa, "sfa_states": comp.info.n_sfa,
                     "product_table": table.info["product_table"], "table_in_lds": table.info["table_in_lds"],
                     "gbs": data.size / (ms * 1e-3) / 1e9, "accept": acc, "accept_parity": acc == want[1]}
            if kind == "nsfa":
                qp, accp = sfa.match(table, prefix).tolist()
                entry["prefix_set_parity"] = (comp.nsfa_set(qp), bool(accp)) == (want_set, want_acc)
                entry["nfa_states"] = comp.nsfa_sets()[2]
            row[kind] = entry
            del table, comp
        rows.append(row)
    return {"rows": rows}


def kernel_source_hash() -> str:
    """Hash of the HIP sources and headers the match kernels are built from."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_1405_0562_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed PMC record, or None if the
    record is missing or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or not kernel.startswith(rec.get("kernel", "?")):
        return None
    return rec.get("traffic_bytes")


def batching_leg(seed: int, n_docs: int, plain_docs: int):
    """Batched form on the batching workload vs the plain per-job path."""
    import numpy as np
    import torch
    import paper_1405_0562_amd as sfa
    import workloads as W
    from oracle.automata import compile_regex
    from oracle import scan

    regexes = W.c4_regexes(seed)
    tables = [sfa.load(sfa.compile(rx)) for rx in regexes]
    data, off = W.c4_docs(seed, n_docs)
    x = torch.from_numpy(data).cuda()
    nt = len(tables)
    jobs = np.array([(d, t) for d in range(n_docs) for t in range(nt)], dtype=np.uint32)
    tuner = sfa.Autotuner(cache_path=os.path.join("/tmp", "sfa_autotune_bench.json"), reps=2)
    opt, entry = tuner.tune(tables, x, off, jobs)
    b = sfa.Batch(tables, off, jobs, opt)
    g = sfa.GraphBatch(b, x)
    g.replay()
    torch.cuda.synchronize()
    reps = 5
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record()
    for _ in range(reps):
        g.replay()
    e_ev.record()
    torch.cuda.synchronize()
    batch_ms = s_ev.elapsed_time(e_ev) / reps
    got = b.out.cpu().numpy()
    # parity: every job against the oracle (Algorithm 2 in C per document)
    dfas = [compile_regex(rx) for rx in regexes]
    tabs = [scan.table_u32(d) for d in dfas]
    want = np.empty((len(jobs), 2), dtype=np.int64)
    for d in range(n_docs):
        doc = data[off[d]:off[d + 1]]
        for t in range(nt):
            q = scan.scan(dfas[t], doc, table=tabs[t])
            want[d * nt + t] = (q, int(dfas[t].accept[q]))
    ok = bool(np.array_equal(got.astype(np.int64), want))
    # plain path: one sfa_match per job, in job order, on one stream
    outs = torch.empty((plain_docs * nt, 2), dtype=torch.int32, device="cuda")
    views = [x[off[d]:off[d + 1]] for d in range(plain_docs)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in range(plain_docs):
        for t in range(nt):
            sfa.match(tables[t], views[d], out=outs[d * nt + t])
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    ok = ok and np.array_equal(outs.cpu().numpy(), got[:plain_docs * nt])
    total = int(off[-1])
    return {
        "workload": "%d docs (lognormal, median 4 KiB, sigma 2, max %d B) x %d regexes, %d jobs, %.1f MB"
                    % (n_docs, int(np.diff(off).max()), nt, len(jobs), total / 1e6),
        "batch_ms": batch_ms, "docs_per_s": n_docs / (batch_ms * 1e-3), "jobs_per_s": len(jobs) / (batch_ms * 1e-3),
        "matched_gbs": total * nt / (batch_ms * 1e-3) / 1e9, "unique_input_gbs": total / (batch_ms * 1e-3) / 1e9,
        "plain_docs_per_s": plain_docs / plain_s, "plain_jobs_per_s": plain_docs * nt / plain_s,
        "plain_sample_docs": plain_docs, "speedup_docs_per_s": (n_docs / (batch_ms * 1e-3)) / (plain_docs / plain_s),
        "options": {"piece_bytes": opt.piece_bytes, "units_per_lane": opt.units_per_lane},
        "graph_replayed": True, "parity": ok, "parity_jobs": len(jobs),
    }


def serving_leg(seed: int, n_req: int, loads=(0.5, 0.8, 2.0, 4.0), big_bytes: int = 8 << 20):
    """Continuous-batching server vs the plain FIFO path under the same
    Poisson arrivals, at several multiples of the plain path's saturation rate."""
    import numpy as np
    import paper_1405_0562_amd as sfa
    import workloads as W
    from paper_1405_0562_amd.serve import GpuBackend, PlainBackend, Server, run_open_loop, Request

    regexes = W.c5_regexes(seed)
    tables = [sfa.load(sfa.compile(rx)) for rx in regexes]
    plain = PlainBackend(tables)
    # plain saturation rate R, closed loop
    probe = W.c5_requests(seed + 100, n_req=300, qps=1.0)
    for r in probe[:20]:
        plain.run_one(Request(0, r.table, r.data, 0.0))
    t0 = time.perf_counter()
    for r in probe:
        plain.run_one(Request(0, r.table, r.data, 0.0))
    R = len(probe) / (time.perf_counter() - t0)
    backend = GpuBackend(tables, pool_bytes=1 << 30, n_streams=3)
    points = []
    for mult in loads:
        qps = mult * R
        reqs = W.c5_requests(seed, n_req=n_req, qps=qps)
        arrivals = [(r.arrival_s, r.table, r.data) for r in reqs]
        srv = Server(backend, pool_bytes=1 << 30, max_inflight=3, big_bytes=big_bytes)
        # no collector pauses inside either timed loop
        gc.collect()
        gc.disable()
        run_open_loop(srv, arrivals)
        st = srv.latency_stats()
        served = {r.rid: r.result for r in srv.finished}
        # plain FIFO under the same arrivals: one request at a time, in order
        t0 = time.perf_counter()
        lat, equal = [], True
        for i, (at, tb, data) in enumerate(arrivals):
            now = time.perf_counter() - t0
            if now < at:
                time.sleep(at - now)
            res = plain.run_one(Request(i, tb, data, at))
            lat.append(time.perf_counter() - t0 - at)
            equal = equal and served.get(i) == res
        span = time.perf_counter() - t0
        gc.enable()
        lat = np.array(lat)
        total = sum(int(a[2].size) for a in arrivals)
        points.append({"load_x_plain_saturation": mult, "qps": qps,
                       "served": {k: st[k] for k in ("p50_ms", "p99_ms", "gbs", "launches")},
                       "plain_fifo": {"p50_ms": float(np.percentile(lat, 50) * 1e3),
                                      "p99_ms": float(np.percentile(lat, 99) * 1e3),
                                      "gbs": total / max(1e-9, span) / 1e9},
                       "results_equal_plain": equal})
    return {"workload": "%d requests per load point, Pareto(1.2, 1 KiB) lengths up to 64 MiB, 16 tables, "
                        "Poisson arrivals; plain saturation %.0f req/s" % (n_req, R),
            "plain_saturation_qps": R, "points": points}


def measure(name: str, seed: int, steps: int, warmup: int, copies_arg: int, spec_steps: int,
            cpu_budget: float, no_cpu: bool, cache_dir: str | None = None) -> dict:
    """One single-stream workload: timed sfa_match launches, the
    streaming-read reference, the speculative kernel, and the oracle's
    result over all the bytes (plus its timing when cpu_budget > 0)."""
    import torch
    import paper_1405_0562_amd as sfa

    wl = WORKLOADS[name]
    rx, host, prof = cached_input(name, seed, cache_dir)
    n = host.size
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    comp = sfa.compile(rx)
    table = sfa.load(comp, profile_sample=prof)
    copies = copies_arg or max(1, min(8, (1 << 30) // n))
    bufs = [torch.from_numpy(host).to(dev) for _ in range(copies)]
    out = torch.empty(2, dtype=torch.int32, device=dev)
    n_chunks = wl["n_chunks"]
    use_sfa = comp.info.n_sfa > 0
    fn = sfa.match if use_sfa else sfa.match_speculative
    stream = torch.cuda.current_stream()

    for i in range(warmup):
        fn(table, bufs[i % copies], n_chunks=n_chunks, out=out)
    torch.cuda.synchronize()
    got = out.tolist()

    # HIP events on the launch stream bracket the timed region: their
    # difference over K back-to-back launches is the kernel's average launch
    # duration (the host stays ahead, so no idle gaps enter it)
    start_ev, end_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start_ev.record(stream)
    for i in range(steps):
        fn(table, bufs[i % copies], n_chunks=n_chunks, out=out)
    end_ev.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_avg_ms = start_ev.elapsed_time(end_ev) / steps
    ms_per_step = wall * 1e3 / steps
    achieved = n / (kern_avg_ms * 1e-3) / 1e9
    got_timed = out.tolist()

    # reference: the library's streaming-read kernel over the same buffers in
    # the same run (every byte read once, wave-coalesced 16-byte loads, no
    # other work), a second denominator beside the 8 TB/s peak
    ref = None
    if n:
        acc = torch.zeros(1, dtype=torch.int32, device=dev)
        for b in bufs[:2]:
            sfa.stream_read(b, acc)
        torch.cuda.synchronize()
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(4, min(steps, 50))
        r0.record(stream)
        for i in range(reps):
            sfa.stream_read(bufs[i % copies], acc)
        r1.record(stream)
        torch.cuda.synchronize()
        ref_ms = r0.elapsed_time(r1) / reps
        ref = {"kind": "k_stream_read (sfa_stream_read) over the same input buffers",
               "gbs": n / (ref_ms * 1e-3) / 1e9, "ms": ref_ms}

    spec = None
    if use_sfa and spec_steps > 0:
        sfa.match_speculative(table, bufs[0], n_chunks=n_chunks, out=out)
        torch.cuda.synchronize()
        s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_ev.record(stream)
        for i in range(spec_steps):
            sfa.match_speculative(table, bufs[i % copies], n_chunks=n_chunks, out=out)
        e_ev.record(stream)
        torch.cuda.synchronize()
        spec_ms = s_ev.elapsed_time(e_ev) / spec_steps
        spec = {"gbs": n / (spec_ms * 1e-3) / 1e9, "ms": spec_ms, "result": out.tolist()}
    del bufs
    torch.cuda.empty_cache()

    cpu, want = (None, None)
    if not no_cpu:
        cpu, want = cpu_baseline(rx, host, cpu_budget)
    del host
    kname = "k_sfa_lds" if use_sfa and table.info["table_in_lds"] else ("k_sfa_global" if use_sfa else "k_spec_walk")
    traffic = recorded_traffic(name, kname)   # HBM bytes per launch (scaled PMC), or None
    parity = None if want is None else (got == want and got_timed == want
                                        and (spec is None or spec["result"] == want))
    return {
        "name": name, "n": n, "rx": rx, "copies": copies, "n_chunks": n_chunks,
        "ms_per_step": ms_per_step, "value": n / (ms_per_step * 1e-3) / 1e9,
        "config": {"workload": wl["desc"], "n_bytes": n, "n_chunks": n_chunks,
                   "regex": rx if len(rx) < 80 else rx[:77] + "...", "seed": seed,
                   "input_copies_rotated": copies,
                   "n_dfa": comp.info.n_dfa, "n_sfa": comp.info.n_sfa, "n_classes": comp.info.n_classes,
                   "table_in_lds": table.info["table_in_lds"], "hot_rows": table.info["hot_rows"],
                   "hot_rows_ranked_by": ("walk over an independent 1 MiB sample" if prof is not None
                                          else "walk over uniformly random classes"),
                   "path": "sfa" if use_sfa else "speculative"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_over_algorithmic": (traffic / n) if traffic else None,
                     "traffic_gbs": (traffic / (kern_avg_ms * 1e-3) / 1e9) if traffic else None,
                     "kernel": kname, "kernel_avg_ms": kern_avg_ms,
                     "algorithmic_bytes_per_launch": n,
                     "stream_read_reference": ref,
                     "frac_of_stream_read": (achieved / ref["gbs"]) if ref else None},
        "cpu_baseline": cpu,
        "result": got,
        "oracle_result": want,
        "parity": parity,
        "speculative": spec,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copies", type=int, default=0, help="rotating input copies (0 = auto)")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--speculative-steps", type=int, default=3)
    ap.add_argument("--input-cache", default=None,
                    help="directory in which generated inputs are stored and reused (profiler passes)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other single-stream workloads reported beside the headline")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-docs", type=int, default=10000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=3000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device-to-device copy of the workload size (counter calibration)")
    ap.add_argument("--study", choices=["crossover", "rn", "nsfa", "batch"], default=None,
                    help="run a study instead of the benchmark and print its JSON")
    ap.add_argument("--batch-piece", type=int, default=2048, help="--study batch: piece bytes")
    ap.add_argument("--batch-units", type=int, default=2, help="--study batch: pieces per lane")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    if args.study == "crossover":
        print(json.dumps({"study": "small-input crossover", **crossover_study(args.seed)}), flush=True)
        return
    if args.study == "nsfa":
        print(json.dumps({"study": "D-SFA and N-SFA", **nsfa_study(args.seed, 1 << 28)}), flush=True)
        return
    if args.study == "batch":
        print(json.dumps({"study": "batch kernel", **batch_study(args.seed, args.batch_docs, args.batch_piece,
                                                                 args.batch_units, args.steps)}), flush=True)
        return
    if args.study == "rn":
        print(json.dumps({"study": "r_n scalability and placement", **rn_study(args.seed, 1 << 30)}), flush=True)
        return
    wl = WORKLOADS[args.workload]
    if args.calibrate_copy:
        dev = torch.device("cuda", 0)
        src = torch.empty(wl["n"], dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": wl["n"], "launches": args.steps}))
        return

    def progress(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    progress("workload %s" % args.workload)
    head = measure(args.workload, args.seed, args.steps, args.warmup, args.copies, args.speculative_steps,
                   args.cpu_budget, args.no_cpu, args.input_cache)
    extra = {}
    if not args.no_extra:
        for name in ("c2_4g", "c2"):
            if name == args.workload:
                continue
            progress("workload %s" % name)
            m = measure(name, args.seed, args.steps, args.warmup, 0, args.speculative_steps, 0.0, args.no_cpu,
                        args.input_cache)
            extra[name] = {k: m[k] for k in ("value", "ms_per_step", "config", "roofline", "result",
                                             "oracle_result", "parity", "speculative")}
    progress("batching")
    batching = None if args.no_batch else batching_leg(args.seed, args.batch_docs, args.batch_docs)
    progress("serving")
    serving = None if args.no_serve else serving_leg(args.seed, args.serve_requests)

    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
        "result": head["result"],
        "oracle_result": head["oracle_result"],
        "parity": head["parity"],
        "speculative": head["speculative"],
        "single_stream_beside": extra,
        "batching": batching,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)
    bad = [m for m in [head] + list(extra.values()) if m["parity"] is False]
    if bad or (batching and not batching["parity"]):
        sys.exit(1)


if __name__ == "__main__":
    main()
