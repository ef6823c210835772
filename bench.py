"""Benchmark: single-stream SFA matching throughput on one MI355X.

A step is one sfa_match call (Algorithm 5: chunk walks from the identity,
ordered composition, apply to q0) over one device-resident input.  The
default workload is the regex (a|b)*a(a|b){4} over 256 MiB of uniform
{a, b} bytes split into 65,536 chunks.  Several copies of the input are
rotated so that consecutive steps do not hit in the 256 MB Infinity Cache.

Prints one JSON line (see the keys below).  The oracle (sequential DFA,
Algorithm 2, plain C on one host core) is timed beside it on a bounded
sample and also checks the GPU result.
"""
from __future__ import annotations

import argparse
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
    "c2": dict(desc="regex (a|b)*a(a|b){4}, 256 MiB uniform over {a,b}, 65536 chunks",
               n=1 << 28, n_chunks=65536),
    "c2_4g": dict(desc="regex (a|b)*a(a|b){4}, 4 GiB uniform over {a,b}, library-chosen chunks",
                  n=1 << 32, n_chunks=0),
    "c3": dict(desc="regex .*(w1|...|w20).* with 20 seeded 8-letter keywords, 4 GiB uniform over a-z and space, "
                    "keywords planted at rate 1e-6, library-chosen chunks",
               n=1 << 32, n_chunks=0),
}


def make_input(name: str, seed: int):
    import workloads as W
    if name.startswith("c2"):
        return W.REGEX_C2, W.c2_input(seed, WORKLOADS[name]["n"])
    if name == "c3":
        kws = W.c3_keywords(seed)
        return W.c3_regex(kws), W.c3_input(seed, WORKLOADS[name]["n"], kws, rate=1e-6)
    raise ValueError(name)


def cpu_baseline(rx, data, budget_s: float):
    """The oracle (Algorithm 2 in C, one core) over a bounded sample."""
    from oracle.automata import compile_regex
    from oracle import scan
    d = compile_regex(rx)
    tab = scan.table_u32(d)
    full_q = None
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
    return {
        "value": total_bytes / elapsed / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
        "sample": "%d full pass(es) of the same %d-byte input, %.1f s" % (reps, data.size, elapsed),
    }, [full_q, int(d.accept[full_q])]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copies", type=int, default=0, help="rotating input copies (0 = auto)")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--speculative-steps", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device-to-device copy of the workload size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1405_0562_amd as sfa

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
    rx, host = make_input(args.workload, args.seed)
    n = host.size
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    comp = sfa.compile(rx)
    table = sfa.load(comp)
    copies = args.copies or max(1, min(8, (1 << 30) // n))
    bufs = [torch.from_numpy(host).to(dev) for _ in range(copies)]
    out = torch.empty(2, dtype=torch.int32, device=dev)
    n_chunks = wl["n_chunks"]
    use_sfa = comp.info.n_sfa > 0
    fn = sfa.match if use_sfa else sfa.match_speculative
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        fn(table, bufs[i % copies], n_chunks=n_chunks, out=out)
    torch.cuda.synchronize()
    got = out.tolist()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        fn(table, bufs[i % copies], n_chunks=n_chunks, out=out)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    kern_avg_ms = float(np.mean(kern_ms))
    ms_per_step = wall * 1e3 / args.steps
    value = n / (ms_per_step * 1e-3) / 1e9
    achieved = n / (kern_avg_ms * 1e-3) / 1e9

    spec = None
    if use_sfa and args.speculative_steps > 0:
        sfa.match_speculative(table, bufs[0], n_chunks=n_chunks, out=out)
        torch.cuda.synchronize()
        s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_ev.record(stream)
        for i in range(args.speculative_steps):
            sfa.match_speculative(table, bufs[i % copies], n_chunks=n_chunks, out=out)
        e_ev.record(stream)
        torch.cuda.synchronize()
        spec_ms = s_ev.elapsed_time(e_ev) / args.speculative_steps
        spec = {"gbs": n / (spec_ms * 1e-3) / 1e9, "ms": spec_ms, "result": out.tolist()}

    cpu, want = (None, None)
    if not args.no_cpu:
        cpu, want = cpu_baseline(rx, host, args.cpu_budget)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n_bytes": n, "n_chunks": n_chunks,
                   "regex": rx if len(rx) < 80 else rx[:77] + "...", "seed": args.seed,
                   "input_copies_rotated": copies,
                   "n_dfa": comp.info.n_dfa, "n_sfa": comp.info.n_sfa, "n_classes": comp.info.n_classes,
                   "table_in_lds": table.info["table_in_lds"], "path": "sfa" if use_sfa else "speculative"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_sfa_walk" if use_sfa else "k_spec_walk", "kernel_avg_ms": kern_avg_ms,
                     "algorithmic_bytes_per_launch": n},
        "cpu_baseline": cpu,
        "result": got,
        "oracle_result": want,
        "parity": (got == want) if want is not None else None,
        "speculative": spec,
    }
    print(json.dumps(line), flush=True)
    if want is not None and got != want:
        sys.exit(1)


if __name__ == "__main__":
    main()
