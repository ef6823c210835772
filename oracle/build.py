"""Build the oracle's C part (``seqscan.c``: Algorithm 2; ``cpu_sfa.c``:
Algorithm 5 on host threads) with gcc.  Test infrastructure."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "_seqscan.so")


def build(force: bool = True) -> str:
    srcs = [os.path.join(HERE, f) for f in ("seqscan.c", "cpu_sfa.c")]
    if force or not os.path.exists(SO) or os.path.getmtime(SO) < max(os.path.getmtime(s) for s in srcs):
        tmp = SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, *srcs])
        os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build())
