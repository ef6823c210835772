"""Build the oracle's C part (``seqscan.c``) with gcc.  Test infrastructure."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "_seqscan.so")


def build(force: bool = True) -> str:
    src = os.path.join(HERE, "seqscan.c")
    if force or not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(src):
        tmp = SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build())
