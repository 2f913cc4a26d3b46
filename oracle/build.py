"""Compile the FP64 oracle (`askit_oracle.c`) into `liboracle.so` with gcc.

The oracle is test infrastructure: building it is part of building the
checker, not of the HIP library.  -ffp-contract=off keeps every product
unfused, so the canonical distance sums are reproducible bit for bit.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "askit_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


ASAN_OUT = os.path.join(HERE, "liboracle_asan.so")


def build_asan(force: bool = True) -> str:
    """The same source under AddressSanitizer and UndefinedBehaviorSanitizer
    (`liboracle_asan.so`): loaded instead of `liboracle.so` when
    ASKIT_ORACLE_ASAN=1, by a process that preloads the ASan runtime."""
    if not force and os.path.exists(ASAN_OUT) and os.path.getmtime(ASAN_OUT) >= os.path.getmtime(SRC):
        return ASAN_OUT
    tmp = ASAN_OUT + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, ASAN_OUT)
    return ASAN_OUT


if __name__ == "__main__":
    if "--asan" in sys.argv:
        print(build_asan(force="--lazy" not in sys.argv))
    else:
        print(build(force="--lazy" not in sys.argv))
