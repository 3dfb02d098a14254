"""Compile the oracle's C core (test infrastructure only) with gcc.

The library is written next to this file as ``libtfhe_ref.so``.  It is
loaded only by the tests, by the package smoke check and by the benchmark's
CPU-baseline leg.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tfhe_ref.c")
LIB = os.path.join(HERE, "libtfhe_ref.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-fno-strict-aliasing",
           "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
