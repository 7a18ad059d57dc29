"""Compile the oracle's C source into oracle/libks_oracle.so (gcc, FP64).

Generic x86-64 code (no -march=native): the library built here also runs on the
benchmark host, whose CPU model may differ.  build(native=True, out=...) makes
a copy tuned for the machine it is built on (-march=native), which the
benchmark's CPU baseline compiles on its own host.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ks_oracle.c")
LIB = os.path.join(HERE, "libks_oracle.so")


def build(force: bool = True, src: str = SRC, out: str = LIB, native: bool = False) -> str:
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           *(["-march=native"] if native else []), "-I", HERE, src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
