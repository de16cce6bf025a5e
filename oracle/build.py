"""Compiles the CPU oracle into ``oracle/liboracle.so`` (gcc, plain C11).

-ffp-contract=off keeps every multiply and add separately rounded, exactly as
the source spells them; fma() is used only where the source calls it.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "rbl_oracle.c")


def library_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def stale() -> bool:
    lib = library_path()
    return (not os.path.exists(lib)) or os.path.getmtime(lib) < os.path.getmtime(SOURCE)


def build(extra_flags=()) -> str:
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", *extra_flags, "-o", tmp, SOURCE, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
