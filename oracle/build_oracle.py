"""Builds the CPU oracle shared library with g++ (test infrastructure only).

``build()`` compiles ``bitonic_oracle.cpp`` into ``liboracle.so`` next to
this file.  ``build_mutant(m, outdir)`` compiles the same source with a
planted mistake (``-DORACLE_MUTANT=m``) for the tests that show the oracle's
pins catch such mistakes.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bitonic_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

MUTANTS = {
    1: "no alternation of block directions (standard network)",
    2: "stride off by one (standard network)",
    3: "half-cleaner partner instead of the mirror (flip network)",
    4: "keys compared as unsigned",
    5: "last step of every phase dropped",
    6: "padding with zeros instead of INT32_MAX",
    7: "float32 negatives ordered by increasing magnitude",
    8: "pairs with equal keys ordered by value descending",
    9: "int64 keys compared on their low 32 bits only",
    10: "float64 negatives ordered by increasing magnitude",
}


def _compile(out: str, extra: list[str]) -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", out + ".tmp",
           SRC] + extra
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build() -> str:
    return _compile(LIB, [])


def build_mutant(mutant: int, outdir: str) -> str:
    return _compile(os.path.join(outdir, f"liboracle_mutant{mutant}.so"),
                    [f"-DORACLE_MUTANT={mutant}"])


if __name__ == "__main__":
    print(build())
