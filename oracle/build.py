"""Compile the oracle's C part (test infrastructure; never linked by the library).

The same Jacobi source is built twice: ``_jacobi.so`` in extended precision
(the default oracle) and ``_jacobi64.so`` in double precision.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jacobi.c")
LIBS = {
    "extended": (os.path.join(HERE, "_jacobi.so"), []),
    "double": (os.path.join(HERE, "_jacobi64.so"), ["-DJACOBI_DOUBLE"]),
}
LIB = LIBS["extended"][0]


def build(force: bool = True, precision: str | None = None) -> str:
    """Build the shared library of ``precision`` (both when None); return the path of ``precision``'s."""
    for prec, (path, defs) in LIBS.items():
        if precision is not None and prec != precision:
            continue
        if not force and os.path.exists(path) and os.path.getmtime(path) >= os.path.getmtime(SRC):
            continue
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *defs, "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return LIBS[precision or "extended"][0]


if __name__ == "__main__":
    build(force="--lazy" not in sys.argv)
    for p, _ in LIBS.values():
        print(p)
