"""Build step for the oracle's C library (test infrastructure only).

Compiles ``radic_oracle.c`` with gcc into ``liboracle.so`` next to this file.
Plain -O2, no fast-math, so IEEE semantics are kept.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "radic_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compile `src` (default: the oracle) into the shared library `out`."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def stale() -> bool:
    """True when the library is missing or older than its source."""
    return not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)


if __name__ == "__main__":
    print(build(verbose=True))
