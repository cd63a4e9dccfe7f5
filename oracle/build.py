"""Compile the oracle's C code into ``oracle/libzfo.so`` (plain gcc, -O2).

Test infrastructure only (see ``oracle/__init__.py``)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libzfo.so")
SRC = [os.path.join(HERE, "zfo.c")]


def build(force=True):
    """Compile the oracle library; with force=False only when it is missing."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp] + SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
