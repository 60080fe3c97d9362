"""Compile the oracle's C sources (oracle/csrc/*.c) into a shared library, if any exist.

Test infrastructure only: building the checker is not using it.
"""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build():
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.c")))
    if not srcs:
        return None
    out = os.path.join(HERE, "liboracle.so")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", out] + srcs + ["-lm"], check=True)
    return out
