"""Compile the serial CPU oracle into oracle/liboracle.so with g++.

Test infrastructure: the product library never links or loads the result.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "odp_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build_native(directory: str) -> str:
    """A copy of the oracle compiled for the CPU it runs on (-O3 -march=native),
    for timing it as a CPU baseline; built where it will run, never shipped."""
    path = os.path.join(directory, "liboracle_native.so")
    cmd = ["g++", "-O3", "-march=native", "-std=c++17", "-shared", "-fPIC", "-o", path, SRC]
    subprocess.run(cmd, check=True)
    return path


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-O3", "-std=c++17", "-shared", "-fPIC", "-Wall", "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
